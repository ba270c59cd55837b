// MFMA operand-tile layout of the per-sub-circuit inverses (batched sweep).
//
// An n x n inverse is zero-padded to np = roundup(n, 32) and cut into A-operand
// tiles of 16 rows: BF16 tiles are 16 x 32 (v_mfma_f32_16x16x32_bf16), FP64
// tiles are 16 x 8 (two v_mfma_f64_16x16x4f64 steps).  Tile (mt, kt) is stored
// at ((mt * (np / K) + kt) * 64 + lane) * E + j, lane-major, E = 16 bytes of
// elements per lane, so one 16-byte load per lane fetches a whole operand:
//   BF16: lane l holds A[16 mt + l%16][32 kt + 8 (l/16) + j], j < 8
//   FP64: lane l holds A[16 mt + l%16][8 kt + l/16] (j = 0) and
//         A[16 mt + l%16][8 kt + 4 + l/16] (j = 1)
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace vtm {

__host__ __device__ inline int tile_pad(int n) { return (n + 31) & ~31; }

template <typename T>
struct MfmaTypes;
template <>
struct MfmaTypes<__bf16> {
    using TV = float;           // vectors and waves of the BF16 path
    using TB = __bf16;          // its right-hand side (the staged operand is BF16)
    static constexpr int K = 32;
    static constexpr int E = 8;
};
template <>
struct MfmaTypes<double> {
    using TV = double;
    using TB = double;
    static constexpr int K = 8;
    static constexpr int E = 2;
};

// LDS bytes for the staged right-hand-side block (np rows, rc columns)
template <typename T>
__host__ __device__ inline size_t tile_lds_bytes(int np, int rc) {
    if constexpr (sizeof(T) == 2)
        return size_t(rc) * (np + 8) * sizeof(T);   // [n][k], row stride np + 8
    else
        return size_t(np) * rc * sizeof(T);         // [k][n]
}

// Batched port-to-port sweep: the BF16 path also stages h (FP32, row stride rc + 16,
// so that the epilogue's four 16-lane row groups fall in disjoint LDS banks) when
// the operator leaves room for it; the FP64 path stages the waves unpadded.

// row stride of the staged incident waves of the batched port-to-port sweep
template <typename T>
__host__ __device__ inline int pp_stage_stride(int qp, int rc) {
    if constexpr (sizeof(T) == 2)
        return qp + 8;                         // [n][k]
    else
        return rc;                             // [k][n]
}

// LDS bytes of the batched port-to-port sweep: staged waves, then (BF16, when
// with_h) h
template <typename T>
__host__ __device__ inline size_t pp_lds_bytes(int qp, int rc, bool with_h = true) {
    if constexpr (sizeof(T) == 2)
        return size_t(rc) * (qp + 8) * sizeof(T) +
               (with_h ? size_t(qp) * (rc + 16) * sizeof(float) : 0);
    else
        return size_t(qp) * rc * sizeof(T);
}

// (r, c) of the d-th stored element of a padded block
template <typename T>
__host__ __device__ inline void tile_rc(int np, int64_t d, int& r, int& c) {
    constexpr int K = MfmaTypes<T>::K, E = MfmaTypes<T>::E;
    const int j = int(d % E);
    const int lane = int((d / E) % 64);
    const int64_t tile = d / (64 * E);
    const int kt_n = np / K;
    const int mt = int(tile / kt_n), kt = int(tile % kt_n);
    const int m = lane % 16, q = lane / 16;
    r = mt * 16 + m;
    if constexpr (sizeof(T) == 2)
        c = kt * 32 + 8 * q + j;
    else
        c = kt * 8 + 4 * j + q;
}

}  // namespace vtm
