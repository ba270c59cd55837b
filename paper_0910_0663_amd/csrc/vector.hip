// Vector utilities: renumbering gathers/scatters, fills, precision casts,
// the refinement update, wave import/export and the branch gradient.
#include "kernels.hpp"

namespace vtm {

namespace {

constexpr int kBlock = 256;

__global__ void k_gather(int n, int nrhs, const int32_t* __restrict__ perm, const double* __restrict__ src,
                         double* __restrict__ dst) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(n) * nrhs) return;
    const int64_t i = t / nrhs;
    const int r = int(t - i * nrhs);
    dst[t] = src[int64_t(r) * n + perm[i]];
}

__global__ void k_scatter(int n, int nrhs, const int32_t* __restrict__ iperm, const double* __restrict__ src,
                          double* __restrict__ dst) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(n) * nrhs) return;
    const int r = int(t / n);
    const int64_t j = t - int64_t(r) * n;
    dst[t] = src[int64_t(iperm[j]) * nrhs + r];
}

// The same two renumberings for many right-hand sides, as transposes through an
// LDS tile of 64 rows x 64 right-hand sides: each side of the tile is read or
// written along its contiguous direction (the caller's [nrhs][n] rows, the
// internal [n][nrhs] rows), where the one-element kernels above touch a
// different cache line per lane on one side.
constexpr int kTile = 64;

__global__ void __launch_bounds__(kBlock)
    k_gather_tiled(int n, int nrhs, const int32_t* __restrict__ perm, const double* __restrict__ src,
                   double* __restrict__ dst) {
    __shared__ double tile[kTile][kTile + 1];
    const int i0 = blockIdx.x * kTile, r0 = blockIdx.y * kTile;
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    const int i = i0 + lx;
    const int pi = i < n ? perm[i] : 0;
#pragma unroll
    for (int k = 0; k < kTile / (kBlock / 64); ++k) {
        const int rr = ly + k * (kBlock / 64);
        const int r = r0 + rr;
        tile[rr][lx] = (i < n && r < nrhs) ? src[int64_t(r) * n + pi] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTile / (kBlock / 64); ++k) {
        const int ii = ly + k * (kBlock / 64);
        const int i2 = i0 + ii, r = r0 + lx;
        if (i2 < n && r < nrhs) dst[int64_t(i2) * nrhs + r] = tile[lx][ii];
    }
}

__global__ void __launch_bounds__(kBlock)
    k_scatter_tiled(int n, int nrhs, const int32_t* __restrict__ iperm, const double* __restrict__ src,
                    double* __restrict__ dst) {
    __shared__ double tile[kTile][kTile + 1];
    const int j0 = blockIdx.x * kTile, r0 = blockIdx.y * kTile;
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kTile / (kBlock / 64); ++k) {
        const int jj = ly + k * (kBlock / 64);
        const int j = j0 + jj, r = r0 + lx;
        tile[jj][lx] = (j < n && r < nrhs) ? src[int64_t(iperm[j]) * nrhs + r] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTile / (kBlock / 64); ++k) {
        const int rr = ly + k * (kBlock / 64);
        const int r = r0 + rr, j = j0 + lx;
        if (j < n && r < nrhs) dst[int64_t(r) * n + j] = tile[lx][rr];
    }
}

// Vertex tearing: plan row r takes w[r] times its original node src[r]'s entry
// (an interfacial node's source is split between its twins); the input is a
// caller's [nrhs][n_in] vector or an [n_in][nrhs] one.
__global__ void k_expand(int rows, int nrhs, int n_in, const int32_t* __restrict__ src,
                         const double* __restrict__ w, const double* __restrict__ in, int in_rhs_major,
                         double* __restrict__ out) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(rows) * nrhs) return;
    const int64_t r = t / nrhs;
    const int j = int(t - r * nrhs);
    const int64_t s = src[r];
    out[t] = w[r] * (in_rhs_major ? in[int64_t(j) * n_in + s] : in[s * nrhs + j]);
}

// The original nodes' values from the plan rows: the row itself, or the mean of
// an interfacial node's two twins (r1 >= 0); output [nrhs][n] or [n][nrhs].
template <typename TX>
__global__ void k_restrict(int n, int nrhs, const int32_t* __restrict__ r0, const int32_t* __restrict__ r1,
                           const TX* __restrict__ x, double* __restrict__ out, int out_rhs_major) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(n) * nrhs) return;
    int64_t i;
    int j;
    if (out_rhs_major) {
        j = int(t / n);
        i = t - int64_t(j) * n;
    } else {
        i = t / nrhs;
        j = int(t - i * nrhs);
    }
    double v = double(x[int64_t(r0[i]) * nrhs + j]);
    if (r1[i] >= 0) v = 0.5 * (v + double(x[int64_t(r1[i]) * nrhs + j]));
    out[t] = v;
}

template <typename T>
__global__ void k_fill(int64_t count, T value, T* __restrict__ dst) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < count) dst[t] = value;
}

template <typename TS, typename TD>
__global__ void k_convert(int64_t count, const TS* __restrict__ src, TD* __restrict__ dst) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < count) dst[t] = static_cast<TD>(static_cast<float>(src[t]));
}

template <>
__global__ void k_convert<float, double>(int64_t count, const float* __restrict__ src, double* __restrict__ dst) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < count) dst[t] = double(src[t]);
}

template <typename TD>
__global__ void k_add(int64_t count, const TD* __restrict__ d, double* __restrict__ x) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < count) x[t] += double(d[t]);
}

template <typename TV>
__global__ void k_waves_io(int64_t np, int nrhs, const int32_t* __restrict__ abi2port, TV* __restrict__ a,
                           double* __restrict__ abi, int to_abi) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= np * nrhs) return;
    const int r = int(t / np);
    const int64_t q = t - int64_t(r) * np;
    const int64_t k = int64_t(abi2port[q]) * nrhs + r;
    if (to_abi)
        abi[t] = double(a[k]);
    else
        a[k] = TV(abi[t]);
}

__global__ void k_grad(int64_t m, int n, int nrhs, const double* __restrict__ x, const double* __restrict__ lam,
                       const int32_t* __restrict__ ij, double* __restrict__ out) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const int i = ij[2 * e], j = ij[2 * e + 1];
    if (i < 0 || i >= n || j < 0 || j >= n) {  // a branch naming no node: no read, NaN out
        out[e] = __builtin_nan("");
        return;
    }
    double acc = 0.0;
    for (int r = 0; r < nrhs; ++r) {
        const int64_t o = int64_t(r) * n;
        acc += (lam[o + i] - lam[o + j]) * (x[o + i] - x[o + j]);
    }
    out[e] = -acc;
}

// dL/dA over the entries of a sparse pattern: out[k] = -sum_r lam[r][row[k]] x[r][col[k]]
__global__ void k_grad_entries(int64_t nnz, int n, int nrhs, const double* __restrict__ x,
                               const double* __restrict__ lam, const int32_t* __restrict__ row,
                               const int32_t* __restrict__ col, double* __restrict__ out) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    const int i = row[k], j = col[k];
    double acc = 0.0;
    for (int r = 0; r < nrhs; ++r) {
        const int64_t o = int64_t(r) * n;
        acc += lam[o + i] * x[o + j];
    }
    out[k] = -acc;
}

inline unsigned blocks_for(int64_t count, int bs = kBlock) { return unsigned((count + bs - 1) / bs); }

}  // namespace

hipError_t launch_grad_entries(int64_t nnz, int n, int nrhs, const double* x, const double* lam, const int32_t* row,
                               const int32_t* col, double* dL_dA, hipStream_t st) {
    if (nnz == 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_entries, dim3(blocks_for(nnz)), dim3(kBlock), 0, st, nnz, n, nrhs, x, lam, row, col,
                       dL_dA);
    return hipGetLastError();
}

hipError_t launch_expand(int rows, int nrhs, int n_in, const int32_t* src, const double* w, const double* in,
                         bool in_rhs_major, double* out, hipStream_t st) {
    const int64_t total = int64_t(rows) * nrhs;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_expand, dim3(unsigned((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, rows, nrhs, n_in,
                       src, w, in, in_rhs_major ? 1 : 0, out);
    return hipGetLastError();
}

template <typename TX>
hipError_t launch_restrict(int n, int nrhs, const int32_t* r0, const int32_t* r1, const TX* x, double* out,
                           bool out_rhs_major, hipStream_t st) {
    const int64_t total = int64_t(n) * nrhs;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_restrict<TX>, dim3(unsigned((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, n, nrhs, r0,
                       r1, x, out, out_rhs_major ? 1 : 0);
    return hipGetLastError();
}
template hipError_t launch_restrict<double>(int, int, const int32_t*, const int32_t*, const double*, double*, bool,
                                            hipStream_t);
template hipError_t launch_restrict<float>(int, int, const int32_t*, const int32_t*, const float*, double*, bool,
                                           hipStream_t);

// right-hand sides from which the renumberings go through LDS tiles
constexpr int kTiledRhs = 16;

hipError_t launch_gather(int n, int nrhs, const int32_t* perm, const double* src, double* dst,
                         hipStream_t st) {
    if (nrhs >= kTiledRhs && n > 0) {
        hipLaunchKernelGGL(k_gather_tiled, dim3(unsigned((n + kTile - 1) / kTile), unsigned((nrhs + kTile - 1) / kTile)),
                           dim3(kBlock), 0, st, n, nrhs, perm, src, dst);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(int64_t(n) * nrhs)), dim3(kBlock), 0, st, n, nrhs, perm, src,
                       dst);
    return hipGetLastError();
}

hipError_t launch_scatter(int n, int nrhs, const int32_t* iperm, const double* src, double* dst,
                          hipStream_t st) {
    if (nrhs >= kTiledRhs && n > 0) {
        hipLaunchKernelGGL(k_scatter_tiled, dim3(unsigned((n + kTile - 1) / kTile), unsigned((nrhs + kTile - 1) / kTile)),
                           dim3(kBlock), 0, st, n, nrhs, iperm, src, dst);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(int64_t(n) * nrhs)), dim3(kBlock), 0, st, n, nrhs, iperm,
                       src, dst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(int64_t count, T value, T* dst, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks_for(count)), dim3(kBlock), 0, st, count, value, dst);
    return hipGetLastError();
}

template <typename TS, typename TD>
hipError_t launch_convert(int64_t count, const TS* src, TD* dst, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_convert<TS, TD>), dim3(blocks_for(count)), dim3(kBlock), 0, st, count, src, dst);
    return hipGetLastError();
}

template <typename TD>
hipError_t launch_add(int64_t count, const TD* d, double* x, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_add<TD>, dim3(blocks_for(count)), dim3(kBlock), 0, st, count, d, x);
    return hipGetLastError();
}

template <typename TV>
hipError_t launch_waves_io(int64_t np, int nrhs, const int32_t* abi2port, TV* a, double* abi, bool to_abi,
                           hipStream_t st) {
    if (np * nrhs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_waves_io<TV>, dim3(blocks_for(np * nrhs)), dim3(kBlock), 0, st, np, nrhs, abi2port, a,
                       abi, to_abi ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_grad(int64_t m, int n, int nrhs, const double* x, const double* lam, const int32_t* ij,
                       double* dL_dg, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad, dim3(blocks_for(m)), dim3(kBlock), 0, st, m, n, nrhs, x, lam, ij, dL_dg);
    return hipGetLastError();
}

template hipError_t launch_fill<double>(int64_t, double, double*, hipStream_t);
template hipError_t launch_fill<float>(int64_t, float, float*, hipStream_t);
template hipError_t launch_fill<int>(int64_t, int, int*, hipStream_t);
template hipError_t launch_convert<double, float>(int64_t, const double*, float*, hipStream_t);
template hipError_t launch_convert<float, double>(int64_t, const float*, double*, hipStream_t);
template hipError_t launch_convert<double, __bf16>(int64_t, const double*, __bf16*, hipStream_t);
template hipError_t launch_fill<__bf16>(int64_t, __bf16, __bf16*, hipStream_t);
template hipError_t launch_add<float>(int64_t, const float*, double*, hipStream_t);
template hipError_t launch_add<double>(int64_t, const double*, double*, hipStream_t);
template hipError_t launch_waves_io<double>(int64_t, int, const int32_t*, double*, double*, bool, hipStream_t);
template hipError_t launch_waves_io<float>(int64_t, int, const int32_t*, float*, double*, bool, hipStream_t);

}  // namespace vtm
