// Setup kernels: every sub-circuit's tearing-modified matrix and its inverse.
//
// K_s = A_ss + diag(dmod): the untorn diagonal block of the sub-circuit with, at
// every port node, the cut branch g replaced by the port conductance G (the
// "C + W" block of eq. 11 once the twin is eliminated).  Inverted by
// Gauss-Jordan elimination with partial pivoting, in FP64, then written in the
// working precision and the column-group layout of layout.hpp.
#include <climits>

#include "kernels.hpp"
#include "layout.hpp"
#include "tiles.hpp"

namespace vtm {

namespace {

constexpr int kBlock = 256;

__device__ inline void arg_better(double& bv, int& bi, double v, int i) {
    if (v > bv || (v == bv && i < bi)) {
        bv = v;
        bi = i;
    }
}

// Block-wide argmax of |col[i * stride]| over rows i in [lo, n); ties go to the
// lowest row.  Returns INT_MAX if no entry is a number.  All threads call it.
__device__ int block_argmax(const double* colp, int stride, int lo, int n, double* red_v, int* red_i) {
    double bv = -1.0;
    int bi = INT_MAX;
    for (int i = lo + int(threadIdx.x); i < n; i += blockDim.x) arg_better(bv, bi, fabs(colp[i * stride]), i);
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        arg_better(bv, bi, ov, oi);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red_v[wave] = bv;
        red_i[wave] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = red_v[0];
        int i = red_i[0];
        for (int w = 1; w < int(blockDim.x >> 6); ++w) arg_better(v, i, red_v[w], red_i[w]);
        red_i[0] = i;
    }
    __syncthreads();
    const int p = red_i[0];
    __syncthreads();
    return p;
}

// Writes the column-major FP64 inverse Mcm (Mcm[c * n + r] = Kinv(r, c)) into
// dst in the column-group layout; destination-ordered, so stores are coalesced.
template <typename TO>
__device__ void store_layout(const double* Mcm, int n, TO* dst) {
    const int64_t cnt = int64_t(n) * n;
    for (int64_t d = threadIdx.x; d < cnt; d += blockDim.x) {
        int r, c;
        inv_rc<TO>(n, d, r, c);
        dst[d] = TO(Mcm[int64_t(c) * n + r]);
    }
}

// ---------------------------------------------------------------------------
// LDS path: one workgroup per sub-circuit with n <= kLdsSetupMax.  M holds K^T
// row-major, so the in-place inverse is Kinv column-major.
// ---------------------------------------------------------------------------
template <typename TO, bool COLMAJOR>
__global__ void __launch_bounds__(kBlock)
    k_setup_lds(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs,
                const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                const double* __restrict__ val, const double* __restrict__ dmod, TO* __restrict__ out,
                int* flag) {
    __shared__ double M[kLdsSetupMax * kLdsSetupMax];
    __shared__ double fcol[kLdsSetupMax];
    __shared__ int ipiv[kLdsSetupMax];
    __shared__ double red_v[kBlock / 64];
    __shared__ int red_i[kBlock / 64];

    const int s = blockIdx.x;
    const int off = sub_off[s];
    const int n = sub_off[s + 1] - off;
    if (n > kLdsSetupMax) return;
    const int tid = threadIdx.x, bs = blockDim.x;

    for (int t = tid; t < n * n; t += bs) M[t] = 0.0;
    __syncthreads();
    for (int r = tid; r < n; r += bs) {
        for (int k = rowptr[off + r]; k < rowptr[off + r + 1]; ++k) {
            const int c = col[k] - off;
            if (c >= 0 && c < n) M[c * n + r] += val[k];
        }
        M[r * n + r] += dmod[off + r];
    }
    __syncthreads();

    bool bad = false;
    for (int k = 0; k < n; ++k) {
        int p = block_argmax(M + k, n, k, n, red_v, red_i);
        if (p == INT_MAX) {
            bad = true;
            p = k;
        }
        if (tid == 0) ipiv[k] = p;
        if (p != k)
            for (int j = tid; j < n; j += bs) {
                const double t = M[k * n + j];
                M[k * n + j] = M[p * n + j];
                M[p * n + j] = t;
            }
        __syncthreads();
        double pv = M[k * n + k];
        if (pv == 0.0 || !isfinite(pv)) {
            bad = true;
            pv = 1.0;
        }
        for (int i = tid; i < n; i += bs) fcol[i] = M[i * n + k];
        __syncthreads();
        for (int j = tid; j < n; j += bs) M[k * n + j] = (j == k ? 1.0 : M[k * n + j]) / pv;
        __syncthreads();
        for (int t = tid; t < n * n; t += bs) {
            const int i = t / n, j = t - i * n;
            if (i != k) M[t] = (j == k ? 0.0 : M[t]) - fcol[i] * M[k * n + j];
        }
        __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
        const int p = ipiv[k];
        if (p != k)
            for (int i = tid; i < n; i += bs) {
                const double t = M[i * n + k];
                M[i * n + k] = M[i * n + p];
                M[i * n + p] = t;
            }
        __syncthreads();
    }
    if constexpr (COLMAJOR) {
        for (int t = tid; t < n * n; t += bs) out[kofs[s] + t] = TO(M[t]);
    } else {
        store_layout<TO>(M, n, out + kofs[s]);
    }
    if (bad && tid == 0) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// Global path (n > kLdsSetupMax): assemble K^T into FP64 scratch ...
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
    k_assemble(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs,
               const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
               const double* __restrict__ val, const double* __restrict__ dmod, double* __restrict__ out) {
    const int s = blockIdx.x;
    const int off = sub_off[s];
    const int n = sub_off[s + 1] - off;
    if (n <= kLdsSetupMax) return;
    double* M = out + kofs[s];
    const int tid = threadIdx.x, bs = blockDim.x;
    for (int64_t t = tid; t < int64_t(n) * n; t += bs) M[t] = 0.0;
    __syncthreads();
    for (int r = tid; r < n; r += bs) {
        for (int k = rowptr[off + r]; k < rowptr[off + r + 1]; ++k) {
            const int c = col[k] - off;
            if (c >= 0 && c < n) M[int64_t(c) * n + r] += val[k];
        }
        M[int64_t(r) * n + r] += dmod[off + r];
    }
}

// ... and invert it in place, nb columns at a time.  The panel is eliminated in
// LDS (pivot search over all rows below the diagonal); its row swaps and its
// elimination steps are then applied to every other column as one rank-kb
// update: R <- P R + (E_J - I_J) (P R)_J, where E_J are the panel columns after
// elimination and P the panel's row swaps.  Columns are unscrambled at the end.
template <int NB>
__global__ void __launch_bounds__(kBlock)
    k_gj_global(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs,
                double* __restrict__ base, int nb, int* flag) {
    extern __shared__ double sm[];
    const int s = blockIdx.x;
    const int n = sub_off[s + 1] - sub_off[s];
    if (n <= kLdsSetupMax) return;
    double* M = base + kofs[s];
    double* Pn = sm;                 // [n][nb]
    double* fcol = Pn + n * nb;      // [n]
    double* red_v = fcol + n;        // [4]
    int* red_i = reinterpret_cast<int*>(red_v + 4);
    int* ipiv = red_i + 4;           // [n]
    const int tid = threadIdx.x, bs = blockDim.x;
    bool bad = false;

    for (int k0 = 0; k0 < n; k0 += nb) {
        const int kb = min(nb, n - k0);
        for (int t = tid; t < n * kb; t += bs) {
            const int i = t / kb, jj = t - i * kb;
            Pn[i * nb + jj] = M[int64_t(i) * n + k0 + jj];
        }
        __syncthreads();
        for (int kk = 0; kk < kb; ++kk) {
            const int k = k0 + kk;
            int p = block_argmax(Pn + kk, nb, k, n, red_v, red_i);
            if (p == INT_MAX) {
                bad = true;
                p = k;
            }
            if (tid == 0) ipiv[k] = p;
            if (p != k)
                for (int jj = tid; jj < kb; jj += bs) {
                    const double t = Pn[k * nb + jj];
                    Pn[k * nb + jj] = Pn[p * nb + jj];
                    Pn[p * nb + jj] = t;
                }
            __syncthreads();
            double pv = Pn[k * nb + kk];
            if (pv == 0.0 || !isfinite(pv)) {
                bad = true;
                pv = 1.0;
            }
            for (int i = tid; i < n; i += bs) fcol[i] = Pn[i * nb + kk];
            __syncthreads();
            for (int jj = tid; jj < kb; jj += bs) Pn[k * nb + jj] = (jj == kk ? 1.0 : Pn[k * nb + jj]) / pv;
            __syncthreads();
            for (int t = tid; t < n * kb; t += bs) {
                const int i = t / kb, jj = t - i * kb;
                if (i != k) Pn[i * nb + jj] = (jj == kk ? 0.0 : Pn[i * nb + jj]) - fcol[i] * Pn[k * nb + jj];
            }
            __syncthreads();
        }
        for (int c = tid; c < n; c += bs) {
            if (c >= k0 && c < k0 + kb) continue;
            double rj[NB];
#pragma unroll
            for (int kk = 0; kk < NB; ++kk) {
                if (kk < kb) {
                    const int k = k0 + kk, p = ipiv[k];
                    if (p != k) {
                        const double t = M[int64_t(k) * n + c];
                        M[int64_t(k) * n + c] = M[int64_t(p) * n + c];
                        M[int64_t(p) * n + c] = t;
                    }
                }
            }
#pragma unroll
            for (int kk = 0; kk < NB; ++kk) rj[kk] = kk < kb ? M[int64_t(k0 + kk) * n + c] : 0.0;
            for (int i = 0; i < n; ++i) {
                double acc = M[int64_t(i) * n + c];
#pragma unroll
                for (int kk = 0; kk < NB; ++kk)
                    if (kk < kb) acc += (Pn[i * nb + kk] - (i == k0 + kk ? 1.0 : 0.0)) * rj[kk];
                M[int64_t(i) * n + c] = acc;
            }
        }
        __syncthreads();
        for (int t = tid; t < n * kb; t += bs) {
            const int i = t / kb, jj = t - i * kb;
            M[int64_t(i) * n + k0 + jj] = Pn[i * nb + jj];
        }
        __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
        const int p = ipiv[k];
        if (p != k)
            for (int i = tid; i < n; i += bs) {
                const double t = M[int64_t(i) * n + k];
                M[int64_t(i) * n + k] = M[int64_t(i) * n + p];
                M[int64_t(i) * n + p] = t;
            }
        __syncthreads();
    }
    if (bad && tid == 0) atomicOr(flag, 1);
}

// column-major FP64 scratch -> working precision, column-group layout
template <typename TO>
__global__ void __launch_bounds__(kBlock)
    k_to_layout(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs,
                const double* __restrict__ src, TO* __restrict__ dst) {
    const int s = blockIdx.x;
    const int n = sub_off[s + 1] - sub_off[s];
    if (n <= kLdsSetupMax) return;
    store_layout<TO>(src + kofs[s], n, dst + kofs[s]);
}

// column-major FP64 scratch -> zero-padded MFMA operand tiles (tiles.hpp)
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_to_tiles(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs,
               const int64_t* __restrict__ mofs, const double* __restrict__ src, T* __restrict__ dst) {
    const int s = blockIdx.x;
    const int n = sub_off[s + 1] - sub_off[s];
    const int np = tile_pad(n);
    const double* M = src + kofs[s];
    T* o = dst + mofs[s];
    const int64_t cnt = int64_t(np) * np;
    for (int64_t d = threadIdx.x; d < cnt; d += blockDim.x) {
        int r, c;
        tile_rc<T>(np, d, r, c);
        o[d] = (r < n && c < n) ? static_cast<T>(M[int64_t(c) * n + r]) : static_cast<T>(0.0);
    }
}

// the large sub-circuits: assemble and invert in FP64 scratch (column-major)
hipError_t invert_large(int S, int max_ns, const int32_t* sub_off, const int64_t* kofs, const int32_t* rowptr,
                        const int32_t* col, const double* val, const double* dmod, double* scratch64, int* flag,
                        hipStream_t st) {
    if (!scratch64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_assemble, dim3(S), dim3(kBlock), 0, st, sub_off, kofs, rowptr, col, val, dmod, scratch64);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // panel width: as many columns as fit next to the pivot bookkeeping in 64 KiB of LDS
    constexpr int kLds = 65536;
    const int fixed = max_ns * (8 + 4) + 64;
    int nb = (kLds - fixed) / (8 * max_ns);
    if (nb < 1) return hipErrorInvalidValue;
    nb = nb > 16 ? 16 : nb;
    const size_t lds = size_t(max_ns) * nb * 8 + fixed;
    hipLaunchKernelGGL(k_gj_global<16>, dim3(S), dim3(kBlock), lds, st, sub_off, kofs, scratch64, nb, flag);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_setup_tiles(int S, int max_ns, const int32_t* sub_off, const int64_t* kofs, const int64_t* mofs,
                              const int32_t* rowptr, const int32_t* col, const double* val, const double* dmod,
                              T* out, double* scratch64, int* flag, hipStream_t st) {
    if (!scratch64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_setup_lds<double, true>), dim3(S), dim3(kBlock), 0, st, sub_off, kofs, rowptr, col, val,
                       dmod, scratch64, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (max_ns > kLdsSetupMax) {
        e = invert_large(S, max_ns, sub_off, kofs, rowptr, col, val, dmod, scratch64, flag, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_to_tiles<T>, dim3(S), dim3(kBlock), 0, st, sub_off, kofs, mofs, scratch64, out);
    return hipGetLastError();
}

template <typename TO>
hipError_t launch_setup(int S, int max_ns, const int32_t* sub_off, const int64_t* kofs, const int32_t* rowptr,
                        const int32_t* col, const double* val, const double* dmod, TO* out, double* scratch64,
                        int* flag, hipStream_t st) {
    hipLaunchKernelGGL((k_setup_lds<TO, false>), dim3(S), dim3(kBlock), 0, st, sub_off, kofs, rowptr, col, val,
                       dmod, out, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || max_ns <= kLdsSetupMax) return e;
    e = invert_large(S, max_ns, sub_off, kofs, rowptr, col, val, dmod, scratch64, flag, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_to_layout<TO>, dim3(S), dim3(kBlock), 0, st, sub_off, kofs, scratch64, out);
    return hipGetLastError();
}

template hipError_t launch_setup<double>(int, int, const int32_t*, const int64_t*, const int32_t*, const int32_t*,
                                         const double*, const double*, double*, double*, int*, hipStream_t);
template hipError_t launch_setup<float>(int, int, const int32_t*, const int64_t*, const int32_t*, const int32_t*,
                                        const double*, const double*, float*, double*, int*, hipStream_t);
template hipError_t launch_setup_tiles<__bf16>(int, int, const int32_t*, const int64_t*, const int64_t*,
                                              const int32_t*, const int32_t*, const double*, const double*, __bf16*,
                                              double*, int*, hipStream_t);
template hipError_t launch_setup_tiles<double>(int, int, const int32_t*, const int64_t*, const int64_t*,
                                              const int32_t*, const int32_t*, const double*, const double*, double*,
                                              double*, int*, hipStream_t);

}  // namespace vtm
