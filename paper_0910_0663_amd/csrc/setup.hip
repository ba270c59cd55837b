// Setup kernels: every sub-circuit's tearing-modified matrix and its inverse.
//
// K_s = A_ss + diag(dmod): the untorn diagonal block of the sub-circuit with, at
// every port node, the cut branch g replaced by the port conductance G (the
// "C + W" block of eq. 11 once the twin is eliminated).  Inverted by
// Gauss-Jordan elimination with partial pivoting, in FP64, then written in the
// working precision and the column-group layout of layout.hpp.
#include <algorithm>
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
__device__ void store_layout(const double* Mcm, int n, TO* dst, int part = 0, int parts = 1) {
    const int64_t cnt = int64_t(n) * n;
    for (int64_t d = int64_t(part) * blockDim.x + threadIdx.x; d < cnt; d += int64_t(blockDim.x) * parts) {
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

// ... and invert it in place, NB columns at a time (blocked Gauss-Jordan with
// partial pivoting; NB = 16).  Each panel step is a few
// launches, so that a few large sub-circuits still spread over the whole chip.
// k_gj_panel (one workgroup per sub-circuit) eliminates the panel's columns
// (pivot search over all rows below the diagonal; the panel E_J in global
// memory, [n][NB] at panel + (2 NB + 1) sub_off[s]); k_gj_swap applies the
// panel's row swaps P to every other column and keeps their pivot rows
// (P R)_J ([NB][n] right after E_J; then n doubles of scratch for the pivot
// column), one column per thread.  k_gj_update then applies the elimination to
// every other column as one rank-kb update, R <- P R + (E_J - I_J) (P R)_J, over
// a grid of column blocks x row blocks.  k_gj_unscramble undoes the pivoting's
// column order at the end.
constexpr int kNB = 16;
constexpr int kWideNB = 16;       // panel width of the very large sub-circuits (32 measured no faster:
                                  // the update is bound by its arithmetic, not by passes over K)
constexpr int kMaxLarge = 16384;  // largest sub-circuit (the planner's limit)
constexpr int kPanelBlock = 1024;
constexpr int kUpdateRows = 128;  // rows per thread of the update

__global__ void __launch_bounds__(kPanelBlock)
    k_gj_panel(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs, double* __restrict__ base,
               int k0, double* __restrict__ panel, int32_t* __restrict__ ipiv, int* flag) {
    __shared__ double red_v[kPanelBlock / 64];
    __shared__ int red_i[kPanelBlock / 64];
    const int s = blockIdx.x;
    const int off = sub_off[s], n = sub_off[s + 1] - off;
    if (n <= kLdsSetupMax || k0 >= n || n > kMaxLarge) return;
    const int kb = min(kNB, n - k0);
    double* M = base + kofs[s];
    double* Pn = panel + int64_t(off) * (2 * kNB + 1);
    double* R = Pn + int64_t(n) * kNB;
    double* fcol = R + int64_t(n) * kNB;
    const int tid = threadIdx.x, bs = blockDim.x;
    bool bad = false;
    for (int t = tid; t < n * kb; t += bs) {
        const int i = t / kb, jj = t - i * kb;
        Pn[i * kNB + jj] = M[int64_t(i) * n + k0 + jj];
    }
    __syncthreads();
    for (int kk = 0; kk < kb; ++kk) {
        const int k = k0 + kk;
        int p = block_argmax(Pn + kk, kNB, k, n, red_v, red_i);
        if (p == INT_MAX) {
            bad = true;
            p = k;
        }
        if (tid == 0) ipiv[off + k] = p;
        if (p != k)
            for (int jj = tid; jj < kb; jj += bs) {
                const double t = Pn[k * kNB + jj];
                Pn[k * kNB + jj] = Pn[p * kNB + jj];
                Pn[p * kNB + jj] = t;
            }
        __syncthreads();
        double pv = Pn[k * kNB + kk];
        if (pv == 0.0 || !isfinite(pv)) {
            bad = true;
            pv = 1.0;
        }
        for (int i = tid; i < n; i += bs) fcol[i] = Pn[i * kNB + kk];
        __syncthreads();
        for (int jj = tid; jj < kb; jj += bs) Pn[k * kNB + jj] = (jj == kk ? 1.0 : Pn[k * kNB + jj]) / pv;
        __syncthreads();
        for (int t = tid; t < n * kb; t += bs) {
            const int i = t / kb, jj = t - i * kb;
            if (i != k) Pn[i * kNB + jj] = (jj == kk ? 0.0 : Pn[i * kNB + jj]) - fcol[i] * Pn[k * kNB + jj];
        }
        __syncthreads();
    }
    // the panel's columns are final for this step
    for (int t = tid; t < n * kb; t += bs) {
        const int i = t / kb, jj = t - i * kb;
        M[int64_t(i) * n + k0 + jj] = Pn[i * kNB + jj];
    }
    if (bad && tid == 0) atomicOr(flag, 1);
}

// The same panel elimination for a few very large sub-circuits, where one
// workgroup's chain of 16 pivot steps over n rows is the setup's bottleneck:
// each step is two launches, the pivot (search, row swap, scaling of the pivot
// row; one workgroup per sub-circuit) and the elimination of every other row of
// the panel (one row per thread over a grid of row blocks).  k_gjw_load and
// k_gjw_store move the panel between K and the panel buffer.
template <int NB>
__global__ void __launch_bounds__(kBlock)
    k_gjw_load(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs,
               const double* __restrict__ base, int k0, double* __restrict__ panel, int store) {
    const int s = blockIdx.x;
    const int off = sub_off[s], n = sub_off[s + 1] - off;
    if (n <= kLdsSetupMax || k0 >= n || n > kMaxLarge) return;
    const int i = blockIdx.y * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int kb = min(NB, n - k0);
    double* M = const_cast<double*>(base) + kofs[s] + int64_t(i) * n + k0;
    double* Pn = panel + int64_t(off) * (2 * NB + 1) + int64_t(i) * NB;
    for (int jj = 0; jj < kb; ++jj) {
        if (store)
            M[jj] = Pn[jj];
        else
            Pn[jj] = M[jj];
    }
}

template <int NB>
__global__ void __launch_bounds__(kPanelBlock)
    k_gjw_pivot(const int32_t* __restrict__ sub_off, int k0, int kk, double* __restrict__ panel,
                int32_t* __restrict__ ipiv, int* flag) {
    __shared__ double red_v[kPanelBlock / 64];
    __shared__ int red_i[kPanelBlock / 64];
    const int s = blockIdx.x;
    const int off = sub_off[s], n = sub_off[s + 1] - off;
    if (n <= kLdsSetupMax || n > kMaxLarge) return;
    const int kb = min(NB, n - k0);
    if (k0 >= n || kk >= kb) return;
    const int k = k0 + kk;
    double* Pn = panel + int64_t(off) * (2 * NB + 1);
    const int tid = threadIdx.x, bs = blockDim.x;
    int p = block_argmax(Pn + kk, NB, k, n, red_v, red_i);
    bool bad = false;
    if (p == INT_MAX) {
        bad = true;
        p = k;
    }
    if (tid == 0) ipiv[off + k] = p;
    if (p != k)
        for (int jj = tid; jj < kb; jj += bs) {
            const double t = Pn[k * NB + jj];
            Pn[k * NB + jj] = Pn[p * NB + jj];
            Pn[p * NB + jj] = t;
        }
    __syncthreads();
    double pv = Pn[k * NB + kk];
    if (pv == 0.0 || !isfinite(pv)) {
        bad = true;
        pv = 1.0;
    }
    __syncthreads();  // every thread has read the pivot before row k is scaled
    for (int jj = tid; jj < kb; jj += bs) Pn[k * NB + jj] = (jj == kk ? 1.0 : Pn[k * NB + jj]) / pv;
    if (bad && tid == 0) atomicOr(flag, 1);
}

template <int NB>
__global__ void __launch_bounds__(kBlock)
    k_gjw_elim(const int32_t* __restrict__ sub_off, int k0, int kk, double* __restrict__ panel) {
    const int s = blockIdx.x;
    const int off = sub_off[s], n = sub_off[s + 1] - off;
    if (n <= kLdsSetupMax || n > kMaxLarge) return;
    const int kb = min(NB, n - k0);
    if (k0 >= n || kk >= kb) return;
    const int k = k0 + kk;
    const int i = blockIdx.y * blockDim.x + threadIdx.x;
    if (i >= n || i == k) return;
    double* Pn = panel + int64_t(off) * (2 * NB + 1);
    const double f = Pn[i * NB + kk];
    for (int jj = 0; jj < kb; ++jj)
        Pn[i * NB + jj] = (jj == kk ? 0.0 : Pn[i * NB + jj]) - f * Pn[k * NB + jj];
}

// every other column: the panel's row swaps, and its pivot rows kept for the update
template <int NB>
__global__ void __launch_bounds__(kBlock)
    k_gj_swap(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs, double* __restrict__ base,
              int k0, double* __restrict__ panel, const int32_t* __restrict__ ipiv) {
    const int s = blockIdx.x;
    const int off = sub_off[s], n = sub_off[s + 1] - off;
    if (n <= kLdsSetupMax || k0 >= n || n > kMaxLarge) return;
    const int kb = min(NB, n - k0);
    const int c = blockIdx.y * blockDim.x + threadIdx.x;
    if (c >= n || (c >= k0 && c < k0 + kb)) return;
    double* M = base + kofs[s];
    double* R = panel + int64_t(off) * (2 * NB + 1) + int64_t(n) * NB;
    for (int kk = 0; kk < kb; ++kk) {
        const int k = k0 + kk, p = ipiv[off + k];
        if (p != k) {
            const double t = M[int64_t(k) * n + c];
            M[int64_t(k) * n + c] = M[int64_t(p) * n + c];
            M[int64_t(p) * n + c] = t;
        }
    }
    for (int kk = 0; kk < kb; ++kk) R[int64_t(kk) * n + c] = M[int64_t(k0 + kk) * n + c];
}

// The rank-kb update of every column outside the panel, one column per thread and
// kUpdateRows rows per workgroup: the workgroup first stages its rows of
// E_J - I_J in LDS (zero beyond kb, so no term needs a branch), then each thread
// takes its column's pivot rows (P R)_J into registers and walks its rows eight at
// a time with their loads issued together.  Each entry accumulates its kb
// products in panel order.
template <int NB>
__global__ void __launch_bounds__(kBlock)
    k_gj_update(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs, double* __restrict__ base,
                int k0, const double* __restrict__ panel) {
    __shared__ double e_s[kUpdateRows][NB];
    const int s = blockIdx.x;
    const int off = sub_off[s], n = sub_off[s + 1] - off;
    if (n <= kLdsSetupMax || k0 >= n || n > kMaxLarge) return;  // uniform over the workgroup
    const int kb = min(NB, n - k0);
    const int i0 = blockIdx.z * kUpdateRows, i1 = min(n, i0 + kUpdateRows);
    if (i0 >= n) return;                                         // uniform over the workgroup
    const double* Pn = panel + int64_t(off) * (2 * NB + 1);
    const double* R = Pn + int64_t(n) * NB;
    for (int t = threadIdx.x; t < kUpdateRows * NB; t += blockDim.x) {
        const int ii = t / NB, kk = t - ii * NB, i = i0 + ii;
        e_s[ii][kk] = (i < i1 && kk < kb) ? Pn[int64_t(i) * NB + kk] - (i == k0 + kk ? 1.0 : 0.0) : 0.0;
    }
    __syncthreads();
    const int c = blockIdx.y * blockDim.x + threadIdx.x;
    if (c >= n || (c >= k0 && c < k0 + kb)) return;  // no barrier follows
    double* M = base + kofs[s];
    double rj[NB];
#pragma unroll
    for (int kk = 0; kk < NB; ++kk) rj[kk] = kk < kb ? R[int64_t(kk) * n + c] : 0.0;
    constexpr int U = 8;
    int i = i0;
    for (; i + U <= i1; i += U) {
        double m[U];
#pragma unroll
        for (int u = 0; u < U; ++u) m[u] = M[int64_t(i + u) * n + c];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int kk = 0; kk < NB; ++kk) m[u] += e_s[i - i0 + u][kk] * rj[kk];
#pragma unroll
        for (int u = 0; u < U; ++u) M[int64_t(i + u) * n + c] = m[u];
    }
    for (; i < i1; ++i) {
        double acc = M[int64_t(i) * n + c];
#pragma unroll
        for (int kk = 0; kk < NB; ++kk) acc += e_s[i - i0][kk] * rj[kk];
        M[int64_t(i) * n + c] = acc;
    }
}

__global__ void __launch_bounds__(kBlock)
    k_gj_unscramble(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs, double* __restrict__ base,
                    const int32_t* __restrict__ ipiv) {
    const int s = blockIdx.x;
    const int off = sub_off[s], n = sub_off[s + 1] - off;
    if (n <= kLdsSetupMax || n > kMaxLarge) return;
    const int i = blockIdx.y * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double* row = base + kofs[s] + int64_t(i) * n;
    for (int k = n - 1; k >= 0; --k) {
        const int p = ipiv[off + k];
        if (p != k) {
            const double t = row[k];
            row[k] = row[p];
            row[p] = t;
        }
    }
}

// column-major FP64 scratch -> working precision, column-group layout
template <typename TO>
__global__ void __launch_bounds__(kBlock)
    k_to_layout(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs,
                const double* __restrict__ src, TO* __restrict__ dst) {
    const int s = blockIdx.x;
    const int n = sub_off[s + 1] - sub_off[s];
    if (n <= kLdsSetupMax) return;
    store_layout<TO>(src + kofs[s], n, dst + kofs[s], int(blockIdx.y), int(gridDim.y));
}

// column-major FP64 scratch -> zero-padded MFMA operand tiles (tiles.hpp)
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_to_tiles(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs,
               const int64_t* __restrict__ mofs, const double* __restrict__ src, T* __restrict__ dst,
               int transpose) {
    const int s = blockIdx.x;
    const int n = sub_off[s + 1] - sub_off[s];
    const int np = tile_pad(n);
    const double* M = src + kofs[s];
    T* o = dst + mofs[s];
    const int64_t cnt = int64_t(np) * np;
    for (int64_t d = int64_t(blockIdx.y) * blockDim.x + threadIdx.x; d < cnt; d += int64_t(blockDim.x) * gridDim.y) {
        int r, c;
        tile_rc<T>(np, d, r, c);
        // element (r, c) of K^-1 (column-major), or of K^-T: element (c, r)
        const int64_t at = transpose ? int64_t(r) * n + c : int64_t(c) * n + r;
        o[d] = (r < n && c < n) ? static_cast<T>(M[at]) : static_cast<T>(0.0);
    }
}

// workgroups per sub-circuit for an n x n copy: enough for some 2048 workgroups in all
int copy_parts(int S, int n) {
    const int64_t per = (int64_t(n) * n + 4095) / 4096;  // at 16 elements per thread
    const int64_t want = (2048 + S - 1) / S;
    return int(std::max<int64_t>(1, std::min<int64_t>(per, want)));
}

// the large sub-circuits: assemble and invert in FP64 scratch (column-major)
hipError_t invert_large(int S, int max_ns, const int32_t* sub_off, const int64_t* kofs, const int32_t* rowptr,
                        const int32_t* col, const double* val, const double* dmod, double* scratch64, double* panel,
                        int32_t* ipiv, int* flag, hipStream_t st) {
    if (!scratch64 || !panel || !ipiv || max_ns > kMaxLarge) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_assemble, dim3(S), dim3(kBlock), 0, st, sub_off, kofs, rowptr, col, val, dmod, scratch64);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 cols(unsigned(S), unsigned((max_ns + kBlock - 1) / kBlock));
    const dim3 tiles(unsigned(S), cols.y, unsigned((max_ns + kUpdateRows - 1) / kUpdateRows));
    // above 2,048 nodes the panel's pivot steps are spread over the chip (two launches each)
    if (max_ns > 2048) {
        constexpr int NB = kWideNB;
        for (int k0 = 0; k0 < max_ns; k0 += NB) {
            hipLaunchKernelGGL(k_gjw_load<NB>, cols, dim3(kBlock), 0, st, sub_off, kofs, scratch64, k0, panel, 0);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            for (int kk = 0; kk < NB; ++kk) {
                hipLaunchKernelGGL(k_gjw_pivot<NB>, dim3(S), dim3(kPanelBlock), 0, st, sub_off, k0, kk, panel, ipiv,
                                   flag);
                if ((e = hipGetLastError()) != hipSuccess) return e;
                hipLaunchKernelGGL(k_gjw_elim<NB>, cols, dim3(kBlock), 0, st, sub_off, k0, kk, panel);
                if ((e = hipGetLastError()) != hipSuccess) return e;
            }
            hipLaunchKernelGGL(k_gjw_load<NB>, cols, dim3(kBlock), 0, st, sub_off, kofs, scratch64, k0, panel, 1);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(k_gj_swap<NB>, cols, dim3(kBlock), 0, st, sub_off, kofs, scratch64, k0, panel, ipiv);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(k_gj_update<NB>, tiles, dim3(kBlock), 0, st, sub_off, kofs, scratch64, k0, panel);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    } else {
        for (int k0 = 0; k0 < max_ns; k0 += kNB) {
            hipLaunchKernelGGL(k_gj_panel, dim3(S), dim3(kPanelBlock), 0, st, sub_off, kofs, scratch64, k0, panel,
                               ipiv, flag);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(k_gj_swap<kNB>, cols, dim3(kBlock), 0, st, sub_off, kofs, scratch64, k0, panel, ipiv);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(k_gj_update<kNB>, tiles, dim3(kBlock), 0, st, sub_off, kofs, scratch64, k0, panel);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL(k_gj_unscramble, cols, dim3(kBlock), 0, st, sub_off, kofs, scratch64, ipiv);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_setup_tiles(int S, int max_ns, const int32_t* sub_off, const int64_t* kofs, const int64_t* mofs,
                              const int32_t* rowptr, const int32_t* col, const double* val, const double* dmod,
                              T* out, double* scratch64, double* panel, int32_t* ipiv, int* flag, hipStream_t st,
                              T* out_t) {
    if (!scratch64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_setup_lds<double, true>), dim3(S), dim3(kBlock), 0, st, sub_off, kofs, rowptr, col, val,
                       dmod, scratch64, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (max_ns > kLdsSetupMax) {
        e = invert_large(S, max_ns, sub_off, kofs, rowptr, col, val, dmod, scratch64, panel, ipiv, flag, st);
        if (e != hipSuccess) return e;
    }
    const dim3 grid(unsigned(S), unsigned(copy_parts(S, tile_pad(max_ns))));
    hipLaunchKernelGGL(k_to_tiles<T>, grid, dim3(kBlock), 0, st, sub_off, kofs, mofs, scratch64, out, 0);
    e = hipGetLastError();
    if (e != hipSuccess || !out_t) return e;
    hipLaunchKernelGGL(k_to_tiles<T>, grid, dim3(kBlock), 0, st, sub_off, kofs, mofs, scratch64, out_t, 1);
    return hipGetLastError();
}

template <typename TO>
hipError_t launch_setup(int S, int max_ns, const int32_t* sub_off, const int64_t* kofs, const int32_t* rowptr,
                        const int32_t* col, const double* val, const double* dmod, TO* out, double* scratch64,
                        double* panel, int32_t* ipiv, int* flag, hipStream_t st) {
    hipLaunchKernelGGL((k_setup_lds<TO, false>), dim3(S), dim3(kBlock), 0, st, sub_off, kofs, rowptr, col, val,
                       dmod, out, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || max_ns <= kLdsSetupMax) return e;
    e = invert_large(S, max_ns, sub_off, kofs, rowptr, col, val, dmod, scratch64, panel, ipiv, flag, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_to_layout<TO>, dim3(S, copy_parts(S, max_ns)), dim3(kBlock), 0, st, sub_off, kofs, scratch64,
                       out);
    return hipGetLastError();
}

template hipError_t launch_setup<double>(int, int, const int32_t*, const int64_t*, const int32_t*, const int32_t*,
                                         const double*, const double*, double*, double*, double*, int32_t*, int*,
                                         hipStream_t);
template hipError_t launch_setup<float>(int, int, const int32_t*, const int64_t*, const int32_t*, const int32_t*,
                                        const double*, const double*, float*, double*, double*, int32_t*, int*,
                                        hipStream_t);
template hipError_t launch_setup_tiles<__bf16>(int, int, const int32_t*, const int64_t*, const int64_t*,
                                              const int32_t*, const int32_t*, const double*, const double*, __bf16*,
                                              double*, double*, int32_t*, int*, hipStream_t, __bf16*);
template hipError_t launch_setup_tiles<double>(int, int, const int32_t*, const int64_t*, const int64_t*,
                                              const int32_t*, const int32_t*, const double*, const double*, double*,
                                              double*, double*, int32_t*, int*, hipStream_t, double*);

}  // namespace vtm
