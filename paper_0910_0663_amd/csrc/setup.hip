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
constexpr int kRegSetupMax = 64;  // sub-circuits up to this size: one wavefront each, rows in registers

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
    if (n > kLdsSetupMax || n <= kRegSetupMax) return;  // k_setup_reg takes n <= kRegSetupMax
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
// Register path: one wavefront per sub-circuit with n <= kRegSetupMax, lane j
// holding row j of K.  The same Gauss-Jordan steps as k_setup_lds, which works
// on M = K^T: its pivot search over M's column k is a search along K's row k,
// its swap of M's rows k and p swaps K's columns k and p in every lane's row, and
// each of its row operations on M is a column operation on K that every lane
// applies to its own row, in the same order and arithmetic.  The result (M^-1,
// row-major) is K^-1 with row r in lane r; the final column unscrambling of M is
// a permutation of those rows, applied where they are stored.  Row k of K is
// passed to the wavefront through LDS; an entry at a run-time index of a lane's
// row is read and written through selects (a register array indexed at run time
// would go to scratch memory).  No workgroup-wide barrier is needed beyond the
// wavefront's own.
// ---------------------------------------------------------------------------
template <typename TO, bool COLMAJOR>
__global__ void __launch_bounds__(64)
    k_setup_reg(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs,
                const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                const double* __restrict__ val, const double* __restrict__ dmod, TO* __restrict__ out,
                int* flag) {
    __shared__ double prow[kRegSetupMax];
    __shared__ int ipiv[kRegSetupMax];
    const int s = blockIdx.x;
    const int off = sub_off[s];
    const int n = sub_off[s + 1] - off;
    if (n > kRegSetupMax) return;  // uniform over the workgroup
    const int j = threadIdx.x;
    const bool mine = j < n;
    double row[kRegSetupMax];
#pragma unroll
    for (int c = 0; c < kRegSetupMax; ++c) row[c] = 0.0;
    // K's row j, summed as k_setup_lds sums M's column j: the row's entries, then dmod
    if (mine) {
        // the row's entries 8 at a time (its columns are distinct), each added to the
        // entry of its column
        for (int k0 = rowptr[off + j], k1 = rowptr[off + j + 1]; k0 < k1; k0 += 8) {
            int ce[8];
            double ve[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int c = k0 + e < k1 ? col[k0 + e] - off : -1;
                ce[e] = c >= 0 && c < n ? c : -1;  // entries outside the sub-circuit: none
                ve[e] = k0 + e < k1 ? val[k0 + e] : 0.0;
            }
#pragma unroll
            for (int cc = 0; cc < kRegSetupMax; ++cc) {
                double v = row[cc];
#pragma unroll
                for (int e = 0; e < 8; ++e) v = ce[e] == cc ? v + ve[e] : v;
                row[cc] = v;
            }
        }
        const double d = dmod[off + j];
#pragma unroll
        for (int cc = 0; cc < kRegSetupMax; ++cc) row[cc] = cc == j ? row[cc] + d : row[cc];
    }
    bool bad = false;
    // Each lane keeps its row rotated: at column step k, register slot i holds
    // column (i + k) mod 64, so the step's column is always slot 0 and every register
    // index below is fixed at compile time; the row turns by one slot per step.
    // Row k of K goes through LDS in the same slot order (prow[i]: column (i + k) mod
    // 64), so every lane reads its slot i at prow[i].
    for (int k = 0; k < n; ++k) {
        // pivot: the largest |K(k, i)|, i >= k, ties to the lowest i (none: INT_MAX)
        if (j == k)
#pragma unroll
            for (int i = 0; i < kRegSetupMax; ++i) prow[i] = row[i];
        __syncthreads();
        // the diagonal is the pivot when it is a number and no entry to its right is
        // larger in magnitude (ties go to the lowest column, k): one ballot; otherwise
        // the full search across the lanes
        const double dk = fabs(prow[0]);
        int p = k;
        if (!(dk >= 0.0) || __ballot(j > k && j < n && fabs(prow[j - k]) > dk) != 0) {
            double bv = -1.0;
            p = INT_MAX;
            if (j >= k && j < n) arg_better(bv, p, fabs(prow[j - k]), j);
            for (int o = 32; o > 0; o >>= 1) {
                const double ov = __shfl_xor(bv, o, 64);
                const int oi = __shfl_xor(p, o, 64);
                arg_better(bv, p, ov, oi);
            }
        }
        if (p == INT_MAX) {
            bad = true;
            p = k;
        }
        if (j == 0) ipiv[k] = p;
        if (p != k) {  // uniform: columns k (slot 0) and p (slot p - k) of every row trade places
            const int sp = p - k;
            const double a = row[0];
            double b = 0.0;
#pragma unroll
            for (int i = 1; i < kRegSetupMax; ++i) b = i == sp ? row[i] : b;
#pragma unroll
            for (int i = 1; i < kRegSetupMax; ++i) row[i] = i == sp ? a : row[i];
            row[0] = b;
            __syncthreads();  // the search has read prow
            // row k of K after the swap
            if (j == k)
#pragma unroll
                for (int i = 0; i < kRegSetupMax; ++i) prow[i] = row[i];
        }
        __syncthreads();
        // the pivot and the multipliers (M's column k)
        double pv = prow[0];
        if (pv == 0.0 || !isfinite(pv)) {
            bad = true;
            pv = 1.0;
        }
        const double rk = (j == k ? 1.0 : row[0]) / pv;  // M(k, j) scaled
        // the update, each slot written back one slot lower (the turn for the next step)
        const double r0 = rk;
#pragma unroll
        for (int i = 1; i < kRegSetupMax; ++i)
            row[i - 1] = (j == k ? 0.0 : row[i]) - prow[i] * rk;
        row[kRegSetupMax - 1] = r0;
        __syncthreads();
    }
    // after n steps slot i holds column (i + n) mod 64
    // M's columns k and ipiv[k] swapped for k = n-1 .. 0: K^-1's rows, so lane j's
    // row goes to the position those swaps carry it to
    int pos = j;
    for (int k = n - 1; k >= 0; --k) {
        const int p = ipiv[k];
        if (pos == k)
            pos = p;
        else if (pos == p)
            pos = k;
    }
    if (mine) {
        TO* dst = out + kofs[s];
#pragma unroll
        for (int i = 0; i < kRegSetupMax; ++i) {
            const int c = (i + n) & (kRegSetupMax - 1);
            if (c < n) {
                if constexpr (COLMAJOR)
                    dst[int64_t(c) * n + pos] = TO(row[i]);
                else
                    dst[inv_offset<TO>(n, pos, c)] = TO(row[i]);
            }
        }
    }
    if (bad && j == 0) atomicOr(flag, 1);
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
// partial pivoting).  Each panel step is a few launches, so that a few large
// sub-circuits still spread over the whole chip.  k_gj_panel_reg (one workgroup
// per sub-circuit, a row per thread) or k_gjw_pivot / k_gjw_elim (a launch each
// per column, for large or few sub-circuits) eliminate the panel's columns (pivot
// search over all rows below the diagonal) and leave E_J in global memory,
// column-major [NB][n] at the sub-circuit's panel slot; k_gj_swap applies
// the panel's row swaps P to every other column and keeps their pivot rows
// (P R)_J ([NB][n] right after E_J, then n doubles of scratch for the pivot
// column), one column per thread.  k_gj_update then applies the elimination to
// every other column as one rank-kb update, R <- P R + (E_J - I_J) (P R)_J, on
// the FP64 matrix cores.  k_gj_unscramble undoes the pivoting's column order at
// the end.  Each pass over K moves 16 n^2 bytes for 4 n^2 NB flops, so the panel
// is as wide as the update's MFMA throughput allows: K is read and written
// n / NB times.
constexpr int kNB = 32;           // panel width up to kWide64 nodes
constexpr int kWideNB = 64;       // panel width from kWide64 nodes
constexpr int kWide64 = 8192;
constexpr int kOneGroupMinSubs = 256;  // one workgroup eliminates each sub-circuit's panel (up to
                                       // kPanelBlock nodes) when there are enough to fill the chip
constexpr int kMaxLarge = 16384;  // largest sub-circuit (the planner's limit)
constexpr int kPanelBlock = 1024;
constexpr int kUpdWaves = 4;      // wavefronts per workgroup of the update
constexpr int kUpdRows = 512;     // rows per workgroup of the update (eight 16-row tiles per wavefront)

// doubles per node of the panel buffer for NB-column panels: E_J, (P R)_J, the
// pivot column, and one of padding that keeps every row of E_J 16-byte aligned
__host__ __device__ constexpr int panel_stride(int NB) { return 2 * NB + 2; }

typedef double dx4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// Raw buffer access with the hardware's range check: a load at or past the
// resource's byte count returns zero and such a store is dropped, so a lane is
// masked by giving it kOffOut (at least the byte count of any buffer here: an
// inverse of kMaxLarge nodes is exactly 2^31 bytes) instead of a branch.
constexpr int kBufWord3 = 0x00020000;  // gfx9 descriptor word 3: 32-bit data format
constexpr unsigned kOffOut = 0x80000000u;
__device__ inline __amdgpu_buffer_rsrc_t buf(const double* p, int64_t doubles) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), 0, int(unsigned(doubles * 8)), kBufWord3);
}
__device__ inline double buf_load(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, int(off), 0, 0));
}
__device__ inline void buf_store(__amdgpu_buffer_rsrc_t r, unsigned off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, int(off), 0, 0);
}

// Block-wide argmax of the threads' own candidates (v < 0: none); ties go to the
// lowest row, and no candidate that is a number gives INT_MAX, as block_argmax.
__device__ int block_argmax_own(double v, int idx, double* red_v, int* red_i) {
    double bv = -1.0;
    int bi = INT_MAX;
    if (v >= 0.0 || v != v) arg_better(bv, bi, v, idx);  // a NaN candidate never wins, as there
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
        double v0 = red_v[0];
        int i0 = red_i[0];
        for (int w = 1; w < int(blockDim.x >> 6); ++w) arg_better(v0, i0, red_v[w], red_i[w]);
        red_i[0] = i0;
    }
    __syncthreads();
    const int p = red_i[0];
    __syncthreads();
    return p;
}

// The panel elimination for sub-circuits of up to blockDim.x (at most
// kPanelBlock) nodes, one workgroup per sub-circuit, with row i of the panel in
// thread i's registers.  Column by column: the pivot search (ties to the lowest
// row), rows k and p trade places through LDS, the pivot row is scaled and
// published in LDS, and every other row updates itself.  No panel in LDS, so
// several workgroups share a CU.  Each thread keeps its row rotated: at step kk
// register slot t holds panel column (t + kk) mod NB, so the step's column is
// always slot 0, every register index is fixed at compile time, and the row
// turns by one slot per step (the pivot row is published in the same slot
// order).  The pivot search is first one ballot per wavefront: the diagonal is
// the pivot when it is a number and no row below holds a larger entry, which is
// what the full search (run otherwise) would find.
template <int NB>
__global__ void __launch_bounds__(kPanelBlock)
    k_gj_panel_reg(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs, double* __restrict__ base,
                   int k0, double* __restrict__ panel, int32_t* __restrict__ ipiv, int* flag) {
    static_assert((NB & (NB - 1)) == 0, "the rotation wraps by masking");
    __shared__ double red_v[kPanelBlock / 64];
    __shared__ int red_i[kPanelBlock / 64];
    __shared__ int any_w[kPanelBlock / 64];
    __shared__ double prow[NB], xrow[NB], pv_s;
    const int s = blockIdx.x;
    const int off = sub_off[s], n = sub_off[s + 1] - off;
    if (n <= kLdsSetupMax || k0 >= n || n > int(blockDim.x)) return;  // uniform over the workgroup
    const int kb = min(NB, n - k0);
    double* M = base + kofs[s];
    double* slot = panel + int64_t(off) * panel_stride(NB);  // E_J column-major: entry (i, jj) at jj n + i
    const int i = threadIdx.x;
    const bool mine = i < n;
    const int nw = int(blockDim.x) >> 6;
    double row[NB];
#pragma unroll
    for (int jj = 0; jj < NB; ++jj) row[jj] = (mine && jj < kb) ? M[int64_t(i) * n + k0 + jj] : 0.0;
    bool bad = false;
    for (int kk = 0; kk < kb; ++kk) {
        const int k = k0 + kk;
        // the diagonal, then one ballot per wavefront for a larger entry below it
        if (i == k) pv_s = row[0];
        __syncthreads();
        const double d = fabs(pv_s);
        const unsigned long long big = __ballot(mine && i > k && fabs(row[0]) > d);
        if ((i & 63) == 0) any_w[i >> 6] = big != 0ull;
        __syncthreads();
        bool search = !(d >= 0.0);  // a diagonal that is not a number never wins
        for (int w = 0; w < nw; ++w) search = search || any_w[w] != 0;
        int p = k;
        if (search) {  // uniform
            p = block_argmax_own(mine && i >= k ? fabs(row[0]) : -1.0, i, red_v, red_i);
            if (p == INT_MAX) {
                bad = true;
                p = k;
            }
        }
        if (i == 0) ipiv[off + k] = p;
        if (p != k) {  // uniform: rows k and p trade places through LDS
            if (i == k)
#pragma unroll
                for (int jj = 0; jj < NB; ++jj) prow[jj] = row[jj];
            if (i == p)
#pragma unroll
                for (int jj = 0; jj < NB; ++jj) xrow[jj] = row[jj];
            __syncthreads();
            if (i == k)
#pragma unroll
                for (int jj = 0; jj < NB; ++jj) row[jj] = xrow[jj];
            if (i == p)
#pragma unroll
                for (int jj = 0; jj < NB; ++jj) row[jj] = prow[jj];
            __syncthreads();
            if (i == k) pv_s = row[0];
            __syncthreads();
        }
        double pv = pv_s;
        if (pv == 0.0 || !isfinite(pv)) {
            bad = true;
            pv = 1.0;
        }
        // the pivot row scaled (its own column becomes 1 / pv), each slot written
        // back one slot lower (the turn for the next step)
        if (i == k) {
            prow[0] = 1.0 / pv;
#pragma unroll
            for (int t = 1; t < NB; ++t) {
                prow[t] = row[t] / pv;
                row[t - 1] = prow[t];
            }
            row[NB - 1] = prow[0];
        }
        __syncthreads();
        if (mine && i != k) {
            const double f = row[0];
#pragma unroll
            for (int t = 1; t < NB; ++t) row[t - 1] = row[t] - f * prow[t];
            row[NB - 1] = 0.0 - f * prow[0];
        }
    }
    // the panel's columns are final for this step; k_gj_update reads them from the slot.
    // After kb steps slot t holds column (t + kb) mod NB.
    if (mine)
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            const int jj = (t + kb) & (NB - 1);
            if (jj < kb) {
                M[int64_t(i) * n + k0 + jj] = row[t];
                slot[int64_t(jj) * n + i] = row[t];
            }
        }
    if (bad && i == 0) atomicOr(flag, 1);
}

// The same panel elimination for a few very large sub-circuits, where one
// workgroup's chain of pivot steps over n rows is the setup's bottleneck: each
// step is two launches, the pivot (search, row swap, scaling of the pivot row;
// one workgroup per sub-circuit) and the elimination of every other row of the
// panel (one row per thread over a grid of row blocks, column by column, so the
// loads of a wavefront are contiguous).  k_gjw_load moves the panel between K
// and the panel buffer (store = 1: back into K).
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
    double* E = panel + int64_t(off) * panel_stride(NB) + i;
    for (int jj = 0; jj < kb; ++jj) {
        if (store)
            M[jj] = E[int64_t(jj) * n];
        else
            E[int64_t(jj) * n] = M[jj];
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
    double* E = panel + int64_t(off) * panel_stride(NB);
    const int tid = threadIdx.x, bs = blockDim.x;
    int p = block_argmax(E + int64_t(kk) * n, 1, k, n, red_v, red_i);
    bool bad = false;
    if (p == INT_MAX) {
        bad = true;
        p = k;
    }
    if (tid == 0) ipiv[off + k] = p;
    if (p != k)
        for (int jj = tid; jj < kb; jj += bs) {
            const double t = E[int64_t(jj) * n + k];
            E[int64_t(jj) * n + k] = E[int64_t(jj) * n + p];
            E[int64_t(jj) * n + p] = t;
        }
    __syncthreads();
    double pv = E[int64_t(kk) * n + k];
    if (pv == 0.0 || !isfinite(pv)) {
        bad = true;
        pv = 1.0;
    }
    __syncthreads();  // every thread has read the pivot before row k is scaled
    for (int jj = tid; jj < kb; jj += bs) E[int64_t(jj) * n + k] = (jj == kk ? 1.0 : E[int64_t(jj) * n + k]) / pv;
    if (bad && tid == 0) atomicOr(flag, 1);
}

// Row i of the panel (every row but the pivot row k): its kb entries and the
// pivot row's are all loaded before the first store (the panel is read and
// written through one pointer, so loads and stores interleaved in a loop would
// wait on each other), then E[i][jj] <- E[i][jj] - E[i][kk] E[k][jj] with the
// pivot column itself replaced by -E[i][kk] E[k][kk].
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
    double* E = panel + int64_t(off) * panel_stride(NB);
    const auto rE = buf(E, int64_t(NB) * n);
    double row[NB], piv[NB];
#pragma unroll
    for (int jj = 0; jj < NB; ++jj) {
        row[jj] = buf_load(rE, jj < kb ? unsigned(jj * n + i) * 8u : kOffOut);
        piv[jj] = buf_load(rE, jj < kb ? unsigned(jj * n + k) * 8u : kOffOut);
    }
    const double f = buf_load(rE, unsigned(kk * n + i) * 8u);
#pragma unroll
    for (int jj = 0; jj < NB; ++jj)
        buf_store(rE, jj < kb ? unsigned(jj * n + i) * 8u : kOffOut, (jj == kk ? 0.0 : row[jj]) - f * piv[jj]);
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
    double* R = panel + int64_t(off) * panel_stride(NB) + int64_t(n) * NB;
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

// The rank-kb update of every column outside the panel on v_mfma_f64_16x16x4f64:
// a workgroup takes kUpdRows rows x 16 CT columns, its wavefronts every fourth
// 16-row tile.  The NB panel columns are spread over the MFMA's four k slots: in
// step q (of NB / 4), slot g = lane / 16 carries panel column g NB / 4 + q.  A
// lane holds the A operand E_J[row][g NB / 4 + q] - I_J (row lane % 16 of the
// tile; the column-major panel makes each step's load four 128-byte segments),
// the B operand (P R)_J[g NB / 4 + q][column] for its CT column tiles (loaded
// once), and the accumulators, which are the entries of R themselves (row 4 v + g
// of the tile, column lane % 16), loaded and stored as four 128-byte row
// segments per instruction.  Masked lanes use out-of-range buffer offsets, so no
// load or store sits behind a branch and the next tile's loads, issued before
// this tile's MFMAs, stay in flight while they run.  Columns of the panel are
// left as the panel elimination wrote them.
template <int NB, int CT>
__global__ void __launch_bounds__(kUpdWaves * 64)
    k_gj_update(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs, double* __restrict__ base,
                int k0, const double* __restrict__ panel, int S, int ncb) {
    constexpr int Q = NB / 4;  // MFMA steps
    // one-dimensional grid over (row block, sub-circuit) pairs t and column blocks cb:
    // the column blocks of one pair, which read the same rows of its panel, run one
    // after another on one XCD (so those rows come from its L2), and consecutive pairs
    // go to different XCDs, so that a run of large sub-circuits spreads over the chip.
    // Blocks are dealt round-robin to the 8 XCDs: XCD b % 8 takes pairs t = 8 i + b % 8.
    const int x = int(blockIdx.x) & 7, j = int(blockIdx.x) >> 3;
    const int cb = j % ncb, t = (j / ncb) * 8 + x;
    const int s = t % S, rb = t / S;  // rb past the last row block: r0 >= n below
    const int off = sub_off[s], n = sub_off[s + 1] - off;
    if (n <= kLdsSetupMax || k0 >= n || n > kMaxLarge) return;
    const int kb = min(NB, n - k0);
    const int c0 = cb * (16 * CT), r0 = rb * kUpdRows;
    if (c0 >= n || r0 >= n) return;
    const int r1 = min(n, r0 + kUpdRows);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, l16 = lane & 15;
    const double* E = panel + int64_t(off) * panel_stride(NB);
    const auto rE = buf(E, int64_t(NB) * n), rR = buf(E + int64_t(n) * NB, int64_t(NB) * n);
    const auto rM = buf(base + kofs[s], int64_t(n) * n);
    double b[CT][Q];
    unsigned mcol[CT], scol[CT];  // byte offset of the lane's column in row 0: loads, stores
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        const int c = c0 + 16 * t + l16;
        mcol[t] = c < n ? unsigned(c) * 8u : kOffOut;
        scol[t] = (c < n && (c < k0 || c >= k0 + kb)) ? mcol[t] : kOffOut;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int kk = g * Q + q;
            b[t][q] = buf_load(rR, (kk < kb && c < n) ? unsigned(kk * n + c) * 8u : kOffOut);
        }
    }
    const unsigned rowb = unsigned(n) * 8u;  // bytes per row of R
    // byte offset of row i (or kOffOut past r1), to be added to a column offset
    // that is itself kOffOut when masked (any sum with kOffOut stays out of range)
    auto row_off = [&](int i) { return i < r1 ? unsigned(i) * rowb : kOffOut; };
    auto load = [&](int i0, double (&a)[Q], dx4 (&acc)[CT]) {
        const int ia = i0 + l16;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int kk = g * Q + q;
            const bool ok = ia < r1 && kk < kb;
            const double e = buf_load(rE, ok ? unsigned(kk * n + ia) * 8u : kOffOut);
            a[q] = ok && ia == k0 + kk ? e - 1.0 : e;
        }
#pragma unroll
        for (int t = 0; t < CT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const unsigned ro = row_off(i0 + g + 4 * v);
                acc[t][v] = buf_load(rM, (ro | mcol[t]) >= kOffOut ? kOffOut : ro + mcol[t]);
            }
    };
    auto update = [&](int i0, const double (&a)[Q], dx4 (&acc)[CT]) {
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int t = 0; t < CT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[t][q], acc[t], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < CT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const unsigned ro = row_off(i0 + g + 4 * v);
                buf_store(rM, (ro | scol[t]) >= kOffOut ? kOffOut : ro + scol[t], acc[t][v]);
            }
    };
    // two register sets, alternating: tile j + 1 is loading while tile j computes
    constexpr int step = 16 * kUpdWaves;
    double a0[Q], a1[Q];
    dx4 m0[CT], m1[CT];
    int i0 = r0 + 16 * wave;
    if (i0 >= r1) return;
    load(i0, a0, m0);
    for (;;) {
        const int i1 = i0 + step;
        load(i1, a1, m1);  // every lane out of range past r1
        update(i0, a0, m0);
        if (i1 >= r1) break;
        const int i2 = i1 + step;
        load(i2, a0, m0);
        update(i1, a1, m1);
        if (i2 >= r1) break;
        i0 = i2;
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

template <int NB>
hipError_t launch_update(int S, int max_ns, const int32_t* sub_off, const int64_t* kofs, double* scratch64, int k0,
                         const double* panel, hipStream_t st) {
    constexpr int CT = 4;  // column tiles per wavefront (the B operand stays in registers)
    const int ncb = (max_ns + 16 * CT - 1) / (16 * CT), nrb = (max_ns + kUpdRows - 1) / kUpdRows;
    const int64_t blocks = 8 * int64_t(ncb) * ((int64_t(S) * nrb + 7) / 8);
    if (blocks > INT_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_gj_update<NB, CT>), dim3(unsigned(blocks)), dim3(kUpdWaves * 64), 0, st, sub_off, kofs,
                       scratch64, k0, panel, S, ncb);
    return hipGetLastError();
}

// panels eliminated by one workgroup per sub-circuit (max_ns <= kPanelBlock), a
// row per thread in registers, as many threads as the largest sub-circuit has
// rows (smaller workgroups reduce faster and share a CU)
template <int NB>
hipError_t invert_panels(int S, int max_ns, const int32_t* sub_off, const int64_t* kofs, double* scratch64,
                         double* panel, int32_t* ipiv, int* flag, hipStream_t st) {
    if (max_ns > kPanelBlock) return hipErrorInvalidValue;
    const dim3 cols(unsigned(S), unsigned((max_ns + kBlock - 1) / kBlock));
    hipError_t e;
    const unsigned reg_threads = unsigned((max_ns + 63) / 64 * 64);
    for (int k0 = 0; k0 < max_ns; k0 += NB) {
        hipLaunchKernelGGL(k_gj_panel_reg<NB>, dim3(S), dim3(reg_threads), 0, st, sub_off, kofs, scratch64, k0,
                           panel, ipiv, flag);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_gj_swap<NB>, cols, dim3(kBlock), 0, st, sub_off, kofs, scratch64, k0, panel, ipiv);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = launch_update<NB>(S, max_ns, sub_off, kofs, scratch64, k0, panel, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// panels whose pivot steps are launches of their own, spread over the chip
template <int NB>
hipError_t invert_wide(int S, int max_ns, const int32_t* sub_off, const int64_t* kofs, double* scratch64,
                       double* panel, int32_t* ipiv, int* flag, hipStream_t st) {
    const dim3 cols(unsigned(S), unsigned((max_ns + kBlock - 1) / kBlock));
    hipError_t e;
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
        if ((e = launch_update<NB>(S, max_ns, sub_off, kofs, scratch64, k0, panel, st)) != hipSuccess) return e;
    }
    return hipSuccess;
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
    // larger sub-circuits, or a few, spread each pivot step over the chip (two launches per column)
    if (max_ns <= kPanelBlock && S >= kOneGroupMinSubs)
        e = invert_panels<kNB>(S, max_ns, sub_off, kofs, scratch64, panel, ipiv, flag, st);
    else if (max_ns < kWide64)
        e = invert_wide<kNB>(S, max_ns, sub_off, kofs, scratch64, panel, ipiv, flag, st);
    else
        e = invert_wide<kWideNB>(S, max_ns, sub_off, kofs, scratch64, panel, ipiv, flag, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gj_unscramble, cols, dim3(kBlock), 0, st, sub_off, kofs, scratch64, ipiv);
    return hipGetLastError();
}

}  // namespace

int64_t setup_panel_doubles(int64_t n, int max_ns) {
    if (max_ns <= kLdsSetupMax) return 0;
    return n * panel_stride(max_ns < kWide64 ? kNB : kWideNB);
}

template <typename T>
hipError_t launch_setup_tiles(int S, int max_ns, const int32_t* sub_off, const int64_t* kofs, const int64_t* mofs,
                              const int32_t* rowptr, const int32_t* col, const double* val, const double* dmod,
                              T* out, double* scratch64, double* panel, int32_t* ipiv, int* flag, hipStream_t st,
                              T* out_t) {
    if (!scratch64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_setup_reg<double, true>), dim3(S), dim3(64), 0, st, sub_off, kofs, rowptr, col, val, dmod,
                       scratch64, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (max_ns > kRegSetupMax) {
        hipLaunchKernelGGL((k_setup_lds<double, true>), dim3(S), dim3(kBlock), 0, st, sub_off, kofs, rowptr, col, val,
                           dmod, scratch64, flag);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
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
    hipLaunchKernelGGL((k_setup_reg<TO, false>), dim3(S), dim3(64), 0, st, sub_off, kofs, rowptr, col, val, dmod, out,
                       flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || max_ns <= kRegSetupMax) return e;
    hipLaunchKernelGGL((k_setup_lds<TO, false>), dim3(S), dim3(kBlock), 0, st, sub_off, kofs, rowptr, col, val,
                       dmod, out, flag);
    e = hipGetLastError();
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
