// HIP kernels of the VTM hot path for gfx950 (CDNA4, 64-wide wavefronts).
//
//   setup     : forms every sub-circuit's tearing-modified matrix and inverts it
//               (Gauss-Jordan with partial pivoting; in LDS when it fits).
//   sweep     : per sub-circuit, the local solve of eq. 11 as a dense GEMV
//               with the stored inverse, fused with the wave update of eq. 11's
//               second line and the exchange to the twin port.
//   residual  : FP64 r = b - A x on the untorn matrix with per-column sums of
//               squares in a fixed order (bitwise reproducible).
#include "kernels.hpp"

#include <climits>

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
__device__ int block_argmax(const double* colp, int stride, int lo, int n, double* red_v,
                            int* red_i) {
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

template <typename T>
__device__ inline T to(double v) {
    return T(v);
}

// ---------------------------------------------------------------------------
// Setup, LDS path: one workgroup per sub-circuit with ns <= kLdsSetupMax.
// M holds K^T row-major, so the in-place inverse is K^-1 column-major.
// ---------------------------------------------------------------------------
template <typename TO>
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
    TO* o = out + kofs[s];
    for (int t = tid; t < n * n; t += bs) o[t] = to<TO>(M[t]);
    if (bad && tid == 0) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// Setup, global path (ns > kLdsSetupMax): assemble K^T into FP64 scratch ...
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

// ... and invert it in place, NB columns at a time.  The panel is eliminated in
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

template <typename TO>
__global__ void __launch_bounds__(kBlock)
    k_copy_large(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs,
                 const double* __restrict__ src, TO* __restrict__ dst) {
    const int s = blockIdx.x;
    const int n = sub_off[s + 1] - sub_off[s];
    if (n <= kLdsSetupMax) return;
    const int64_t o = kofs[s], cnt = int64_t(n) * n;
    for (int64_t t = threadIdx.x; t < cnt; t += blockDim.x) dst[o + t] = to<TO>(src[o + t]);
}

// ---------------------------------------------------------------------------
// Sweep: one workgroup per sub-circuit.
// ---------------------------------------------------------------------------
template <typename TO, typename TV>
__global__ void __launch_bounds__(kBlock)
    k_sweep(const TO* __restrict__ K, const int64_t* __restrict__ kofs,
            const int32_t* __restrict__ sub_off, const int32_t* __restrict__ port_off,
            const int32_t* __restrict__ port_node, const int32_t* __restrict__ port_slot,
            const int32_t* __restrict__ port_twin, const TV* __restrict__ pc,
            const TV* __restrict__ pbeta, const TV* __restrict__ pgamma, const TV* __restrict__ b,
            const TV* __restrict__ a_cur, TV* __restrict__ a_next, TV* __restrict__ x, int nrhs, int rc,
            int max_ns, int max_slot, int adjoint) {
    // block (s, y): sub-circuit s, right-hand sides [r0, r0 + w)
    extern __shared__ char smem[];
    TV* rhs = reinterpret_cast<TV*>(smem);
    TV* xs = rhs + max_ns * rc;
    const int s = blockIdx.x;
    const int r0 = blockIdx.y * rc;
    const int w = min(rc, nrhs - r0);
    const int off = sub_off[s];
    const int ns = sub_off[s + 1] - off;
    const int p0 = port_off[s], p1 = port_off[s + 1];
    const int tid = threadIdx.x, bs = blockDim.x;
    const int nv = ns * w;

    for (int t = tid; t < nv; t += bs) {
        const int row = t / w, rr = t - row * w;
        rhs[t] = b[int64_t(off + row) * nrhs + r0 + rr];
    }
    __syncthreads();
    // incident waves enter at the port nodes: rhs += c * a (ports of one node in slot order)
    for (int pb = p0; pb < p1; pb += bs) {
        const int p = pb + tid;
        const bool ok = p < p1;
        const int node = ok ? port_node[p] : 0;
        const int slot = ok ? port_slot[p] : -1;
        const TV c = ok ? pc[p] : TV(0);
        for (int sl = 0; sl <= max_slot; ++sl) {
            if (slot == sl)
                for (int r = 0; r < w; ++r) rhs[node * w + r] += c * a_cur[int64_t(p) * nrhs + r0 + r];
            __syncthreads();
        }
    }
    // local solve x = K^-1 rhs (K^-T for the adjoint), inverse stored column-major
    const TO* Ks = K + kofs[s];
    for (int t = tid; t < nv; t += bs) {
        const int row = t / w, rr = t - row * w;
        TV a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        const int64_t step = adjoint ? 1 : ns;
        const TO* kp = adjoint ? Ks + int64_t(row) * ns : Ks + row;
        int c = 0;
        for (; c + 3 < ns; c += 4) {
            a0 += TV(kp[(c + 0) * step]) * rhs[(c + 0) * w + rr];
            a1 += TV(kp[(c + 1) * step]) * rhs[(c + 1) * w + rr];
            a2 += TV(kp[(c + 2) * step]) * rhs[(c + 2) * w + rr];
            a3 += TV(kp[(c + 3) * step]) * rhs[(c + 3) * w + rr];
        }
        for (; c < ns; ++c) a0 += TV(kp[c * step]) * rhs[c * w + rr];
        const TV v = (a0 + a1) + (a2 + a3);
        xs[t] = v;
        x[int64_t(off + row) * nrhs + r0 + rr] = v;
    }
    __syncthreads();
    // outgoing wave W u - i = beta * x + gamma * a, received by the twin next sweep
    for (int p = p0 + tid; p < p1; p += bs) {
        const int node = port_node[p];
        const int64_t tw = int64_t(port_twin[p]) * nrhs + r0;
        const int64_t pa = int64_t(p) * nrhs + r0;
        const TV be = pbeta[p], ga = pgamma[p];
        for (int r = 0; r < w; ++r) a_next[tw + r] = be * xs[node * w + r] + ga * a_cur[pa + r];
    }
}

// ---------------------------------------------------------------------------
// Residual
// ---------------------------------------------------------------------------
template <typename TX>
__global__ void __launch_bounds__(kBlock)
    k_resid(int n, int nrhs, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
            const double* __restrict__ val, const double* __restrict__ b, const TX* __restrict__ x,
            double* __restrict__ r_out, double* __restrict__ partial) {
    __shared__ double s_rr[kBlock], s_bb[kBlock];
    const int tid = threadIdx.x;
    const int per = blockDim.x / nrhs;
    const int used = per * nrhs;
    double rr = 0.0, bb = 0.0;
    if (tid < used) {
        const int rhs = tid % nrhs, rl = tid / nrhs;
        for (int64_t i = int64_t(blockIdx.x) * per + rl; i < n; i += int64_t(gridDim.x) * per) {
            const double bv = b[i * nrhs + rhs];
            double sacc = bv;
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
                sacc -= val[k] * double(x[int64_t(col[k]) * nrhs + rhs]);
            if (r_out) r_out[i * nrhs + rhs] = sacc;
            rr += sacc * sacc;
            bb += bv * bv;
        }
    }
    s_rr[tid] = rr;
    s_bb[tid] = bb;
    __syncthreads();
    for (int j = tid; j < nrhs; j += blockDim.x) {
        double a = 0.0, c = 0.0;
        for (int q = 0; q < per; ++q) {
            a += s_rr[q * nrhs + j];
            c += s_bb[q * nrhs + j];
        }
        partial[(int64_t(blockIdx.x) * nrhs + j) * 2 + 0] = a;
        partial[(int64_t(blockIdx.x) * nrhs + j) * 2 + 1] = c;
    }
}

__global__ void k_norms_final(int nblocks, int nrhs, const double* __restrict__ partial,
                              double* __restrict__ norms) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= 2 * nrhs) return;
    double a = 0.0;
    for (int q = 0; q < nblocks; ++q) a += partial[int64_t(q) * nrhs * 2 + j];
    norms[j] = a;
}

// ---------------------------------------------------------------------------
// Vector utilities
// ---------------------------------------------------------------------------
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

template <typename T>
__global__ void k_fill(int64_t count, T value, T* __restrict__ dst) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < count) dst[t] = value;
}

template <typename TS, typename TD>
__global__ void k_convert(int64_t count, const TS* __restrict__ src, TD* __restrict__ dst) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < count) dst[t] = TD(src[t]);
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

inline unsigned blocks_for(int64_t count, int bs = kBlock) { return unsigned((count + bs - 1) / bs); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <typename TO>
hipError_t launch_setup(int S, int max_ns, const int32_t* sub_off, const int64_t* kofs,
                        const int32_t* rowptr, const int32_t* col, const double* val,
                        const double* dmod, TO* out, double* scratch64, int* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_setup_lds<TO>, dim3(S), dim3(kBlock), 0, st, sub_off, kofs, rowptr, col, val,
                       dmod, out, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || max_ns <= kLdsSetupMax) return e;
    hipLaunchKernelGGL(k_assemble, dim3(S), dim3(kBlock), 0, st, sub_off, kofs, rowptr, col, val, dmod,
                       scratch64);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // panel width: as many columns as fit next to the pivot bookkeeping in 64 KiB of LDS
    constexpr int kLds = 65536;
    const int fixed = max_ns * (8 + 4) + 64;
    int nb = (kLds - fixed) / (8 * max_ns);
    if (nb < 1) return hipErrorInvalidValue;
    nb = nb > 16 ? 16 : nb;
    const size_t lds = size_t(max_ns) * nb * 8 + fixed;
    hipLaunchKernelGGL(k_gj_global<16>, dim3(S), dim3(kBlock), lds, st, sub_off, kofs, scratch64, nb, flag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (static_cast<void*>(scratch64) != static_cast<void*>(out)) {
        hipLaunchKernelGGL(k_copy_large<TO>, dim3(S), dim3(kBlock), 0, st, sub_off, kofs, scratch64, out);
        e = hipGetLastError();
    }
    return e;
}

template <typename TO, typename TV>
hipError_t launch_sweep(int S, int max_ns, int nrhs, const TO* K, const int64_t* kofs,
                        const int32_t* sub_off, PortArrays ports, const TV* pc, const TV* pbeta,
                        const TV* pgamma, const TV* b, const TV* a_cur, TV* a_next, TV* x, bool adjoint,
                        hipStream_t st) {
    // right-hand sides per block: rhs and x of the sub-circuit must fit 64 KiB of LDS
    int rc = int(65536 / (size_t(2) * max_ns * sizeof(TV)));
    if (rc < 1) return hipErrorInvalidValue;
    rc = rc > nrhs ? nrhs : rc;
    const int bs = (max_ns * rc <= 64) ? 64 : kBlock;
    const size_t lds = size_t(2) * max_ns * rc * sizeof(TV);
    const unsigned ny = unsigned((nrhs + rc - 1) / rc);
    hipLaunchKernelGGL((k_sweep<TO, TV>), dim3(S, ny), dim3(bs), lds, st, K, kofs, sub_off, ports.off,
                       ports.node, ports.slot, ports.twin, pc, pbeta, pgamma, b, a_cur, a_next, x, nrhs, rc,
                       max_ns, ports.max_slot, adjoint ? 1 : 0);
    return hipGetLastError();
}

template <typename TX>
hipError_t launch_residual(int n, int nrhs, const int32_t* rowptr, const int32_t* col, const double* val,
                           const double* b, const TX* x, double* r_out, double* partial, double* norms,
                           hipStream_t st) {
    if (nrhs > kBlock) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_resid<TX>, dim3(kResidBlocks), dim3(kBlock), 0, st, n, nrhs, rowptr, col, val, b, x,
                       r_out, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_norms_final, dim3(blocks_for(2 * nrhs, 64)), dim3(64), 0, st, kResidBlocks, nrhs,
                       partial, norms);
    return hipGetLastError();
}

hipError_t launch_gather(int n, int nrhs, const int32_t* perm, const double* src, double* dst,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(int64_t(n) * nrhs)), dim3(kBlock), 0, st, n, nrhs, perm, src,
                       dst);
    return hipGetLastError();
}

hipError_t launch_scatter(int n, int nrhs, const int32_t* iperm, const double* src, double* dst,
                          hipStream_t st) {
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

// explicit instantiations
template hipError_t launch_setup<double>(int, int, const int32_t*, const int64_t*, const int32_t*,
                                         const int32_t*, const double*, const double*, double*, double*,
                                         int*, hipStream_t);
template hipError_t launch_setup<float>(int, int, const int32_t*, const int64_t*, const int32_t*,
                                        const int32_t*, const double*, const double*, float*, double*, int*,
                                        hipStream_t);
template hipError_t launch_sweep<double, double>(int, int, int, const double*, const int64_t*,
                                                 const int32_t*, PortArrays, const double*, const double*,
                                                 const double*, const double*, const double*, double*,
                                                 double*, bool, hipStream_t);
template hipError_t launch_sweep<float, float>(int, int, int, const float*, const int64_t*, const int32_t*,
                                               PortArrays, const float*, const float*, const float*,
                                               const float*, const float*, float*, float*, bool, hipStream_t);
template hipError_t launch_residual<double>(int, int, const int32_t*, const int32_t*, const double*,
                                            const double*, const double*, double*, double*, double*,
                                            hipStream_t);
template hipError_t launch_residual<float>(int, int, const int32_t*, const int32_t*, const double*,
                                           const double*, const float*, double*, double*, double*,
                                           hipStream_t);
template hipError_t launch_fill<double>(int64_t, double, double*, hipStream_t);
template hipError_t launch_fill<float>(int64_t, float, float*, hipStream_t);
template hipError_t launch_convert<double, float>(int64_t, const double*, float*, hipStream_t);
template hipError_t launch_convert<float, double>(int64_t, const float*, double*, hipStream_t);
template hipError_t launch_add<float>(int64_t, const float*, double*, hipStream_t);
template hipError_t launch_add<double>(int64_t, const double*, double*, hipStream_t);
template hipError_t launch_waves_io<double>(int64_t, int, const int32_t*, double*, double*, bool, hipStream_t);
template hipError_t launch_waves_io<float>(int64_t, int, const int32_t*, float*, double*, bool, hipStream_t);

}  // namespace vtm
