// FP64 residual of the untorn system, r = b - A x, with per-column sums of r^2
// and b^2 (the convergence test ||b - A x||_2 / ||b||_2 <= tol).  Sums are
// formed in a fixed order, so results are bitwise reproducible.
#include "kernels.hpp"
#include "layout.hpp"

namespace vtm {

namespace {

constexpr int kBlock = 256;

// One row of b - A x with every load of the row issued before the first use:
// the NZ column indices and values (scalar loads when the row is wave-uniform),
// then the NZ gathers of x, then the subtractions in the row's order (the same
// arithmetic as a loop over the row, which would wait on each gather in turn).
template <int NZ, typename TX>
__device__ inline double row_residual(double bv, int k0, const int32_t* __restrict__ col,
                                      const double* __restrict__ val, const TX* __restrict__ x, int nrhs, int rhs) {
    int c[NZ];
    double v[NZ];
    TX xv[NZ];
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
        c[j] = col[k0 + j];
        v[j] = val[k0 + j];
    }
#pragma unroll
    for (int j = 0; j < NZ; ++j) xv[j] = x[int64_t(c[j]) * nrhs + rhs];
    double acc = bv;
#pragma unroll
    for (int j = 0; j < NZ; ++j) acc -= v[j] * double(xv[j]);
    return acc;
}

// thread (row slot, rhs): the block's threads cover per = 256 / nrhs rows at a time.
// UNI (nrhs a multiple of 64): each wavefront holds whole rows of one row slot, so
// the row index is wave-uniform and the row's index and value loads are scalar
// loads, issued once per wavefront instead of once per lane.
template <typename TX, bool UNI>
__global__ void __launch_bounds__(kBlock)
    k_resid(int n, int nrhs, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
            const double* __restrict__ val, const double* __restrict__ b, const TX* __restrict__ x,
            double* __restrict__ r_out, float* __restrict__ r32, __bf16* __restrict__ r16,
            double* __restrict__ partial) {
    __shared__ double s_rr[kBlock], s_bb[kBlock];
    const int tid = threadIdx.x;
    const int per = blockDim.x / nrhs;
    const int used = per * nrhs;
    double rr = 0.0, bb = 0.0;
    // each XCD takes one contiguous range of logical blocks, so that rows whose x
    // rows overlap share an L2; a logical block's rows and partial sums are the
    // same whichever hardware block runs it
    const int lb = xcd_block(int(blockIdx.x), int(gridDim.x));
    if (tid < used) {
        const int rhs = tid % nrhs, rl = tid / nrhs;
        int i0 = lb * per + rl;
        if (UNI) i0 = __builtin_amdgcn_readfirstlane(i0);
        for (int64_t i = i0; i < n; i += int64_t(gridDim.x) * per) {
            const double bv = b[i * nrhs + rhs];
            const int k0 = rowptr[i], nz = rowptr[i + 1] - k0;
            double acc;
            // UNI: nz is wave-uniform, so this branch is a scalar one
            if (UNI && nz == 5)
                acc = row_residual<5>(bv, k0, col, val, x, nrhs, rhs);
            else if (UNI && nz == 7)
                acc = row_residual<7>(bv, k0, col, val, x, nrhs, rhs);
            else if (UNI && nz == 4)
                acc = row_residual<4>(bv, k0, col, val, x, nrhs, rhs);
            else if (UNI && nz == 3)
                acc = row_residual<3>(bv, k0, col, val, x, nrhs, rhs);
            else if (UNI && nz == 6)
                acc = row_residual<6>(bv, k0, col, val, x, nrhs, rhs);
            else {
                acc = bv;
                for (int k = k0; k < k0 + nz; ++k) acc -= val[k] * double(x[int64_t(col[k]) * nrhs + rhs]);
            }
            if (r_out) r_out[i * nrhs + rhs] = acc;
            // the low-precision copies round as a separate cast pass would: via FP32
            if (r32) r32[i * nrhs + rhs] = static_cast<float>(acc);
            if (r16) r16[i * nrhs + rhs] = static_cast<__bf16>(static_cast<float>(acc));
            rr += acc * acc;
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
        partial[(int64_t(lb) * nrhs + j) * 2 + 0] = a;
        partial[(int64_t(lb) * nrhs + j) * 2 + 1] = c;
    }
}

// one block per output value: strided partial sums, then a fixed-shape tree
__global__ void __launch_bounds__(kBlock)
    k_norms_final(int nblocks, int nrhs, const double* __restrict__ partial, double* __restrict__ norms) {
    __shared__ double s[kBlock];
    const int j = blockIdx.x;
    const int tid = threadIdx.x;
    double a = 0.0;
    for (int q = tid; q < nblocks; q += blockDim.x) a += partial[int64_t(q) * nrhs * 2 + j];
    s[tid] = a;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (tid < h) s[tid] += s[tid + h];
        __syncthreads();
    }
    if (tid == 0) norms[j] = s[0];
}

// b - A x of a sweep's iterate from port quantities alone (a local solve meets
// every interior row exactly; A couples sub-circuits only through cut wires):
// per port node n, r_n = sum over its ports p of (G_p - g_p) x_n + g_p x_j(p)
// - c_p a_p, where x_n = (o_p0 - gamma_p0 a_p0) / beta_p0 from its first port,
// x_j(p) likewise from the twin port q, and the outgoing wave o_p of port p is
// a_next[twin(p)].  Waves are [ports][nrhs]; thread (node slot, rhs) as in
// k_resid, partial sums per column in the same layout.
template <typename TV, bool UNI>
__global__ void __launch_bounds__(kBlock)
    k_port_resid(int64_t nn, int nrhs, const int32_t* __restrict__ pn_pfirst, const int32_t* __restrict__ twin,
                 const TV* __restrict__ a_cur, const TV* __restrict__ a_next, const double* __restrict__ c,
                 const double* __restrict__ beta, const double* __restrict__ gamma, const double* __restrict__ gd,
                 const double* __restrict__ g, double* __restrict__ partial) {
    __shared__ double s_rr[kBlock];
    const int tid = threadIdx.x;
    const int per = blockDim.x / nrhs;
    const int used = per * nrhs;
    double rr = 0.0;
    // (blocks in dispatch order: the XCD-contiguous order of k_resid measured
    // slower here, the twins' gathers then crowd one L2)
    if (tid < used) {
        const int rhs = tid % nrhs, rl = tid / nrhs;
        int n0 = blockIdx.x * per + rl;
        if (UNI) n0 = __builtin_amdgcn_readfirstlane(n0);  // as in k_resid
        for (int64_t n = n0; n < nn; n += int64_t(gridDim.x) * per) {
            const int p0 = pn_pfirst[n], p1 = pn_pfirst[n + 1];
            const double xn =
                (double(a_next[int64_t(twin[p0]) * nrhs + rhs]) - gamma[p0] * double(a_cur[int64_t(p0) * nrhs + rhs])) /
                beta[p0];
            double r = 0.0;
            for (int p = p0; p < p1; ++p) {
                const int q = twin[p];
                const double xj =
                    (double(a_next[int64_t(p) * nrhs + rhs]) - gamma[q] * double(a_cur[int64_t(q) * nrhs + rhs])) /
                    beta[q];
                r += gd[p] * xn + g[p] * xj - c[p] * double(a_cur[int64_t(p) * nrhs + rhs]);
            }
            rr += r * r;
        }
    }
    s_rr[tid] = rr;
    __syncthreads();
    for (int j = tid; j < nrhs; j += blockDim.x) {
        double a = 0.0;
        for (int q = 0; q < per; ++q) a += s_rr[q * nrhs + j];
        partial[(int64_t(blockIdx.x) * nrhs + j) * 2 + 0] = a;
        partial[(int64_t(blockIdx.x) * nrhs + j) * 2 + 1] = 0.0;
    }
}

}  // namespace

template <typename TV>
hipError_t launch_port_residual(int64_t n_port_nodes, int nrhs, const int32_t* pn_pfirst, const int32_t* twin,
                                const TV* a_cur, const TV* a_next, const double* c, const double* beta,
                                const double* gamma, const double* gd, const double* g, double* partial, double* norms,
                                hipStream_t st) {
    if (nrhs < 1 || nrhs > kBlock) return hipErrorInvalidValue;
    const int blocks = resid_blocks(n_port_nodes, nrhs);
    if (nrhs % 64 == 0)
        hipLaunchKernelGGL((k_port_resid<TV, true>), dim3(blocks), dim3(kBlock), 0, st, n_port_nodes, nrhs, pn_pfirst,
                           twin, a_cur, a_next, c, beta, gamma, gd, g, partial);
    else
        hipLaunchKernelGGL((k_port_resid<TV, false>), dim3(blocks), dim3(kBlock), 0, st, n_port_nodes, nrhs,
                           pn_pfirst, twin, a_cur, a_next, c, beta, gamma, gd, g, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_norms_final, dim3(2 * nrhs), dim3(kBlock), 0, st, blocks, nrhs, partial, norms);
    return hipGetLastError();
}

template hipError_t launch_port_residual<double>(int64_t, int, const int32_t*, const int32_t*, const double*,
                                                 const double*, const double*, const double*, const double*,
                                                 const double*, const double*, double*, double*, hipStream_t);
template hipError_t launch_port_residual<float>(int64_t, int, const int32_t*, const int32_t*, const float*, const float*,
                                                const double*, const double*, const double*, const double*,
                                                const double*, double*, double*, hipStream_t);

template <typename TX>
hipError_t launch_residual(int n, int nrhs, const int32_t* rowptr, const int32_t* col, const double* val,
                           const double* b, const TX* x, double* r_out, float* r32, __bf16* r16, double* partial,
                           double* norms, hipStream_t st) {
    if (nrhs < 1 || nrhs > kBlock) return hipErrorInvalidValue;
    const int blocks = resid_blocks(n, nrhs);
    if (nrhs % 64 == 0)
        hipLaunchKernelGGL((k_resid<TX, true>), dim3(blocks), dim3(kBlock), 0, st, n, nrhs, rowptr, col, val, b, x,
                           r_out, r32, r16, partial);
    else
        hipLaunchKernelGGL((k_resid<TX, false>), dim3(blocks), dim3(kBlock), 0, st, n, nrhs, rowptr, col, val, b, x,
                           r_out, r32, r16, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_norms_final, dim3(2 * nrhs), dim3(kBlock), 0, st, blocks, nrhs, partial, norms);
    return hipGetLastError();
}

template hipError_t launch_residual<double>(int, int, const int32_t*, const int32_t*, const double*, const double*,
                                            const double*, double*, float*, __bf16*, double*, double*, hipStream_t);
template hipError_t launch_residual<float>(int, int, const int32_t*, const int32_t*, const double*, const double*,
                                           const float*, double*, float*, __bf16*, double*, double*, hipStream_t);

}  // namespace vtm
