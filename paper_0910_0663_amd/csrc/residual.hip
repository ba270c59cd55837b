// FP64 residual of the untorn system, r = b - A x, with per-column sums of r^2
// and b^2 (the convergence test ||b - A x||_2 / ||b||_2 <= tol).  Sums are
// formed in a fixed order, so results are bitwise reproducible.
#include "kernels.hpp"

namespace vtm {

namespace {

constexpr int kBlock = 256;

// thread (row slot, rhs): the block's threads cover per = 256 / nrhs rows at a time
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
            double acc = bv;
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) acc -= val[k] * double(x[int64_t(col[k]) * nrhs + rhs]);
            if (r_out) r_out[i * nrhs + rhs] = acc;
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
        partial[(int64_t(blockIdx.x) * nrhs + j) * 2 + 0] = a;
        partial[(int64_t(blockIdx.x) * nrhs + j) * 2 + 1] = c;
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

}  // namespace

template <typename TX>
hipError_t launch_residual(int n, int nrhs, const int32_t* rowptr, const int32_t* col, const double* val,
                           const double* b, const TX* x, double* r_out, double* partial, double* norms,
                           hipStream_t st) {
    if (nrhs < 1 || nrhs > kBlock) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_resid<TX>, dim3(kResidBlocks), dim3(kBlock), 0, st, n, nrhs, rowptr, col, val, b, x, r_out,
                       partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_norms_final, dim3(2 * nrhs), dim3(kBlock), 0, st, kResidBlocks, nrhs, partial, norms);
    return hipGetLastError();
}

template hipError_t launch_residual<double>(int, int, const int32_t*, const int32_t*, const double*, const double*,
                                            const double*, double*, double*, double*, hipStream_t);
template hipError_t launch_residual<float>(int, int, const int32_t*, const int32_t*, const double*, const double*,
                                           const float*, double*, double*, double*, hipStream_t);

}  // namespace vtm
