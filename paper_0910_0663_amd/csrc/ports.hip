// Port-to-port form of the sweep (the interface-only iteration of the
// Appendix, eqs. 23-26, written for the eliminated twins).
//
// With the incident waves a_s at the q ports of sub-circuit s and
// x = K^-1 (b + sum_p c_p a_p e_i(p)), the outgoing waves are
//     o_p = beta_p x_i(p) + gamma_p a_p = h_p + sum_p' M_pp' a_p'
// with M = diag(beta) K^-1[i(P), i(P)] diag(c) + diag(gamma) and
// h = beta (K^-1 b)[i(P)].  A sweep then streams the q x q operator M instead
// of the n x n inverse; x itself is rebuilt by a full sweep where needed.
#include "kernels.hpp"
#include "layout.hpp"

namespace vtm {

namespace {

constexpr int kBlock = 256;

// M_s in the column-group layout (n = q), from the stored inverse K_s
template <typename TO>
__global__ void __launch_bounds__(kBlock)
    k_port_matrix(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs,
                  const int32_t* __restrict__ port_off, const int32_t* __restrict__ port_node,
                  const double* __restrict__ pc, const double* __restrict__ pbeta, const double* __restrict__ pgamma,
                  const TO* __restrict__ K, const int64_t* __restrict__ pofs, TO* __restrict__ M) {
    const int s = blockIdx.x;
    const int ns = sub_off[s + 1] - sub_off[s];
    const int p0 = port_off[s], q = port_off[s + 1] - p0;
    const TO* Ks = K + kofs[s];
    TO* Ms = M + pofs[s];
    const int64_t cnt = int64_t(q) * q;
    for (int64_t d = threadIdx.x; d < cnt; d += blockDim.x) {
        int r, c;
        inv_rc<TO>(q, d, r, c);
        const int pr = p0 + r, pcol = p0 + c;
        double v = pbeta[pr] * double(Ks[inv_offset<TO>(ns, port_node[pr], port_node[pcol])]) * pc[pcol];
        if (r == c) v += pgamma[pr];
        Ms[d] = TO(v);
    }
}

// h_p = beta_p x_i(p) for x = K^-1 b (one right-hand side)
template <typename TV>
__global__ void __launch_bounds__(kBlock)
    k_port_h(int S, const int32_t* __restrict__ sub_off, const int32_t* __restrict__ port_off,
             const int32_t* __restrict__ port_node, const TV* __restrict__ pbeta, const TV* __restrict__ x,
             TV* __restrict__ h) {
    const int s = blockIdx.x;
    const int off = sub_off[s];
    for (int p = port_off[s] + threadIdx.x; p < port_off[s + 1]; p += blockDim.x)
        h[p] = pbeta[p] * x[off + port_node[p]];
}

template <typename T>
__device__ inline void load16p(const T* p, T (&v)[Group<T>::G]) {
    if constexpr (sizeof(T) == 8) {
        const double2 w = *reinterpret_cast<const double2*>(p);
        v[0] = w.x;
        v[1] = w.y;
    } else {
        const float4 w = *reinterpret_cast<const float4*>(p);
        v[0] = w.x;
        v[1] = w.y;
        v[2] = w.z;
        v[3] = w.w;
    }
}

// One port-to-port sweep, one workgroup per sub-circuit (a_next[twin(p)] =
// h_p + (M a)_p).  SPLIT = 2 (q <= 32, one wavefront): lane l takes row l % 32
// and half the column groups, and the halves are added with a cross-lane
// shuffle.  SPLIT = 1: one row per thread (64 or 256 threads).
template <typename TO, typename TV, int SPLIT>
__global__ void __launch_bounds__(256)
    k_sweep_pp(const TO* __restrict__ M, const int64_t* __restrict__ pofs, const int32_t* __restrict__ port_off,
               const int32_t* __restrict__ port_twin, const TV* __restrict__ h, const TV* __restrict__ a_cur,
               TV* __restrict__ a_next, int max_q) {
    constexpr int G = Group<TO>::G;
    extern __shared__ char smem[];
    TV* av = reinterpret_cast<TV*>(smem);
    const int s = blockIdx.x;
    const int p0 = port_off[s], q = port_off[s + 1] - p0;
    const int lane = threadIdx.x;
    const TO* Ms = M + pofs[s];
    const int ng = q / G, full = ng * G;
    const int bs = blockDim.x;
    for (int t = lane; t < q; t += bs) av[t] = a_cur[p0 + t];
    __syncthreads();
    if constexpr (SPLIT == 2) {
        const int row = lane & 31, half = lane >> 5;
        const int g_lo = half ? (ng + 1) / 2 : 0, g_hi = half ? ng : (ng + 1) / 2;
        TV acc[G];
#pragma unroll
        for (int j = 0; j < G; ++j) acc[j] = TV(0);
        if (row < q) {
#pragma unroll 4
            for (int g = g_lo; g < g_hi; ++g) {
                TO v[G];
                load16p<TO>(Ms + (int64_t(g) * q + row) * G, v);
#pragma unroll
                for (int j = 0; j < G; ++j) acc[j] += TV(v[j]) * av[g * G + j];
            }
            if (half == 0)
                for (int c = full; c < q; ++c) acc[0] += TV(Ms[int64_t(full) * q + int64_t(c - full) * q + row]) * av[c];
        }
        TV v = acc[0];
#pragma unroll
        for (int j = 1; j < G; ++j) v += acc[j];
        v += __shfl_down(v, 32, 64);
        if (half == 0 && row < q) a_next[port_twin[p0 + row]] = h[p0 + row] + v;
    } else {
        for (int row = lane; row < q; row += bs) {
            TV acc[G];
#pragma unroll
            for (int j = 0; j < G; ++j) acc[j] = TV(0);
#pragma unroll 4
            for (int g = 0; g < ng; ++g) {
                TO v[G];
                load16p<TO>(Ms + (int64_t(g) * q + row) * G, v);
#pragma unroll
                for (int j = 0; j < G; ++j) acc[j] += TV(v[j]) * av[g * G + j];
            }
            for (int c = full; c < q; ++c) acc[0] += TV(Ms[int64_t(full) * q + int64_t(c - full) * q + row]) * av[c];
            TV v = acc[0];
#pragma unroll
            for (int j = 1; j < G; ++j) v += acc[j];
            a_next[port_twin[p0 + row]] = h[p0 + row] + v;
        }
    }
}

}  // namespace

template <typename TO>
hipError_t launch_port_matrix(int S, const int32_t* sub_off, const int64_t* kofs, const int32_t* port_off,
                              const int32_t* port_node, const double* pc, const double* pbeta, const double* pgamma,
                              const TO* K, const int64_t* pofs, TO* M, hipStream_t st) {
    hipLaunchKernelGGL(k_port_matrix<TO>, dim3(S), dim3(kBlock), 0, st, sub_off, kofs, port_off, port_node, pc,
                       pbeta, pgamma, K, pofs, M);
    return hipGetLastError();
}

template <typename TV>
hipError_t launch_port_h(int S, const int32_t* sub_off, const int32_t* port_off, const int32_t* port_node,
                         const TV* pbeta, const TV* x, TV* h, hipStream_t st) {
    hipLaunchKernelGGL(k_port_h<TV>, dim3(S), dim3(64), 0, st, S, sub_off, port_off, port_node, pbeta, x, h);
    return hipGetLastError();
}

template <typename TO, typename TV>
hipError_t launch_sweep_pp(int S, int max_q, const TO* M, const int64_t* pofs, const int32_t* port_off,
                           const int32_t* port_twin, const TV* h, const TV* a_cur, TV* a_next, hipStream_t st) {
    const size_t lds = size_t(max_q > 0 ? max_q : 1) * sizeof(TV);
    if (lds > 65536) return hipErrorInvalidValue;
    if (max_q <= 32)
        hipLaunchKernelGGL((k_sweep_pp<TO, TV, 2>), dim3(S), dim3(64), lds, st, M, pofs, port_off, port_twin, h,
                           a_cur, a_next, max_q);
    else
        hipLaunchKernelGGL((k_sweep_pp<TO, TV, 1>), dim3(S), dim3(max_q <= 64 ? 64 : 256), lds, st, M, pofs,
                           port_off, port_twin, h, a_cur, a_next, max_q);
    return hipGetLastError();
}

template hipError_t launch_port_matrix<double>(int, const int32_t*, const int64_t*, const int32_t*, const int32_t*,
                                               const double*, const double*, const double*, const double*,
                                               const int64_t*, double*, hipStream_t);
template hipError_t launch_port_matrix<float>(int, const int32_t*, const int64_t*, const int32_t*, const int32_t*,
                                              const double*, const double*, const double*, const float*,
                                              const int64_t*, float*, hipStream_t);
template hipError_t launch_port_h<double>(int, const int32_t*, const int32_t*, const int32_t*, const double*,
                                          const double*, double*, hipStream_t);
template hipError_t launch_port_h<float>(int, const int32_t*, const int32_t*, const int32_t*, const float*,
                                         const float*, float*, hipStream_t);
template hipError_t launch_sweep_pp<double, double>(int, int, const double*, const int64_t*, const int32_t*,
                                                    const int32_t*, const double*, const double*, double*,
                                                    hipStream_t);
template hipError_t launch_sweep_pp<float, float>(int, int, const float*, const int64_t*, const int32_t*,
                                                  const int32_t*, const float*, const float*, float*, hipStream_t);

}  // namespace vtm
