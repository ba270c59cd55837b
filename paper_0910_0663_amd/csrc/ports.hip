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

#include <algorithm>

#include <type_traits>

namespace vtm {

namespace {

constexpr int kBlock = 256;

// M_s in the column-group layout (n = q), from the stored inverse K_s
template <typename TO>
__global__ void __launch_bounds__(kBlock)
    k_port_matrix(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs,
                  const int32_t* __restrict__ port_off, const int32_t* __restrict__ port_node,
                  const double* __restrict__ pc, const double* __restrict__ pbeta, const double* __restrict__ pgamma,
                  const TO* __restrict__ K, const int64_t* __restrict__ pofs, TO* __restrict__ M, Coupling<double> B) {
    const int s = blockIdx.x;
    const int ns = sub_off[s + 1] - sub_off[s];
    const int p0 = port_off[s], q = port_off[s + 1] - p0;
    const TO* Ks = K + kofs[s];
    TO* Ms = M + pofs[s];
    const int64_t cnt = int64_t(q) * q;
    for (int64_t d = int64_t(blockIdx.y) * blockDim.x + threadIdx.x; d < cnt; d += int64_t(blockDim.x) * gridDim.y) {
        int r, c;
        inv_rc<TO>(q, d, r, c);
        const int pr = p0 + r, pcol = p0 + c;
        const int j = port_node[pcol];
        double v;
        if (B.row) {  // (B K^-1[i(P), i(P)])_{r c}: B's row r over the ports of this sub-circuit
            v = 0.0;
            for (int k = B.row[pr]; k < B.row[pr + 1]; ++k)
                v += B.val[k] * double(Ks[inv_offset<TO>(ns, port_node[B.col[k]], j)]);
            v *= pc[pcol];
        } else {
            v = pbeta[pr] * double(Ks[inv_offset<TO>(ns, port_node[pr], j)]) * pc[pcol];
        }
        if (r == c) v += pgamma[pr];
        Ms[d] = TO(v);
    }
}

// h_p = beta_p x_i(p) for x = K^-1 b, per right-hand side (x and h are
// [rows][nrhs], right-hand side fastest)
template <typename TV>
__global__ void __launch_bounds__(kBlock)
    k_port_h(int nrhs, const int32_t* __restrict__ sub_off, const int32_t* __restrict__ port_off,
             const int32_t* __restrict__ port_node, const TV* __restrict__ pbeta, const TV* __restrict__ x,
             TV* __restrict__ h, Coupling<TV> B) {
    const int s = blockIdx.x;
    const int off = sub_off[s], p0 = port_off[s];
    const int cnt = (port_off[s + 1] - p0) * nrhs;
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
        const int p = p0 + t / nrhs, r = t % nrhs;
        TV v;
        if (B.row) {
            v = TV(0);
            for (int k = B.row[p]; k < B.row[p + 1]; ++k)
                v += B.val[k] * x[int64_t(off + port_node[B.col[k]]) * nrhs + r];
        } else {
            v = pbeta[p] * x[int64_t(off + port_node[p]) * nrhs + r];
        }
        h[int64_t(p) * nrhs + r] = v;
    }
}

// coupled lines: the outgoing waves from the x of a full sweep
template <typename TV>
__global__ void __launch_bounds__(kBlock)
    k_wave_coupled(int n_ports, int nrhs, Coupling<TV> B, const int32_t* __restrict__ port_row,
                   const TV* __restrict__ pgamma, const int32_t* __restrict__ port_twin, const TV* __restrict__ x,
                   const TV* __restrict__ a_cur, TV* __restrict__ a_next) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(n_ports) * nrhs) return;
    const int p = int(t / nrhs), r = int(t - int64_t(p) * nrhs);
    TV v = pgamma[p] * a_cur[t];
    for (int k = B.row[p]; k < B.row[p + 1]; ++k) v += B.val[k] * x[int64_t(port_row[B.col[k]]) * nrhs + r];
    a_next[int64_t(port_twin[p]) * nrhs + r] = v;
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
// shuffle.  SPLIT = 1: one row per thread (64 or 256 threads); with few large
// sub-circuits the rows of each are also spread over gridDim.y workgroups.
template <typename TO, typename TV, int SPLIT>
__global__ void __launch_bounds__(256)
    k_sweep_pp(const TO* __restrict__ M, const int64_t* __restrict__ pofs, const int32_t* __restrict__ port_off,
               const int32_t* __restrict__ port_twin, const TV* __restrict__ h, const TV* __restrict__ a_cur,
               TV* __restrict__ a_next, int max_q) {
    constexpr int G = Group<TO>::G;
    extern __shared__ char smem[];
    TV* av = reinterpret_cast<TV*>(smem);
    const int s = xcd_block(blockIdx.x, gridDim.x);
    const int p0 = port_off[s], q = port_off[s + 1] - p0;
    const int lane = threadIdx.x;
    const TO* Ms = M + pofs[s];
    const int ng = q / G, full = ng * G;
    const int bs = blockDim.x;
    if (int(blockIdx.y) * bs >= q) return;  // no rows for this block (whole workgroup leaves)
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
        for (int row = int(blockIdx.y) * bs + lane; row < q; row += bs * int(gridDim.y)) {
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

// Port-node form for any A (the packed kernel below needs A symmetric): with
// z = K^-1[N, N] t over the k port nodes N of a sub-circuit and
// t_n = sum_{p at n} c_p a_p, the outgoing wave of port p is
// o_p = beta_p z_n(p) + gamma_p a_p + h_p.  K^-1[N, N] (k x k, fewer than the
// q x q entries of M when nodes carry several ports) is stored in the column-
// group layout (n = k) at Sn + nofs[s].
template <typename TO>
__global__ void __launch_bounds__(kBlock)
    k_port_node_dense(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs,
                      const int32_t* __restrict__ pn_off, const int32_t* __restrict__ pn_node,
                      const TO* __restrict__ K, const int64_t* __restrict__ nofs, TO* __restrict__ Sn,
                      int transpose) {
    const int s = blockIdx.x;
    const int ns = sub_off[s + 1] - sub_off[s];
    const int k0 = pn_off[s], k = pn_off[s + 1] - k0;
    const TO* Ks = K + kofs[s];
    TO* out = Sn + nofs[s];
    for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
        const int r = t / k, c = t - r * k;
        const int i = pn_node[k0 + (transpose ? c : r)], j = pn_node[k0 + (transpose ? r : c)];
        out[inv_offset<TO>(k, r, c)] = Ks[inv_offset<TO>(ns, i, j)];
    }
}

// One workgroup per sub-circuit, one port node (row of K^-1[N, N]) per thread.
template <typename TO, typename TV>
__global__ void __launch_bounds__(512)
    k_sweep_ppn(const TO* __restrict__ Sn, const int64_t* __restrict__ nofs, const int32_t* __restrict__ pn_off,
                const int32_t* __restrict__ pn_pfirst, const int32_t* __restrict__ port_off,
                const int32_t* __restrict__ port_twin, const TV* __restrict__ pc, const TV* __restrict__ pbeta,
                const TV* __restrict__ pgamma, const TV* __restrict__ h, const TV* __restrict__ a_cur,
                TV* __restrict__ a_next, int max_npn) {
    constexpr int G = Group<TO>::G;
    extern __shared__ char smem[];
    TV* tv = reinterpret_cast<TV*>(smem);
    TV* zv = tv + max_npn;
    int32_t* pnode = reinterpret_cast<int32_t*>(zv + max_npn);
    const int s = xcd_block(blockIdx.x, gridDim.x);
    const int k0 = pn_off[s], k = pn_off[s + 1] - k0;
    const int p0 = port_off[s], p1 = port_off[s + 1];
    const int tid = threadIdx.x, bs = blockDim.x;
    const TO* Ss = Sn + nofs[s];
    // t per port node, in port order
    for (int j = tid; j < k; j += bs) {
        const int f0 = pn_pfirst[k0 + j], f1 = pn_pfirst[k0 + j + 1];
        TV acc = TV(0);
        for (int p = f0; p < f1; ++p) {
            acc += pc[p] * a_cur[p];
            pnode[p - p0] = j;
        }
        tv[j] = acc;
    }
    __syncthreads();
    // z = K^-1[N, N] t
    const int ng = k / G, full = ng * G;
    for (int row = tid; row < k; row += bs) {
        TV acc[G];
#pragma unroll
        for (int j = 0; j < G; ++j) acc[j] = TV(0);
#pragma unroll 4
        for (int g = 0; g < ng; ++g) {
            TO v[G];
            load16p<TO>(Ss + (int64_t(g) * k + row) * G, v);
#pragma unroll
            for (int j = 0; j < G; ++j) acc[j] += TV(v[j]) * tv[g * G + j];
        }
        for (int c = full; c < k; ++c) acc[0] += TV(Ss[int64_t(full) * k + int64_t(c - full) * k + row]) * tv[c];
        TV v = acc[0];
#pragma unroll
        for (int j = 1; j < G; ++j) v += acc[j];
        zv[row] = v;
    }
    __syncthreads();
    for (int p = p0 + tid; p < p1; p += bs)
        a_next[port_twin[p]] = pbeta[p] * zv[pnode[p - p0]] + pgamma[p] * a_cur[p] + h[p];
}

}  // namespace

template <typename TO>
hipError_t launch_port_node_dense(int S, const int32_t* sub_off, const int64_t* kofs, const int32_t* pn_off,
                                  const int32_t* pn_node, const TO* K, const int64_t* nofs, TO* Sn, bool transpose,
                                  hipStream_t st) {
    hipLaunchKernelGGL(k_port_node_dense<TO>, dim3(S), dim3(kBlock), 0, st, sub_off, kofs, pn_off, pn_node, K, nofs,
                       Sn, transpose ? 1 : 0);
    return hipGetLastError();
}

template <typename TO, typename TV>
hipError_t launch_sweep_ppn(int S, int max_npn, int max_ports, const TO* Sn, const int64_t* nofs,
                            const int32_t* pn_off, const int32_t* pn_pfirst, const int32_t* port_off,
                            const int32_t* port_twin, const TV* pc, const TV* pbeta, const TV* pgamma, const TV* h,
                            const TV* a_cur, TV* a_next, hipStream_t st) {
    const size_t lds = 2 * size_t(max_npn) * sizeof(TV) + size_t(max_ports) * 4;
    if (lds > 65536) return hipErrorInvalidValue;
    // one pass over the rows where possible
    const int bs = std::min(512, std::max(64, ((max_npn + 63) / 64) * 64));
    hipLaunchKernelGGL((k_sweep_ppn<TO, TV>), dim3(S), dim3(bs), lds, st, Sn, nofs, pn_off, pn_pfirst, port_off,
                       port_twin, pc, pbeta, pgamma, h, a_cur, a_next, max_npn);
    return hipGetLastError();
}

template hipError_t launch_port_node_dense<double>(int, const int32_t*, const int64_t*, const int32_t*,
                                                   const int32_t*, const double*, const int64_t*, double*, bool,
                                                   hipStream_t);
template hipError_t launch_port_node_dense<float>(int, const int32_t*, const int64_t*, const int32_t*,
                                                  const int32_t*, const float*, const int64_t*, float*, bool,
                                                  hipStream_t);
template hipError_t launch_sweep_ppn<double, double>(int, int, int, const double*, const int64_t*, const int32_t*,
                                                     const int32_t*, const int32_t*, const int32_t*, const double*,
                                                     const double*, const double*, const double*, const double*,
                                                     double*, hipStream_t);
template hipError_t launch_sweep_ppn<float, float>(int, int, int, const float*, const int64_t*, const int32_t*,
                                                   const int32_t*, const int32_t*, const int32_t*, const float*,
                                                   const float*, const float*, const float*, const float*, float*,
                                                   hipStream_t);

template <typename TO>
hipError_t launch_port_matrix(int S, const int32_t* sub_off, const int64_t* kofs, const int32_t* port_off,
                              const int32_t* port_node, const double* pc, const double* pbeta, const double* pgamma,
                              const TO* K, const int64_t* pofs, TO* M, hipStream_t st, Coupling<double> B) {
    // few sub-circuits: several workgroups each
    const int parts = S < 2048 ? (2048 + S - 1) / S : 1;
    hipLaunchKernelGGL(k_port_matrix<TO>, dim3(S, parts), dim3(kBlock), 0, st, sub_off, kofs, port_off, port_node,
                       pc, pbeta, pgamma, K, pofs, M, B);
    return hipGetLastError();
}

template <typename TV>
hipError_t launch_port_h(int S, int nrhs, const int32_t* sub_off, const int32_t* port_off, const int32_t* port_node,
                         const TV* pbeta, const TV* x, TV* h, hipStream_t st, Coupling<TV> B) {
    hipLaunchKernelGGL(k_port_h<TV>, dim3(S), dim3(nrhs > 1 ? 256 : 64), 0, st, nrhs, sub_off, port_off, port_node,
                       pbeta, x, h, B);
    return hipGetLastError();
}

template <typename TV>
hipError_t launch_wave_coupled(int n_ports, int nrhs, Coupling<TV> B, const int32_t* port_row, const TV* pgamma,
                               const int32_t* port_twin, const TV* x, const TV* a_cur, TV* a_next, hipStream_t st) {
    const int64_t total = int64_t(n_ports) * nrhs;
    if (total == 0) return hipSuccess;
    if (!B.row) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_wave_coupled<TV>, dim3(unsigned((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       n_ports, nrhs, B, port_row, pgamma, port_twin, x, a_cur, a_next);
    return hipGetLastError();
}
template hipError_t launch_wave_coupled<double>(int, int, Coupling<double>, const int32_t*, const double*,
                                                const int32_t*, const double*, const double*, double*, hipStream_t);
template hipError_t launch_wave_coupled<float>(int, int, Coupling<float>, const int32_t*, const float*,
                                               const int32_t*, const float*, const float*, float*, hipStream_t);

template <typename TO, typename TV>
hipError_t launch_sweep_pp(int S, int max_q, const TO* M, const int64_t* pofs, const int32_t* port_off,
                           const int32_t* port_twin, const TV* h, const TV* a_cur, TV* a_next, hipStream_t st) {
    const size_t lds = size_t(max_q > 0 ? max_q : 1) * sizeof(TV);
    if (lds > 65536) return hipErrorInvalidValue;
    if (max_q <= 32)
        hipLaunchKernelGGL((k_sweep_pp<TO, TV, 2>), dim3(S), dim3(64), lds, st, M, pofs, port_off, port_twin, h,
                           a_cur, a_next, max_q);
    else {
        // few sub-circuits with many ports: one-wavefront blocks, each sub-circuit's rows
        // spread over several
        const bool split = S < 1024 && max_q > 64;
        const int bs = split || max_q <= 64 ? 64 : 256;
        const int ry = split ? (max_q + bs - 1) / bs : 1;
        hipLaunchKernelGGL((k_sweep_pp<TO, TV, 1>), dim3(S, ry), dim3(bs), lds, st, M, pofs, port_off, port_twin,
                           h, a_cur, a_next, max_q);
    }
    return hipGetLastError();
}

template hipError_t launch_port_matrix<double>(int, const int32_t*, const int64_t*, const int32_t*, const int32_t*,
                                               const double*, const double*, const double*, const double*,
                                               const int64_t*, double*, hipStream_t, Coupling<double>);
template hipError_t launch_port_matrix<float>(int, const int32_t*, const int64_t*, const int32_t*, const int32_t*,
                                              const double*, const double*, const double*, const float*,
                                              const int64_t*, float*, hipStream_t, Coupling<double>);
template hipError_t launch_port_h<double>(int, int, const int32_t*, const int32_t*, const int32_t*, const double*,
                                          const double*, double*, hipStream_t, Coupling<double>);
template hipError_t launch_port_h<float>(int, int, const int32_t*, const int32_t*, const int32_t*, const float*,
                                         const float*, float*, hipStream_t, Coupling<float>);
template hipError_t launch_sweep_pp<double, double>(int, int, const double*, const int64_t*, const int32_t*,
                                                    const int32_t*, const double*, const double*, double*,
                                                    hipStream_t);
template hipError_t launch_sweep_pp<float, float>(int, int, const float*, const int64_t*, const int32_t*,
                                                  const int32_t*, const float*, const float*, float*, hipStream_t);

}  // namespace vtm

// ---------------------------------------------------------------------------
// Symmetric A: the port-node form.  K^-1 restricted to the port nodes,
// S = K^-1[N, N], is symmetric, and with beta = 2 W c and gamma = 1 - 2 c the
// outgoing waves are
//     o_p = 2 W_p c_p z_n(p) + (1 - 2 c_p) a_p + h_p,   z = S t,  t_n = sum_{p at n} c_p a_p,
// so a sweep streams only the upper triangle of S besides the per-port wave,
// c, h and twin.  The triangle of a sub-circuit with k port nodes is stored as
// pairs of diagonals: pair m holds, for rows r = 0 .. k - 2m - 1, the two
// entries S(r, r + 2m) and S(r, r + 2m + 1) side by side (the second is zero
// in the pair's last row), and starts at 2m (k - m + 1).  Lane r reads both
// entries of every pair with one coalesced 16-byte (FP64) load and receives
// S(r - d, r) from lane r - d.
// ---------------------------------------------------------------------------
namespace vtm {
namespace {

// diagonals per chunk of the packed sweep, each lane's loads of one chunk in
// flight together (even: whole pairs)
constexpr int kPpsChunk = 8;
// chunks issued before the first barrier when two sub-circuits share a wavefront
// (the rest stream that far ahead)
constexpr int kPpsPre = 2;
// wavefronts per sub-circuit when a sub-circuit has 33..64 port nodes (k_sweep_pps_split)
constexpr int kPpsSplit = 8;

// pair m of diagonals (2m, 2m + 1), rows r = 0 .. k - 2m - 1 each holding both entries
__host__ __device__ inline int pair_start(int k, int m) { return 2 * m * (k - m + 1); }

template <typename TO>
__global__ void __launch_bounds__(256)
    k_port_node_matrix(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs,
                       const int32_t* __restrict__ pn_off, const int32_t* __restrict__ pn_node,
                       const TO* __restrict__ K, const int64_t* __restrict__ sofs, TO* __restrict__ Sp) {
    const int s = blockIdx.x;
    const int ns = sub_off[s + 1] - sub_off[s];
    const int k0 = pn_off[s], k = pn_off[s + 1] - k0;
    const TO* Ks = K + kofs[s];
    TO* out = Sp + sofs[s];
    for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
        const int r = t / k, c = t - r * k;
        if (r <= c)
            out[pair_start(k, (c - r) >> 1) + 2 * r + ((c - r) & 1)] =
                Ks[inv_offset<TO>(ns, pn_node[k0 + r], pn_node[k0 + c])];
    }
}

// One wavefront per sub-circuit (HALF: two, 32 lanes each).  Lane r owns port
// node r and port r of its sub-circuit.  The offsets come from scalar loads of
// a wave-uniform base; every other global load of the sweep is issued before
// the first barrier, PRE chunks of CH diagonals among them, and the rest
// stream PRE chunks ahead of use.  Inside a chunk there are no branches: a
// lane past the end of a pair loads a valid entry (the block's first two) and
// multiplies it by a zero of the padded t (each sub-circuit's t takes a
// 64-entry region, zero beyond its k port nodes), so the compiler can keep
// loads in flight across it; the only branch, a wave-uniform exit once the
// chunks pass the larger k of the wavefront, is scalar.
template <typename TO, typename TV, bool HALF>
__device__ inline void pps_unit(int unit, int S, const TO* __restrict__ Sp, const int64_t* __restrict__ sofs,
                                const int32_t* __restrict__ pn_off, const int32_t* __restrict__ pn_pfirst,
                                const int32_t* __restrict__ port_off, const int32_t* __restrict__ port_twin,
                                const TV* __restrict__ pc, const TV* __restrict__ pW, TV W,
                                const TV* __restrict__ h, const TV* __restrict__ a_cur, TV* __restrict__ a_next,
                                TV* ca, TV* tv, TV* zv, int32_t* pnode) {
    constexpr int L = HALF ? 32 : 64;
    constexpr int CH = kPpsChunk;
    constexpr int NCH = L / CH;
    constexpr int PRE = HALF ? kPpsPre : 1;
    static_assert(L % CH == 0 && PRE >= 1 && PRE <= NCH, "diagonal chunks must tile the lanes");
    const int tid = threadIdx.x, r = tid % L, hb = tid - r, half = tid / L;
    const int tb = half * 64;  // this sub-circuit's t region
    // wave-uniform offsets of the (one or two) sub-circuits, indices clamped to S
    const int sb = unit * (64 / L);
    const int sa = min(sb, S), sm = min(sb + 1, S), sz = min(sb + 2, S);
    const int nA = pn_off[sa], nB = pn_off[sm], nC = HALF ? pn_off[sz] : 0;
    const int pA = port_off[sa], pB = port_off[sm], pC = HALF ? port_off[sz] : 0;
    const int64_t eA = sofs[sa], eB = HALF ? sofs[sm] : 0;
    const bool valid = sb + half < S;
    const int n0 = half ? nB : nA, k = valid ? (half ? nC - nB : nB - nA) : 0;
    const int p0 = half ? pB : pA, q = valid ? (half ? pC - pB : pB - pA) : 0;
    const TO* blk = Sp + (valid ? (half ? eB : eA) : 0);
    const bool has_port = r < q;
    TV c = TV(0), a = TV(0), hp = TV(0), w = W;
    int tw = 0;
    if (has_port) {
        const int p = p0 + r;
        c = pc[p];
        a = a_cur[p];
        hp = h[p];
        tw = port_twin[p];
        if (pW) w = pW[p];
        ca[hb + r] = c * a;
    }
    int f0 = 0, f1 = 0;
    if (r < k) f0 = pn_pfirst[n0 + r] - p0;
    {
        const int nx = __shfl(f0, tid + 1);  // lane r + 1's first port (the last lane: q)
        f1 = r + 1 < k ? nx : q;
    }
    TO buf[L];  // diagonal d of this lane's row (compile-time indices only)
    // CH / 2 pairs per chunk, one 16-byte (FP64) load each: S(r, r + 2m), S(r, r + 2m + 1)
    static_assert(CH % 2 == 0, "chunks hold whole pairs");
    using V2 = typename std::conditional<sizeof(TO) == 8, double2, float2>::type;
    auto load = [&](int ci) {
#pragma unroll
        for (int j = 0; j < CH / 2; ++j) {
            const int m = ci * (CH / 2) + j;
            const V2 v2 = *reinterpret_cast<const V2*>(blk + ((r + 2 * m < k) ? pair_start(k, m) + 2 * r : 0));
            buf[2 * m] = v2.x;
            buf[2 * m + 1] = v2.y;
        }
    };
#pragma unroll
    for (int ci = 0; ci < PRE; ++ci) load(ci);
    tv[tid] = TV(0);
    tv[tid + 64] = TV(0);
    __syncthreads();
    // t_n = sum of c_p a_p over the ports at n, in port order
    if (r < k) {
        TV acc = TV(0);
        for (int i = f0; i < f1; ++i) {
            acc += ca[hb + i];
            pnode[hb + i] = r;
        }
        tv[tb + r] = acc;
    }
    __syncthreads();
    // z_r = sum_d S(r, r + d) t_{r+d} + sum_{d>0} S(r - d, r) t_{r-d}; the second
    // product is formed by lane r - d (which holds S(r - d, r)) and shuffled up.
    // d < L keeps tb + r + d inside tv.
    const TV tr = tv[tb + r];
    TV acc = TV(0);
    int kmax = k;
    if (HALF) kmax = max(k, __shfl_xor(k, 32));
    kmax = __builtin_amdgcn_readfirstlane(kmax);  // wave-uniform: the chunk loop branches on scalars
#pragma unroll
    for (int ci = 0; ci < NCH; ++ci) {
        if (ci * CH >= kmax) break;
        if (ci + PRE < NCH) load(ci + PRE);
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int d = ci * CH + j;
            const TV sv = TV(buf[d]);
            acc += sv * tv[tb + r + d];
            const TV up = __shfl(sv * tr, tid - d);
            acc += (d > 0 && r >= d) ? up : TV(0);
        }
    }
    if (r < k) zv[hb + r] = acc;
    __syncthreads();
    if (has_port) a_next[tw] = TV(2) * w * c * zv[hb + pnode[hb + r]] + (TV(1) - TV(2) * c) * a + hp;
}

// One workgroup (one wavefront) per unit: a pair of sub-circuits when HALF.
template <typename TO, typename TV, bool HALF>
__global__ void __launch_bounds__(64)
    k_sweep_pps(int S, const TO* __restrict__ Sp, const int64_t* __restrict__ sofs,
                const int32_t* __restrict__ pn_off, const int32_t* __restrict__ pn_pfirst,
                const int32_t* __restrict__ port_off, const int32_t* __restrict__ port_twin,
                const TV* __restrict__ pc, const TV* __restrict__ pW, TV W, const TV* __restrict__ h,
                const TV* __restrict__ a_cur, TV* __restrict__ a_next, int reverse) {
    __shared__ TV ca[64], tv[128], zv[64];
    __shared__ int32_t pnode[64];
    // every other sweep walks each XCD's units backwards, so that the operators it
    // reads first are the ones the previous sweep read last (still in the
    // memory-side cache), while each XCD keeps the same units (and its L2)
    const int unit = reverse ? xcd_block_reversed(blockIdx.x, gridDim.x) : xcd_block(blockIdx.x, gridDim.x);
    pps_unit<TO, TV, HALF>(unit, S, Sp, sofs, pn_off, pn_pfirst, port_off, port_twin, pc, pW, W, h, a_cur, a_next,
                           ca, tv, zv, pnode);
}

// One sub-circuit of up to 64 port nodes per workgroup of WV wavefronts: lane r of
// every wavefront keeps row r, and wavefront v takes the diagonal chunks
// v, v + WV, ...  All of a wavefront's operator loads are issued at once, before
// the first barrier (WV times fewer per lane than with one wavefront, so the
// sweep of few, large sub-circuits waits on fewer round trips); the partial
// sums z_r of the wavefronts meet in LDS.
template <typename TO, typename TV, int WV>
__global__ void __launch_bounds__(64 * WV)
    k_sweep_pps_split(const TO* __restrict__ Sp, const int64_t* __restrict__ sofs,
                      const int32_t* __restrict__ pn_off, const int32_t* __restrict__ pn_pfirst,
                      const int32_t* __restrict__ port_off, const int32_t* __restrict__ port_twin,
                      const TV* __restrict__ pc, const TV* __restrict__ pW, TV W, const TV* __restrict__ h,
                      const TV* __restrict__ a_cur, TV* __restrict__ a_next, int reverse) {
    constexpr int CH = kPpsChunk, NCH = 64 / CH, LCH = NCH / WV;
    static_assert(WV >= 2 && NCH % WV == 0 && CH % 2 == 0, "chunks must split evenly over the wavefronts");
    __shared__ TV ca[64], tv[128], zp[WV][64];
    __shared__ int32_t pnode[64];
    const int s = reverse ? xcd_block_reversed(blockIdx.x, gridDim.x) : xcd_block(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x, r = tid & 63, wv = tid >> 6;
    const int n0 = pn_off[s], k = pn_off[s + 1] - n0;
    const int p0 = port_off[s], q = port_off[s + 1] - p0;
    const TO* blk = Sp + sofs[s];
    // this wavefront's diagonals d = ci CH + j, ci = li WV + wv (pairs: one 16-byte
    // FP64 load gives S(r, r + 2m) and S(r, r + 2m + 1))
    using V2 = typename std::conditional<sizeof(TO) == 8, double2, float2>::type;
    TO buf[LCH * CH];
#pragma unroll
    for (int li = 0; li < LCH; ++li) {
        const int ci = li * WV + wv;
        if (ci * CH < k) {
#pragma unroll
            for (int j = 0; j < CH / 2; ++j) {
                const int m = ci * (CH / 2) + j;
                const V2 v2 = *reinterpret_cast<const V2*>(blk + ((r + 2 * m < k) ? pair_start(k, m) + 2 * r : 0));
                buf[li * CH + 2 * j] = v2.x;
                buf[li * CH + 2 * j + 1] = v2.y;
            }
        }
    }
    // wavefront 0: the ports (lane r = port p0 + r) and each node's port range
    TV c = TV(0), a = TV(0), hp = TV(0), w = W;
    int tw = 0, f0 = 0, f1 = 0;
    const bool has_port = wv == 0 && r < q;
    if (has_port) {
        const int p = p0 + r;
        c = pc[p];
        a = a_cur[p];
        hp = h[p];
        tw = port_twin[p];
        if (pW) w = pW[p];
        ca[r] = c * a;
    }
    if (wv == 0 && r < k) {
        f0 = pn_pfirst[n0 + r] - p0;
        f1 = pn_pfirst[n0 + r + 1] - p0;
    }
    if (tid < 128) tv[tid] = TV(0);
    __syncthreads();
    // t_n = sum of c_p a_p over the ports at node n, in port order
    if (wv == 0 && r < k) {
        TV acc = TV(0);
        for (int i = f0; i < f1; ++i) {
            acc += ca[i];
            pnode[i] = r;
        }
        tv[r] = acc;
    }
    __syncthreads();
    // partial z_r over this wavefront's diagonals: S(r, r + d) t_{r+d}, and for
    // d > 0 S(r - d, r) t_{r-d}, formed by lane r - d and shuffled up
    const TV tr = tv[r];
    TV acc = TV(0);
#pragma unroll
    for (int li = 0; li < LCH; ++li) {
        const int ci = li * WV + wv;
        if (ci * CH < k) {
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int d = ci * CH + j;
                const TV sv = TV(buf[li * CH + j]);
                acc += sv * tv[r + d];
                const TV up = __shfl(sv * tr, r - d);
                acc += (d > 0 && r >= d) ? up : TV(0);
            }
        }
    }
    zp[wv][r] = acc;
    __syncthreads();
    if (has_port) {
        const int n = pnode[r];
        TV z = TV(0);
#pragma unroll
        for (int v = 0; v < WV; ++v) z += zp[v][n];
        a_next[tw] = TV(2) * w * c * z + (TV(1) - TV(2) * c) * a + hp;
    }
}

}  // namespace

template <typename TO>
hipError_t launch_port_node_matrix(int S, const int32_t* sub_off, const int64_t* kofs, const int32_t* pn_off,
                                   const int32_t* pn_node, const TO* K, const int64_t* sofs, TO* Sp,
                                   hipStream_t st) {
    hipLaunchKernelGGL(k_port_node_matrix<TO>, dim3(S), dim3(256), 0, st, sub_off, kofs, pn_off, pn_node, K, sofs,
                       Sp);
    return hipGetLastError();
}

template <typename TO, typename TV, bool HALF>
hipError_t launch_pps(int S, const TO* Sp, const int64_t* sofs, const int32_t* pn_off, const int32_t* pn_pfirst,
                      const int32_t* port_off, const int32_t* port_twin, const TV* pc, const TV* pW, TV W,
                      const TV* h, const TV* a_cur, TV* a_next, int reverse, hipStream_t st) {
    const int units = HALF ? (S + 1) / 2 : S;
    hipLaunchKernelGGL((k_sweep_pps<TO, TV, HALF>), dim3(units), dim3(64), 0, st, S, Sp, sofs, pn_off, pn_pfirst,
                       port_off, port_twin, pc, pW, W, h, a_cur, a_next, reverse);
    return hipGetLastError();
}

template <typename TO, typename TV>
hipError_t launch_sweep_pps(int S, int max_npn, int max_ports, const TO* Sp, const int64_t* sofs,
                            const int32_t* pn_off, const int32_t* pn_pfirst, const int32_t* port_off,
                            const int32_t* port_twin, const TV* pc, const TV* pW, TV W, const TV* h,
                            const TV* a_cur, TV* a_next, int reverse, hipStream_t st) {
    if (max_npn > 64 || max_ports > 64) return hipErrorInvalidValue;
    if (S == 0) return hipSuccess;
    if (max_npn <= 32 && max_ports <= 32)
        return launch_pps<TO, TV, true>(S, Sp, sofs, pn_off, pn_pfirst, port_off, port_twin, pc, pW, W, h, a_cur,
                                        a_next, reverse, st);
    hipLaunchKernelGGL((k_sweep_pps_split<TO, TV, kPpsSplit>), dim3(S), dim3(64 * kPpsSplit), 0, st, Sp, sofs, pn_off,
                       pn_pfirst, port_off, port_twin, pc, pW, W, h, a_cur, a_next, reverse);
    return hipGetLastError();
}

template hipError_t launch_port_node_matrix<double>(int, const int32_t*, const int64_t*, const int32_t*,
                                                    const int32_t*, const double*, const int64_t*, double*,
                                                    hipStream_t);
template hipError_t launch_port_node_matrix<float>(int, const int32_t*, const int64_t*, const int32_t*,
                                                   const int32_t*, const float*, const int64_t*, float*,
                                                   hipStream_t);
template hipError_t launch_sweep_pps<double, double>(int, int, int, const double*, const int64_t*,
                                                     const int32_t*, const int32_t*, const int32_t*, const int32_t*,
                                                     const double*, const double*, double, const double*,
                                                     const double*, double*, int, hipStream_t);
template hipError_t launch_sweep_pps<float, float>(int, int, int, const float*, const int64_t*, const int32_t*,
                                                   const int32_t*, const int32_t*, const int32_t*, const float*,
                                                   const float*, float, const float*, const float*, float*, int,
                                                   hipStream_t);

}  // namespace vtm
