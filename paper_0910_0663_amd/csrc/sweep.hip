// The sweep kernel: one VTM sweep (eqs. 11 and 14, every line delay one sweep)
// for every sub-circuit at once, one workgroup per sub-circuit (per block of
// right-hand sides):
//   1. rhs = b + c * a at the port nodes (the incident wave entering through the
//      eliminated twin; ports of one node added in a fixed order),
//   2. x = Kinv rhs, a dense GEMV (GEMM over R right-hand sides) with the stored
//      inverse streamed once in 16-byte loads per lane,
//   3. outgoing wave beta * x + gamma * a (eq. 11, second line) written into the
//      twin port's slot of the next wave buffer (the message to the other side).
#include "kernels.hpp"
#include "layout.hpp"

namespace vtm {

namespace {

constexpr int kBlock = 256;

// column groups per prefetched chunk of the single right-hand-side kernel
constexpr int kSweepChunk = 8;

template <typename T>
__device__ inline void load16(const T* p, T (&v)[Group<T>::G]) {
    if constexpr (sizeof(T) == 8) {
        const double2 q = *reinterpret_cast<const double2*>(p);
        v[0] = q.x;
        v[1] = q.y;
    } else {
        const float4 q = *reinterpret_cast<const float4*>(p);
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
        v[3] = q.w;
    }
}

template <typename TO, typename TV, int R>
__global__ void __launch_bounds__(kBlock)
    k_sweep(const TO* __restrict__ K, const int64_t* __restrict__ kofs, const int32_t* __restrict__ sub_off,
            const int32_t* __restrict__ port_off, const int32_t* __restrict__ port_node,
            const int32_t* __restrict__ port_slot, const int32_t* __restrict__ port_twin,
            const TV* __restrict__ pc, const TV* __restrict__ pbeta, const TV* __restrict__ pgamma,
            const TV* __restrict__ b, const TV* __restrict__ a_cur, TV* __restrict__ a_next, TV* __restrict__ x,
            int nrhs, int max_ns, int max_slot, int adjoint, int xs_lds) {
    constexpr int G = Group<TO>::G;
    extern __shared__ char smem[];
    TV* rhs = reinterpret_cast<TV*>(smem);   // [max_ns][R]
    TV* xs = rhs + max_ns * R;               // [max_ns][R] when xs_lds (else the waves read x back)
    const int s = blockIdx.x;
    const int r0 = blockIdx.y * R;
    const int w = min(R, nrhs - r0);
    const int off = sub_off[s];
    const int ns = sub_off[s + 1] - off;
    const int p0 = port_off[s], p1 = port_off[s + 1];
    const int tid = threadIdx.x, bs = blockDim.x;
    // rows of this block: [z * bs, z * bs + bs) + k * bs * gridDim.z (gridDim.z > 1 spreads the
    // rows of a few large sub-circuits over several workgroups)
    const int row0 = int(blockIdx.z) * bs, rstep = bs * int(gridDim.z);
    if (row0 >= ns) return;  // uniform over the workgroup

    for (int t = tid; t < ns * R; t += bs) {
        const int row = t / R, k = t - row * R;
        rhs[t] = k < w ? b[int64_t(off + row) * nrhs + r0 + k] : TV(0);
    }
    __syncthreads();
    for (int pb = p0; pb < p1; pb += bs) {
        const int p = pb + tid;
        const bool ok = p < p1;
        const int node = ok ? port_node[p] : 0;
        const int slot = ok ? port_slot[p] : -1;
        const TV c = ok ? pc[p] : TV(0);
        for (int sl = 0; sl <= max_slot; ++sl) {
            if (slot == sl)
                for (int k = 0; k < w; ++k) rhs[node * R + k] += c * a_cur[int64_t(p) * nrhs + r0 + k];
            __syncthreads();
        }
    }

    const TO* Ks = K + kofs[s];
    const int full = (ns / G) * G;
    for (int row = row0 + tid; row < ns; row += rstep) {
        TV acc[R][G];
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
            for (int j = 0; j < G; ++j) acc[k][j] = TV(0);
        if (!adjoint) {
            const TO* kp = Ks + int64_t(row) * G;
#pragma unroll 4
            for (int c = 0; c < full; c += G) {
                TO v[G];
                load16<TO>(kp + int64_t(c) * ns, v);
#pragma unroll
                for (int j = 0; j < G; ++j)
#pragma unroll
                    for (int k = 0; k < R; ++k) acc[k][j] += TV(v[j]) * rhs[(c + j) * R + k];
            }
            for (int c = full; c < ns; ++c) {
                const TV v = TV(Ks[int64_t(full) * ns + int64_t(c - full) * ns + row]);
#pragma unroll
                for (int k = 0; k < R; ++k) acc[k][0] += v * rhs[c * R + k];
            }
        } else {
            // K^-T: entry (c, row) of the stored inverse
            int c = 0;
            for (; c + G <= ns; c += G) {
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    const TV v = TV(Ks[inv_offset<TO>(ns, c + j, row)]);
#pragma unroll
                    for (int k = 0; k < R; ++k) acc[k][j] += v * rhs[(c + j) * R + k];
                }
            }
            for (; c < ns; ++c) {
                const TV v = TV(Ks[inv_offset<TO>(ns, c, row)]);
#pragma unroll
                for (int k = 0; k < R; ++k) acc[k][0] += v * rhs[c * R + k];
            }
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            TV v = acc[k][0];
#pragma unroll
            for (int j = 1; j < G; ++j) v += acc[k][j];
            if (xs_lds) xs[row * R + k] = v;
            if (k < w) x[int64_t(off + row) * nrhs + r0 + k] = v;
        }
    }
    __syncthreads();
    for (int p = p0 + tid; p < p1; p += bs) {
        const int node = port_node[p];
        if ((node / bs) % int(gridDim.z) != int(blockIdx.z)) continue;  // x of this node was formed elsewhere
        const int64_t tw = int64_t(port_twin[p]) * nrhs + r0;
        const int64_t pa = int64_t(p) * nrhs + r0;
        const int64_t px = int64_t(off + node) * nrhs + r0;
        const TV be = pbeta[p], ga = pgamma[p];
        for (int k = 0; k < w; ++k) a_next[tw + k] = be * (xs_lds ? xs[node * R + k] : x[px + k]) + ga * a_cur[pa + k];
    }
}

// Single right-hand side, forward: the same three steps with the inverse loads
// issued early.  Each thread's first CH column groups are requested before the
// port phase (they do not depend on rhs), and the remaining chunks are double
// buffered, so a wavefront keeps up to 2 * CH * 16 bytes per lane in flight.
template <typename TO, typename TV, int CH>
__global__ void __launch_bounds__(kBlock)
    k_sweep1(const TO* __restrict__ K, const int64_t* __restrict__ kofs, const int32_t* __restrict__ sub_off,
             const int32_t* __restrict__ port_off, const int32_t* __restrict__ port_node,
             const int32_t* __restrict__ port_slot, const int32_t* __restrict__ port_twin,
             const TV* __restrict__ pc, const TV* __restrict__ pbeta, const TV* __restrict__ pgamma,
             const TV* __restrict__ b, const TV* __restrict__ a_cur, TV* __restrict__ a_next, TV* __restrict__ x,
             int max_ns, int max_slot, int xs_lds, int port_rows) {
    constexpr int G = Group<TO>::G;
    extern __shared__ char smem[];
    TV* rhs = reinterpret_cast<TV*>(smem);   // [max_ns]
    TV* xs = rhs + max_ns;                   // [max_ns] when xs_lds (else the waves read x back)
    const int s = xcd_block(blockIdx.x, gridDim.x);
    const int off = sub_off[s];
    const int ns = sub_off[s + 1] - off;
    const int p0 = port_off[s], p1 = port_off[s + 1];
    const int tid = threadIdx.x, bs = blockDim.x;
    // port_rows: only the rows the waves need, the port nodes, which are numbered
    // first in each sub-circuit (its last port's node is the last of them)
    const int nrow = port_rows ? (p1 > p0 ? port_node[p1 - 1] + 1 : 0) : ns;
    const TO* Ks = K + kofs[s];
    const int full = (ns / G) * G;
    const int ngroups = full / G;
    const int nch = (ngroups + CH - 1) / CH;
    // rows of this block: [y * bs, y * bs + bs) + k * bs * gridDim.y (gridDim.y > 1 spreads the
    // rows of a few large sub-circuits over several workgroups)
    const int row0 = int(blockIdx.y) * bs, rstep = bs * int(gridDim.y);
    if (row0 >= nrow) return;  // uniform over the workgroup (its rows, and so its port nodes, are none)

    TO buf0[CH][G], buf1[CH][G];
    auto load_chunk = [&](TO (&buf)[CH][G], int ch, int row) {
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int g = ch * CH + j;
            if (g < ngroups) {
                load16<TO>(Ks + (int64_t(g) * ns + row) * G, buf[j]);
            } else {
#pragma unroll
                for (int q = 0; q < G; ++q) buf[j][q] = TO(0);
            }
        }
    };
    if (row0 + tid < nrow) load_chunk(buf0, 0, row0 + tid);

    for (int t = tid; t < ns; t += bs) rhs[t] = b[off + t];
    __syncthreads();
    for (int pb = p0; pb < p1; pb += bs) {
        const int p = pb + tid;
        const bool ok = p < p1;
        const int node = ok ? port_node[p] : 0;
        const int slot = ok ? port_slot[p] : -1;
        const TV c = ok ? pc[p] : TV(0);
        const TV a = ok ? a_cur[p] : TV(0);
        for (int sl = 0; sl <= max_slot; ++sl) {
            if (slot == sl) rhs[node] += c * a;
            __syncthreads();
        }
    }

    for (int row = row0 + tid; row < nrow; row += rstep) {
        if (row != row0 + tid) load_chunk(buf0, 0, row);
        TV acc[G];
#pragma unroll
        for (int q = 0; q < G; ++q) acc[q] = TV(0);
        auto consume = [&](TO (&buf)[CH][G], int ch) {
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int c0 = (ch * CH + j) * G;
#pragma unroll
                for (int q = 0; q < G; ++q) acc[q] += TV(buf[j][q]) * rhs[min(c0 + q, ns - 1)];
            }
        };
        for (int ch = 0; ch < nch; ch += 2) {
            if (ch + 1 < nch) load_chunk(buf1, ch + 1, row);
            consume(buf0, ch);
            if (ch + 1 < nch) {
                if (ch + 2 < nch) load_chunk(buf0, ch + 2, row);
                consume(buf1, ch + 1);
            }
        }
        for (int c = full; c < ns; ++c)
            acc[0] += TV(Ks[int64_t(full) * ns + int64_t(c - full) * ns + row]) * rhs[c];
        TV v = acc[0];
#pragma unroll
        for (int q = 1; q < G; ++q) v += acc[q];
        if (xs_lds) xs[row] = v;
        x[off + row] = v;
    }
    __syncthreads();
    for (int p = p0 + tid; p < p1; p += bs) {
        const int node = port_node[p];
        if ((node / bs) % int(gridDim.y) == int(blockIdx.y))  // x of this node was formed here
            a_next[port_twin[p]] = pbeta[p] * (xs_lds ? xs[node] : x[off + node]) + pgamma[p] * a_cur[p];
    }
}

template <typename TO, typename TV, int R>
hipError_t launch_r(int S, int max_ns, int nrhs, const TO* K, const int64_t* kofs, const int32_t* sub_off,
                    PortArrays ports, const TV* pc, const TV* pbeta, const TV* pgamma, const TV* b,
                    const TV* a_cur, TV* a_next, TV* x, bool adjoint, bool xs_lds, hipStream_t st) {
    const int bs = max_ns <= 64 ? 64 : kBlock;
    const size_t lds = size_t(xs_lds ? 2 : 1) * max_ns * R * sizeof(TV);
    const unsigned ny = unsigned((nrhs + R - 1) / R);
    // few workgroups in all: the rows of each sub-circuit over several
    const unsigned nz = int64_t(S) * ny < 1024 && max_ns > bs ? unsigned((max_ns + bs - 1) / bs) : 1u;
    if (hipError_t e = raise_lds_limit(reinterpret_cast<const void*>(&k_sweep<TO, TV, R>), lds); e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_sweep<TO, TV, R>), dim3(S, ny, nz), dim3(bs), lds, st, K, kofs, sub_off, ports.off,
                       ports.node, ports.slot, ports.twin, pc, pbeta, pgamma, b, a_cur, a_next, x, nrhs, max_ns,
                       ports.max_slot, adjoint ? 1 : 0, xs_lds ? 1 : 0);
    return hipGetLastError();
}

}  // namespace

template <typename TO, typename TV>
hipError_t launch_sweep(int S, int max_ns, int nrhs, const TO* K, const int64_t* kofs, const int32_t* sub_off,
                        PortArrays ports, const TV* pc, const TV* pbeta, const TV* pgamma, const TV* b,
                        const TV* a_cur, TV* a_next, TV* x, bool adjoint, size_t lds_limit, hipStream_t st,
                        bool port_rows) {
    // right-hand sides per block: rhs and x of the sub-circuit in 64 KiB of LDS; one
    // right-hand side of a larger sub-circuit may use up to lds_limit
    auto fits = [&](int r) { return size_t(2) * max_ns * r * sizeof(TV) <= 65536; };
    // one right-hand side a block also runs with only rhs in LDS (x read back for the waves)
    const bool xs_lds = size_t(2) * max_ns * sizeof(TV) <= lds_limit;
    const bool one = xs_lds || size_t(max_ns) * sizeof(TV) <= lds_limit;
    if (kSweepChunk > 0 && nrhs == 1 && !adjoint && size_t(max_ns) * sizeof(TV) <= lds_limit) {
        // few sub-circuits: one-wavefront blocks, each sub-circuit's rows spread over several
        const bool split = S < 1024 && max_ns > 64;
        const int bs = split || max_ns <= 64 ? 64 : kBlock;
        const int ry = split ? (max_ns + bs - 1) / bs : 1;
        const size_t lds = size_t(xs_lds ? 2 : 1) * max_ns * sizeof(TV);
        constexpr int CH = kSweepChunk > 0 ? kSweepChunk : 1;
        if (hipError_t e = raise_lds_limit(reinterpret_cast<const void*>(&k_sweep1<TO, TV, CH>), lds);
            e != hipSuccess)
            return e;
        hipLaunchKernelGGL((k_sweep1<TO, TV, CH>), dim3(S, ry), dim3(bs), lds, st, K, kofs, sub_off, ports.off,
                           ports.node, ports.slot, ports.twin, pc, pbeta, pgamma, b, a_cur, a_next, x, max_ns,
                           ports.max_slot, xs_lds ? 1 : 0, port_rows ? 1 : 0);
        return hipGetLastError();
    }
    if (nrhs == 1 || !fits(2))
        return one ? launch_r<TO, TV, 1>(S, max_ns, nrhs, K, kofs, sub_off, ports, pc, pbeta, pgamma, b, a_cur,
                                             a_next, x, adjoint, xs_lds, st)
                       : hipErrorInvalidValue;
    if (nrhs == 2 || !fits(4))
        return launch_r<TO, TV, 2>(S, max_ns, nrhs, K, kofs, sub_off, ports, pc, pbeta, pgamma, b, a_cur, a_next,
                                   x, adjoint, true, st);
    if (nrhs <= 4 || !fits(8))
        return launch_r<TO, TV, 4>(S, max_ns, nrhs, K, kofs, sub_off, ports, pc, pbeta, pgamma, b, a_cur, a_next,
                                   x, adjoint, true, st);
    return launch_r<TO, TV, 8>(S, max_ns, nrhs, K, kofs, sub_off, ports, pc, pbeta, pgamma, b, a_cur, a_next, x,
                               adjoint, true, st);
}

template hipError_t launch_sweep<double, double>(int, int, int, const double*, const int64_t*, const int32_t*,
                                                 PortArrays, const double*, const double*, const double*,
                                                 const double*, const double*, double*, double*, bool, size_t,
                                                 hipStream_t, bool);
template hipError_t launch_sweep<float, float>(int, int, int, const float*, const int64_t*, const int32_t*,
                                               PortArrays, const float*, const float*, const float*,
                                               const float*, const float*, float*, float*, bool, size_t,
                                               hipStream_t, bool);

}  // namespace vtm
