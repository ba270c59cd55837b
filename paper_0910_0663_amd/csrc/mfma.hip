// Batched sweep on the matrix cores: for every sub-circuit s,
//   X_s = Kinv_s [b + c * a]_s        (n_s x n_s times n_s x nrhs)
// as a GEMM on MFMA, then the outgoing waves beta * X + gamma * a for every
// port and right-hand side (eq. 11 applied column by column).
//
// Two element types:
//   BF16 inverse x BF16 right-hand sides, FP32 accumulate (v_mfma_f32_16x16x32_bf16),
//        vectors and waves in FP32 (the inner solve of the BF16 refinement);
//   FP64 inverse x FP64 right-hand sides (v_mfma_f64_16x16x4f64), vectors in FP64.
//
// Inverses are stored in A-operand tile order (tiles.hpp): one 16-byte load per
// lane fetches a whole operand, a wavefront's load is 1 KiB contiguous.  The
// right-hand-side block of the sub-circuit is staged once in LDS and feeds the
// B operand.  Each wavefront holds the accumulators of RT 16-row tiles of X and
// walks k: per k tile one LDS read per B fragment serves all RT row tiles, and
// the next k tile's RT A-tiles are in flight while this one's MFMAs issue.
#include "kernels.hpp"
#include "layout.hpp"
#include "tiles.hpp"

namespace vtm {

// batched sweeps: k tiles of A in flight per wavefront (port-to-port FP64, BF16)
constexpr int kMfmaPD64 = 2;
constexpr int kMfmaPD16 = 2;
// full batched sweep: FP64 k tiles of A in flight per wavefront (its inverses are
// up to 72 k tiles long, the port-to-port operators at most 12)
constexpr int kMfmaFullPD64 = 6;
// full batched sweep: right-hand-side items per thread in each round of staging loads
constexpr int kMfmaFullSU = 2;

namespace {

constexpr int kWaves = 8;                 // wavefronts per workgroup
constexpr int kBlock = kWaves * 64;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef double double2v __attribute__((ext_vector_type(2)));

// per element type: A fragment, accumulator, B staging and the MFMA step
template <typename T>
struct Mma;

template <>
struct Mma<__bf16> {
    using TV = float;
    using AFrag = bf16x8;     // 8 bf16: A[m = l%16][k = 8(l/16) .. +7] of a 16 x 32 tile
    using Acc = floatx4;      // D[m = 4(l/16) + v][n = l%16]
    static constexpr int KT = 32;   // k per A tile
    // B staged as rhsT[n][k] (k contiguous), row stride np + 8
    static __device__ int bstride(int np) { return np + 8; }
    static __device__ size_t lds_bytes(int np, int rc) { return size_t(rc) * (np + 8) * sizeof(__bf16); }
    static __device__ void stage(__bf16* sb, int np, int rc, int k, int n, float v) {
        sb[n * (np + 8) + k] = static_cast<__bf16>(v);
    }
    using BFrag = bf16x8;     // B[k = 8(l/16) .. +7][n = l%16] of a 32 x 16 tile
    static __device__ BFrag bfrag(const __bf16* sb, int np, int kt, int nt) {
        const int l = threadIdx.x & 63;
        return *reinterpret_cast<const bf16x8*>(sb + (nt * 16 + (l & 15)) * (np + 8) + kt * 32 + 8 * (l >> 4));
    }
    static __device__ Acc mma(const AFrag& a, const BFrag& b, Acc acc) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    static __device__ int out_row(int l, int v) { return 4 * (l >> 4) + v; }
};

template <>
struct Mma<double> {
    using TV = double;
    using AFrag = double2v;   // A[m = l%16][k = 8kp + l/16] and A[m][k = 8kp + 4 + l/16]
    using Acc = doublex4;     // D[m = (l/16) + 4v][n = l%16]
    static constexpr int KT = 8;
    // B staged as rhs[k][n] (n contiguous), row stride rc
    static __device__ void stage(double* sb, int np, int rc, int k, int n, double v) { sb[k * rc + n] = v; }
    using BFrag = double2v;   // B[k = 8kp + l/16][n = l%16] and B[k + 4][n]
    static __device__ BFrag bfrag(const double* sb, int rc, int kp, int nt) {
        const int l = threadIdx.x & 63;
        const int n = nt * 16 + (l & 15), k = kp * 8 + (l >> 4);
        BFrag b;
        b.x = sb[k * rc + n];
        b.y = sb[(k + 4) * rc + n];
        return b;
    }
    static __device__ Acc mma(const AFrag& a, const BFrag& b, Acc acc) {
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, acc, 0, 0, 0);
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, acc, 0, 0, 0);
    }
    static __device__ int out_row(int l, int v) { return (l >> 4) + 4 * v; }
};

// The GEMM core of the batched sweeps: D = A B for one padded np x np block A
// (tile order, tiles.hpp) and the staged np x w block B in LDS.  A wavefront
// takes up to RT row tiles (mt = wave, wave + W, ...) per pass and walks k: per
// k tile it loads the NT B fragments once from LDS and its row tiles' A tiles
// from HBM (the next k tile's A tiles are already in flight), then issues the
// MFMAs.  epi(row, n, value) receives every element of D (rows < np, n < 16 NT);
// mt_lim >= 0 forms only the first mt_lim row tiles.
template <typename T, int NT, int RT, int WAVES, int PD64 = kMfmaPD64, typename Epi>
__device__ inline void tile_gemm(const T* Ablk, int np, const T* sb, int bsel, int w, Epi epi, int mt_lim = -1) {
    using M = Mma<T>;
    using TV = typename M::TV;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int MT = mt_lim >= 0 ? min(np / 16, mt_lim) : np / 16, KT = np / M::KT;
    const typename M::AFrag* A0 = reinterpret_cast<const typename M::AFrag*>(Ablk) + lane;
    for (int g0 = 0; g0 < MT; g0 += WAVES * RT) {
        int mts[RT];
        int nmy = 0;
#pragma unroll
        for (int j = 0; j < RT; ++j) {
            mts[j] = g0 + wave + j * WAVES;
            if (mts[j] < MT) nmy = j + 1;
        }
        if (nmy == 0) continue;
        typename M::Acc acc[RT][NT];
#pragma unroll
        for (int j = 0; j < RT; ++j)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[j][nt][v] = 0;
        // ring of PD k tiles: tile k sits in abuf[k % PD]; the loads run PD - 1 tiles ahead
        constexpr int PD = sizeof(T) == 8 ? PD64 : kMfmaPD16;
        typename M::AFrag abuf[PD][RT];
#pragma unroll
        for (int d = 0; d < PD - 1; ++d)
#pragma unroll
            for (int j = 0; j < RT; ++j)
                if (j < nmy && d < KT) abuf[d][j] = A0[(int64_t(mts[j]) * KT + d) * 64];
        for (int kt = 0; kt < KT; kt += PD) {
#pragma unroll
            for (int h = 0; h < PD; ++h) {
                const int k = kt + h;
                if (k < KT) {
                    if (k + PD - 1 < KT) {
#pragma unroll
                        for (int j = 0; j < RT; ++j)
                            if (j < nmy) abuf[(h + PD - 1) % PD][j] = A0[(int64_t(mts[j]) * KT + k + PD - 1) * 64];
                    }
                    typename M::BFrag bf[NT];
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) bf[nt] = M::bfrag(sb, bsel, k, nt);
#pragma unroll
                    for (int j = 0; j < RT; ++j)
                        if (j < nmy)
#pragma unroll
                            for (int nt = 0; nt < NT; ++nt)
                                if (nt * 16 < w) acc[j][nt] = M::mma(abuf[h][j], bf[nt], acc[j][nt]);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < RT; ++j) {
            if (j >= nmy) continue;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    epi(mts[j] * 16 + M::out_row(lane, v), nt * 16 + (lane & 15), TV(acc[j][nt][v]),
                        (j * NT + nt) * 4 + v);
        }
    }
}

// Block (y, s): sub-circuit s, right-hand sides [r0, r0 + w), w <= rc <= 16 * NT.
// TB: element type of the right-hand side b (BF16 for the BF16 path: the staged
// operand is BF16 anyway).  write_x = 0 stores x only on port rows (all the
// wave update needs); the last sweep before a residual check passes 1.
template <typename T, typename TB, int NT, int RT>
__global__ void __launch_bounds__(kBlock)
    k_sweep_mfma(const T* __restrict__ K, const int64_t* __restrict__ mofs, const int32_t* __restrict__ sub_off,
                 const int32_t* __restrict__ port_off, const int32_t* __restrict__ port_node,
                 const int32_t* __restrict__ port_twin, const typename Mma<T>::TV* __restrict__ pc,
                 const typename Mma<T>::TV* __restrict__ pbeta, const typename Mma<T>::TV* __restrict__ pgamma,
                 const TB* __restrict__ b, const typename Mma<T>::TV* __restrict__ a_cur,
                 typename Mma<T>::TV* __restrict__ a_next, typename Mma<T>::TV* __restrict__ x, int nrhs, int rc,
                 int write_x, int S, int port_rows) {
    using M = Mma<T>;
    using TV = typename M::TV;
    extern __shared__ char smem[];
    T* sb = reinterpret_cast<T*>(smem);
    // sub-circuits dealt to the XCDs in turn, the column blocks of one sub-circuit
    // (which read its inverse) consecutive on one XCD's L2
    const int u = xcd_item_block(int(blockIdx.x + gridDim.x * blockIdx.y), S, int(gridDim.x), false);
    if (u < 0) return;  // uniform over the workgroup
    const int s = u / int(gridDim.x);
    const int r0 = (u - s * int(gridDim.x)) * rc;
    const int w = min(rc, nrhs - r0);
    const int off = sub_off[s];
    const int ns = sub_off[s + 1] - off;
    const int np = tile_pad(ns);
    const int p0 = port_off[s], p1 = port_off[s + 1];
    const int tid = threadIdx.x;

    // 1. stage B = b + c * a.  Ports of a node are consecutive (slot order);
    //    pfirst/pcount give each row its port range.  b is read V values at a time.
    constexpr int V = 16 / int(sizeof(TB));
    int* pnode = reinterpret_cast<int*>(smem + tile_lds_bytes<T>(np, rc));
    const int nps = p1 - p0;
    short* pfirst = reinterpret_cast<short*>(pnode + nps);
    unsigned char* pcount = reinterpret_cast<unsigned char*>(pfirst + np);
    for (int k = tid; k < np; k += kBlock) pcount[k] = 0;
    for (int p = p0 + tid; p < p1; p += kBlock) pnode[p - p0] = port_node[p];
    __syncthreads();
    for (int q = tid; q < nps; q += kBlock) {
        const int k = pnode[q];
        if (q == 0 || pnode[q - 1] != k) {
            int e = q;
            while (e < nps && pnode[e] == k) ++e;
            pfirst[k] = short(q);
            pcount[k] = static_cast<unsigned char>(e - q);
        }
    }
    __syncthreads();
    const bool vec = (nrhs % V) == 0;
    const int rv = rc / V;
    if (vec) {
        // SU items per thread per round; each item's b load is waited on only after
        // its ports' loads are issued (b is added last), so a round costs about one
        // HBM round trip
        constexpr int SU = kMfmaFullSU;
        const int tot = np * rv;
        for (int t0 = tid; t0 < tot; t0 += SU * kBlock) {
            TB bv[SU][V];
            TV acc[SU][V];
#pragma unroll
            for (int i = 0; i < SU; ++i) {
                const int t = t0 + i * kBlock;
                const int k = t / rv, n0 = (t - k * rv) * V;
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    bv[i][j] = TB(0);
                    acc[i][j] = TV(0);
                }
                if (t < tot && k < ns && n0 < w)
                    *reinterpret_cast<uint4*>(bv[i]) =
                        *reinterpret_cast<const uint4*>(b + int64_t(off + k) * nrhs + r0 + n0);
            }
#pragma unroll
            for (int i = 0; i < SU; ++i) {
                const int t = t0 + i * kBlock;
                const int k = t / rv, n0 = (t - k * rv) * V;
                if (t < tot && k < ns && n0 < w) {
                    const int cnt = pcount[k];
                    for (int q = 0; q < cnt; ++q) {
                        const int p = p0 + pfirst[k] + q;
                        const TV c = pc[p];
                        const TV* ap = a_cur + int64_t(p) * nrhs + r0 + n0;
#pragma unroll
                        for (int j = 0; j < V; ++j) acc[i][j] += c * ap[j];
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < SU; ++i) {
                const int t = t0 + i * kBlock;
                const int k = t / rv, n0 = (t - k * rv) * V;
                if (t < tot) {
#pragma unroll
                    for (int j = 0; j < V; ++j) M::stage(sb, np, rc, k, n0 + j, TV(bv[i][j]) + acc[i][j]);
                }
            }
        }
    } else
    for (int t = tid; t < np * rv; t += kBlock) {
        const int k = t / rv, n0 = (t - k * rv) * V;
        TV v[V];
#pragma unroll
        for (int j = 0; j < V; ++j) v[j] = TV(0);
        if (k < ns && n0 < w) {
            const TB* bp = b + int64_t(off + k) * nrhs + r0 + n0;
            if (vec) {
                TB tmp[V];
                *reinterpret_cast<uint4*>(tmp) = *reinterpret_cast<const uint4*>(bp);
#pragma unroll
                for (int j = 0; j < V; ++j) v[j] = TV(tmp[j]);
            } else {
#pragma unroll
                for (int j = 0; j < V; ++j)
                    if (n0 + j < w) v[j] = TV(bp[j]);
            }
            const int cnt = pcount[k];
            for (int q = 0; q < cnt; ++q) {
                const int p = p0 + pfirst[k] + q;
                const TV c = pc[p];
                const TV* ap = a_cur + int64_t(p) * nrhs + r0 + n0;
#pragma unroll
                for (int j = 0; j < V; ++j)
                    if (n0 + j < w) v[j] += c * ap[j];
            }
        }
#pragma unroll
        for (int j = 0; j < V; ++j) M::stage(sb, np, rc, k, n0 + j, v[j]);
    }
    __syncthreads();

    // 2. X = Kinv B, x stored on the rows the wave update reads (all rows with write_x)
    // (the full inverses are long in k: FP64 keeps more of its tiles in flight);
    // port_rows: only the row tiles of the port nodes, numbered first (the last
    // port's node is the last of them)
    const int mt_lim = port_rows ? (nps > 0 ? pnode[nps - 1] + 16 : 0) / 16 : -1;
    tile_gemm<T, NT, RT, kWaves, kMfmaFullPD64>(K + mofs[s], np, sb, sizeof(T) == 2 ? np : rc, w,
                                                     [&](int row, int n, TV v, int) {
        if (row < ns && n < w && (write_x || pcount[row])) x[int64_t(off + row) * nrhs + r0 + n] = v;
    }, mt_lim);
    __syncthreads();

    // 3. outgoing waves, read back x of the port nodes (written by this workgroup), 4 columns at a time
    const int w4 = (w + 3) / 4;
    if (nrhs % 4 == 0) {
        // whole 4-column chunks (w is a multiple of 4), two per thread per round, all
        // loads of a round issued before its stores
        struct alignas(16) C4 {
            TV e[4];
        };
        constexpr int SU = 2;
        const int tot = nps * w4;
        for (int t0 = tid; t0 < tot; t0 += SU * kBlock) {
            C4 xv[SU], av[SU];
            TV be[SU], ga[SU];
            int tw[SU];
#pragma unroll
            for (int i = 0; i < SU; ++i) {
                const int t = t0 + i * kBlock;
                if (t < tot) {
                    const int q = t / w4, n0 = (t - q * w4) * 4;
                    const int p = p0 + q;
                    be[i] = pbeta[p];
                    ga[i] = pgamma[p];
                    tw[i] = port_twin[p];
                    xv[i] = *reinterpret_cast<const C4*>(x + int64_t(off + pnode[q]) * nrhs + r0 + n0);
                    av[i] = *reinterpret_cast<const C4*>(a_cur + int64_t(p) * nrhs + r0 + n0);
                }
            }
#pragma unroll
            for (int i = 0; i < SU; ++i) {
                const int t = t0 + i * kBlock;
                if (t < tot) {
                    const int q = t / w4, n0 = (t - q * w4) * 4;
                    C4 o;
#pragma unroll
                    for (int j = 0; j < 4; ++j) o.e[j] = be[i] * xv[i].e[j] + ga[i] * av[i].e[j];
                    *reinterpret_cast<C4*>(a_next + int64_t(tw[i]) * nrhs + r0 + n0) = o;
                }
            }
        }
    } else
    for (int t = tid; t < nps * w4; t += kBlock) {
        const int q = t / w4, n0 = (t - q * w4) * 4;
        const int p = p0 + q;
        const TV be = pbeta[p], ga = pgamma[p];
        const TV* xr = x + int64_t(off + pnode[q]) * nrhs + r0;
        const TV* ar = a_cur + int64_t(p) * nrhs + r0;
        TV* nr = a_next + int64_t(port_twin[p]) * nrhs + r0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (n0 + j < w) nr[n0 + j] = be * xr[n0 + j] + ga * ar[n0 + j];
    }
}

// Batched port-to-port sweep (the Appendix's interface-only iteration, eqs.
// 23-26, for many right-hand sides): block (y, s) forms
//   a_next[twin(p)][r] = h[p][r] + sum_p' M_s[p][p'] a_cur[p'][r]
// for the ports p of sub-circuit s and right-hand sides [r0, r0 + w).  M_s
// (q x q, zero-padded to qp = roundup(q, 32)) is stored in A-tile order; the
// block of incident waves is staged in LDS as the B operand (BF16 for the BF16
// path, FP32 accumulate).  WAVES wavefronts per workgroup (the operators are
// small: 64 ports make four 16-row tiles).
template <typename T, int NT, int RT, int WAVES, bool HL>
__global__ void __launch_bounds__(WAVES * 64)
    k_sweep_mfma_pp(const T* __restrict__ Mop, const int64_t* __restrict__ qmofs,
                    const int32_t* __restrict__ port_off, const int32_t* __restrict__ port_twin,
                    const typename Mma<T>::TV* __restrict__ h, const typename Mma<T>::TV* __restrict__ a_cur,
                    typename Mma<T>::TV* __restrict__ a_next, int nrhs, int rc, int reverse, int S) {
    using M = Mma<T>;
    using TV = typename M::TV;
    extern __shared__ char smem[];
    T* sb = reinterpret_cast<T*>(smem);
    // logical block u = (sub-circuit, column block), the column blocks of one
    // sub-circuit (which read the same operator) consecutive on one XCD's L2; every
    // other sweep walks each XCD's sub-circuits backwards (what the previous sweep read
    // last is still in the memory-side cache).  FP64: sub-circuits dealt to the XCDs in
    // turn, so that their uneven costs spread over the chip (grid S rounded up to a
    // multiple of 8); BF16: each XCD a contiguous range (grid S), measured faster there.
    const int b = int(blockIdx.x + gridDim.x * blockIdx.y);
    int u;
    if constexpr (sizeof(T) == 2) {
        const int nb = int(gridDim.x * gridDim.y);
        u = reverse ? xcd_block_reversed(b, nb) : xcd_block(b, nb);
    } else {
        u = xcd_item_block(b, S, int(gridDim.x), reverse != 0);
        if (u < 0) return;  // uniform over the workgroup
    }
    const int s = u / int(gridDim.x);
    const int r0 = (u - s * int(gridDim.x)) * rc;
    const int w = min(rc, nrhs - r0);
    const int p0 = port_off[s], q = port_off[s + 1] - p0;
    const int qp = tile_pad(q);
    const int tid = threadIdx.x;
    // FP64: h of the outputs this lane will produce, loaded into registers before the
    // product so that the epilogue does not wait on it (when one pass of row tiles
    // covers the operator); BF16 stages h in LDS instead (registers cost occupancy)
    const int lane = tid & 63, wave = tid >> 6;
    constexpr bool kPre = sizeof(T) == 8;
    const bool one = qp / 16 <= WAVES * RT;   // one pass of row tiles covers the operator
    const bool pre = kPre && one;
    TV hreg[kPre ? RT * NT * 4 : 1];
#pragma unroll
    for (int j = 0; j < (kPre ? RT : 0); ++j)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = (wave + j * WAVES) * 16 + M::out_row(lane, v), n = nt * 16 + (lane & 15);
                hreg[(j * NT + nt) * 4 + v] =
                    pre && row < q && n < w ? h[int64_t(p0 + row) * nrhs + r0 + n] : TV(0);
            }
    // twin port of each output row, loaded before the product (one pass of row tiles)
    int twr[RT * 4];
#pragma unroll
    for (int j = 0; j < RT; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = (wave + j * WAVES) * 16 + M::out_row(lane, v);
            twr[j * 4 + v] = one && row < q ? port_twin[p0 + row] : 0;
        }
    // BF16 (HL): h of this block staged in LDS beside the waves (its loads overlap
    // theirs); the launch drops HL when there is no room for it (very large operators)
    constexpr bool hl = HL && sizeof(T) == 2;
    const int hst = rc + 16;
    TV* hs = reinterpret_cast<TV*>(smem + tile_lds_bytes<T>(qp, rc));
    const int sst = pp_stage_stride<T>(qp, rc);
    // incident waves (and h) of rows k < qp: 16-byte loads when every row segment is
    // 16-byte aligned (nrhs a multiple of the vector width; r0 and w are then too)
    constexpr int VW = 16 / sizeof(TV);
    struct alignas(16) Vec {
        TV e[VW];
    };
    if (nrhs % VW == 0) {
        // SU vectors per thread per round: all loads of a round are issued before its
        // LDS stores, so a round costs one HBM round trip
        constexpr int SU = 4;
        const int rv = rc / VW, tot = qp * rv;
        for (int t0 = tid; t0 < tot; t0 += SU * WAVES * 64) {
            Vec v[SU], hv[SU];
#pragma unroll
            for (int i = 0; i < SU; ++i) {
#pragma unroll
                for (int j = 0; j < VW; ++j) v[i].e[j] = hv[i].e[j] = TV(0);
                const int t = t0 + i * WAVES * 64;
                const int k = t / rv, n = (t - k * rv) * VW;
                if (t < tot && k < q && n < w) {
                    const int64_t o = int64_t(p0 + k) * nrhs + r0 + n;
                    v[i] = *reinterpret_cast<const Vec*>(a_cur + o);
                    if (hl) hv[i] = *reinterpret_cast<const Vec*>(h + o);
                }
            }
#pragma unroll
            for (int i = 0; i < SU; ++i) {
                const int t = t0 + i * WAVES * 64;
                const int k = t / rv, n = (t - k * rv) * VW;
                if (t < tot) {
#pragma unroll
                    for (int j = 0; j < VW; ++j) M::stage(sb, qp, sst, k, n + j, v[i].e[j]);
                    if (hl) *reinterpret_cast<Vec*>(hs + k * hst + n) = hv[i];
                }
            }
        }
    } else {
        for (int t = tid; t < qp * rc; t += WAVES * 64) {
            const int k = t / rc, n = t - k * rc;
            const bool in = k < q && n < w;
            const int64_t o = int64_t(p0 + k) * nrhs + r0 + n;
            M::stage(sb, qp, sst, k, n, in ? a_cur[o] : TV(0));
            if (hl) hs[k * hst + n] = in ? h[o] : TV(0);
        }
    }
    __syncthreads();
    // epilogue with the twin ports (and, FP64, h) already in registers: one pass of
    // row tiles; idx indexes the register arrays statically once inlined
    auto epi_reg = [&](int row, int n, TV v, int idx) __attribute__((always_inline)) {
        if (row < q && n < w) {
            const TV hv = hl ? hs[row * hst + n] : kPre ? hreg[kPre ? idx : 0] : h[int64_t(p0 + row) * nrhs + r0 + n];
            a_next[int64_t(twr[(idx / (NT * 4)) * 4 + (idx & 3)]) * nrhs + r0 + n] = v + hv;
        }
    };
    // several passes of row tiles: twin ports and h read at the store
    auto epi_mem = [&](int row, int n, TV v, int) __attribute__((always_inline)) {
        if (row < q && n < w) {
            const int p = p0 + row;
            const TV hv = hl ? hs[row * hst + n] : h[int64_t(p) * nrhs + r0 + n];
            a_next[int64_t(port_twin[p]) * nrhs + r0 + n] = v + hv;
        }
    };
    if (one)
        tile_gemm<T, NT, RT, WAVES>(Mop + qmofs[s], qp, sb, sizeof(T) == 2 ? qp : sst, w, epi_reg);
    else
        tile_gemm<T, NT, RT, WAVES>(Mop + qmofs[s], qp, sb, sizeof(T) == 2 ? qp : sst, w, epi_mem);
}

// M_s = diag(beta) Kinv[P, P] diag(c) + diag(gamma) in A-tile order, from the
// FP64 inverses (column-major at kofs[s]) that the batched setup leaves in scratch.
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_port_matrix_tiles(const int32_t* __restrict__ sub_off, const int64_t* __restrict__ kofs,
                        const int32_t* __restrict__ port_off, const int32_t* __restrict__ port_node,
                        const double* __restrict__ pc, const double* __restrict__ pbeta,
                        const double* __restrict__ pgamma, const double* __restrict__ Kinv,
                        const int64_t* __restrict__ qmofs, T* __restrict__ out, Coupling<double> B) {
    const int s = blockIdx.x;
    const int ns = sub_off[s + 1] - sub_off[s];
    const int p0 = port_off[s], q = port_off[s + 1] - p0;
    const int qp = tile_pad(q);
    const double* Ks = Kinv + kofs[s];
    T* o = out + qmofs[s];
    const int64_t cnt = int64_t(qp) * qp;
    for (int64_t d = threadIdx.x; d < cnt; d += blockDim.x) {
        int r, c;
        tile_rc<T>(qp, d, r, c);
        double v = 0.0;
        if (r < q && c < q) {
            const int i = port_node[p0 + r], j = port_node[p0 + c];
            if (B.row) {  // (B Kinv[P, P])_{r c} with B's row r over this sub-circuit's ports
                for (int k = B.row[p0 + r]; k < B.row[p0 + r + 1]; ++k)
                    v += B.val[k] * Ks[int64_t(j) * ns + port_node[B.col[k]]];
                v *= pc[p0 + c];
            } else {
                v = pbeta[p0 + r] * Ks[int64_t(j) * ns + i] * pc[p0 + c];
            }
            if (r == c) v += pgamma[p0 + r];
        }
        o[d] = static_cast<T>(v);
    }
}

template <typename T, int NT, int RT, int WAVES, bool HL>
hipError_t launch_pp_k(int S, int nrhs, int rc, size_t lds, const T* Mop, const int64_t* qmofs,
                       const int32_t* port_off, const int32_t* port_twin, const typename Mma<T>::TV* h,
                       const typename Mma<T>::TV* a_cur, typename Mma<T>::TV* a_next, int reverse, hipStream_t st) {
    auto kern = k_sweep_mfma_pp<T, NT, RT, WAVES, HL>;
    if (hipError_t e = raise_lds_limit(reinterpret_cast<const void*>(kern), lds); e != hipSuccess) return e;
    const unsigned ny = unsigned((nrhs + rc - 1) / rc);
    // FP64: S rounded up to a multiple of 8, every XCD taking whole sub-circuits in turn
    const unsigned gy = sizeof(T) == 2 ? unsigned(S) : unsigned((S + 7) / 8 * 8);
    hipLaunchKernelGGL(kern, dim3(ny, gy), dim3(WAVES * 64), lds, st, Mop, qmofs, port_off, port_twin, h, a_cur,
                       a_next, nrhs, rc, reverse, S);
    return hipGetLastError();
}

// h in LDS (BF16) is a compile-time choice: as a run-time one the epilogue read h
// through generic (flat) addresses
template <typename T, int NT, int RT, int WAVES>
hipError_t launch_pp_t(int S, int nrhs, int rc, size_t lds, const T* Mop, const int64_t* qmofs,
                       const int32_t* port_off, const int32_t* port_twin, const typename Mma<T>::TV* h,
                       const typename Mma<T>::TV* a_cur, typename Mma<T>::TV* a_next, int reverse, int h_lds,
                       hipStream_t st) {
    if constexpr (sizeof(T) == 2)
        if (h_lds)
            return launch_pp_k<T, NT, RT, WAVES, true>(S, nrhs, rc, lds, Mop, qmofs, port_off, port_twin, h, a_cur,
                                                       a_next, reverse, st);
    return launch_pp_k<T, NT, RT, WAVES, false>(S, nrhs, rc, lds, Mop, qmofs, port_off, port_twin, h, a_cur, a_next,
                                                reverse, st);
}

template <typename T, int NT, int RT>
hipError_t launch_t(int S, int nrhs, int rc, size_t lds, const T* K, const int64_t* mofs, const int32_t* sub_off,
                    PortArrays ports, const typename Mma<T>::TV* pc, const typename Mma<T>::TV* pbeta,
                    const typename Mma<T>::TV* pgamma, const typename MfmaTypes<T>::TB* b,
                    const typename Mma<T>::TV* a_cur, typename Mma<T>::TV* a_next, typename Mma<T>::TV* x,
                    bool write_x, hipStream_t st, bool port_rows) {
    auto kern = k_sweep_mfma<T, typename MfmaTypes<T>::TB, NT, RT>;
    if (hipError_t e = raise_lds_limit(reinterpret_cast<const void*>(kern), lds); e != hipSuccess) return e;
    const unsigned ny = unsigned((nrhs + rc - 1) / rc);
    hipLaunchKernelGGL(kern, dim3(ny, unsigned((S + 7) / 8 * 8)), dim3(kBlock), lds, st, K, mofs, sub_off, ports.off,
                       ports.node, ports.twin, pc, pbeta, pgamma, b, a_cur, a_next, x, nrhs, rc, write_x ? 1 : 0, S,
                       port_rows ? 1 : 0);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_sweep_mfma(int S, int max_ns, int max_ports, int nrhs, int variant, int rc_req, size_t lds_limit,
                             const T* K,
                             const int64_t* mofs, const int32_t* sub_off, PortArrays ports,
                             const typename MfmaTypes<T>::TV* pc, const typename MfmaTypes<T>::TV* pbeta,
                             const typename MfmaTypes<T>::TV* pgamma, const typename MfmaTypes<T>::TB* b,
                             const typename MfmaTypes<T>::TV* a_cur, typename MfmaTypes<T>::TV* a_next,
                             typename MfmaTypes<T>::TV* x, bool write_x, hipStream_t st, bool port_rows) {
    const int np = tile_pad(max_ns);
    // widest right-hand-side block (a multiple of 16, at most 64) whose staging fits the LDS limit
    int rc = rc_req > 0 ? ((rc_req + 15) / 16) * 16 : 64;
    if (rc > 64) rc = 64;
    // staged B, the port-node list, and per row its first port (short) and port count (byte)
    auto need = [&](int r) { return tile_lds_bytes<T>(np, r) + size_t(max_ports) * 4 + size_t(np) * 3 + 4; };
    while (rc > 16 && need(rc) > lds_limit) rc -= 16;
    const size_t lds = need(rc);
    if (lds > lds_limit) return hipErrorInvalidValue;
    if (rc > nrhs) rc = ((nrhs + 15) / 16) * 16 < rc ? ((nrhs + 15) / 16) * 16 : rc;
    const int nt = (rc + 15) / 16;
    // variant 0: 3 row tiles per wavefront pass, 1: 5, 2: 1 (fewer registers, more wavefronts)
#define VTM_MFMA_CASE(NTV)                                                                                      \
    if (nt == NTV) {                                                                                            \
        if (variant == 2)                                                                                       \
            return launch_t<T, NTV, 1>(S, nrhs, rc, lds, K, mofs, sub_off, ports, pc, pbeta, pgamma, b, a_cur,  \
                                       a_next, x, write_x, st, port_rows);                                      \
        return variant == 1 ? launch_t<T, NTV, 5>(S, nrhs, rc, lds, K, mofs, sub_off, ports, pc, pbeta, pgamma, \
                                                  b, a_cur, a_next, x, write_x, st, port_rows)                  \
                            : launch_t<T, NTV, 3>(S, nrhs, rc, lds, K, mofs, sub_off, ports, pc, pbeta, pgamma, \
                                                  b, a_cur, a_next, x, write_x, st, port_rows);                 \
    }
    VTM_MFMA_CASE(1)
    VTM_MFMA_CASE(2)
    VTM_MFMA_CASE(3)
    VTM_MFMA_CASE(4)
#undef VTM_MFMA_CASE
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_sweep_mfma_pp(int S, int max_ports, int nrhs, int variant, int rc_req, size_t lds_limit,
                                const T* Mop, const int64_t* qmofs, const int32_t* port_off,
                                const int32_t* port_twin, const typename MfmaTypes<T>::TV* h,
                                const typename MfmaTypes<T>::TV* a_cur, typename MfmaTypes<T>::TV* a_next,
                                int reverse, hipStream_t st) {
    const int qp = tile_pad(max_ports);
    int rc = rc_req > 0 ? ((rc_req + 15) / 16) * 16 : 64;
    if (rc > 64) rc = 64;
    // h in LDS when some block width fits with it, else read at the store
    const int h_lds = pp_lds_bytes<T>(qp, 16, true) <= lds_limit ? 1 : 0;
    while (rc > 16 && pp_lds_bytes<T>(qp, rc, h_lds) > lds_limit) rc -= 16;
    const size_t lds = pp_lds_bytes<T>(qp, rc, h_lds);
    if (lds > lds_limit) return hipErrorInvalidValue;
    if (rc > nrhs) rc = ((nrhs + 15) / 16) * 16 < rc ? ((nrhs + 15) / 16) * 16 : rc;
    const int nt = (rc + 15) / 16;
    // variant: bit 0 = 5 row tiles per pass (else 3), bit 1 = 8 wavefronts per workgroup (else 4),
    // bit 2 = 1 row tile per pass (small operators: fewer registers, more wavefronts in flight)
    const bool deep = (variant & 1) != 0, wide = (variant & 2) != 0, thin = (variant & 4) != 0;
#define VTM_MFMA_PP_CASE(NTV)                                                                                    \
    if (nt == NTV) {                                                                                             \
        if (thin)                                                                                                \
            return wide ? launch_pp_t<T, NTV, 1, 8>(S, nrhs, rc, lds, Mop, qmofs, port_off, port_twin, h, a_cur,   \
                                                    a_next, reverse, h_lds, st)                                         \
                        : launch_pp_t<T, NTV, 1, 4>(S, nrhs, rc, lds, Mop, qmofs, port_off, port_twin, h, a_cur,   \
                                                    a_next, reverse, h_lds, st);                                        \
        if (wide)                                                                                                \
            return deep ? launch_pp_t<T, NTV, 5, 8>(S, nrhs, rc, lds, Mop, qmofs, port_off, port_twin, h, a_cur,   \
                                                    a_next, reverse, h_lds, st)                                         \
                        : launch_pp_t<T, NTV, 3, 8>(S, nrhs, rc, lds, Mop, qmofs, port_off, port_twin, h, a_cur,   \
                                                    a_next, reverse, h_lds, st);                                        \
        return deep ? launch_pp_t<T, NTV, 5, 4>(S, nrhs, rc, lds, Mop, qmofs, port_off, port_twin, h, a_cur,       \
                                                a_next, reverse, h_lds, st)                                             \
                    : launch_pp_t<T, NTV, 3, 4>(S, nrhs, rc, lds, Mop, qmofs, port_off, port_twin, h, a_cur,       \
                                                a_next, reverse, h_lds, st);                                            \
    }
    VTM_MFMA_PP_CASE(1)
    VTM_MFMA_PP_CASE(2)
    VTM_MFMA_PP_CASE(3)
    VTM_MFMA_PP_CASE(4)
#undef VTM_MFMA_PP_CASE
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_port_matrix_tiles(int S, const int32_t* sub_off, const int64_t* kofs, const int32_t* port_off,
                                    const int32_t* port_node, const double* pc, const double* pbeta,
                                    const double* pgamma, const double* Kinv, const int64_t* qmofs, T* out,
                                    hipStream_t st, Coupling<double> B) {
    hipLaunchKernelGGL(k_port_matrix_tiles<T>, dim3(S), dim3(kBlock), 0, st, sub_off, kofs, port_off, port_node, pc,
                       pbeta, pgamma, Kinv, qmofs, out, B);
    return hipGetLastError();
}

template hipError_t launch_sweep_mfma_pp<__bf16>(int, int, int, int, int, size_t, const __bf16*, const int64_t*,
                                                const int32_t*, const int32_t*, const float*, const float*, float*,
                                                int, hipStream_t);
template hipError_t launch_sweep_mfma_pp<double>(int, int, int, int, int, size_t, const double*, const int64_t*,
                                                const int32_t*, const int32_t*, const double*, const double*,
                                                double*, int, hipStream_t);
template hipError_t launch_port_matrix_tiles<__bf16>(int, const int32_t*, const int64_t*, const int32_t*,
                                                    const int32_t*, const double*, const double*, const double*,
                                                    const double*, const int64_t*, __bf16*, hipStream_t,
                                                    Coupling<double>);
template hipError_t launch_port_matrix_tiles<double>(int, const int32_t*, const int64_t*, const int32_t*,
                                                    const int32_t*, const double*, const double*, const double*,
                                                    const double*, const int64_t*, double*, hipStream_t,
                                                    Coupling<double>);
template hipError_t launch_sweep_mfma<__bf16>(int, int, int, int, int, int, size_t, const __bf16*, const int64_t*,
                                             const int32_t*, PortArrays, const float*, const float*, const float*,
                                             const __bf16*, const float*, float*, float*, bool, hipStream_t,
                                             bool);
template hipError_t launch_sweep_mfma<double>(int, int, int, int, int, int, size_t, const double*, const int64_t*,
                                             const int32_t*, PortArrays, const double*, const double*,
                                             const double*, const double*, const double*, double*, double*, bool,
                                             hipStream_t, bool);

}  // namespace vtm
