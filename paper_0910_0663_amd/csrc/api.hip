// C ABI: handle lifetime, setup, the solve driver and the adjoint/gradient calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <type_traits>
#include <array>
#include <chrono>
#include <map>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"
#include "status.hpp"
#include "vtm.h"

namespace {

using vtm::fail;

#define VTM_HIP(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(e_ == hipErrorOutOfMemory ? VTM_E_OOM : VTM_E_HIP,                         \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                        \
    } while (0)

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t count = 0;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    // a buffer of n elements; one of that size already held is kept (refresh
    // re-runs setup's uploads on buffers of unchanged sizes)
    hipError_t alloc(size_t n) {
        if (p && n == count) return hipSuccess;
        reset();
        count = n;
        return hipMalloc(reinterpret_cast<void**>(&p), (n ? n : 1) * sizeof(T));
    }
    void reset() {
        if (p) (void)hipFree(p);
        p = nullptr;
        count = 0;
    }
    template <typename Alloc>
    hipError_t upload(const std::vector<T, Alloc>& v, hipStream_t st) {
        hipError_t e = alloc(v.size());
        if (e != hipSuccess || v.empty()) return e;
        return hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
    }
};

template <typename Alloc>
std::vector<float> to_float(const std::vector<double, Alloc>& v) {
    return std::vector<float>(v.begin(), v.end());
}

}  // namespace

// Workspace of vtm_solve_noalloc, one copy per device, held until the process
// ends: the residual reductions' per-workgroup partial sums (kResidBlocks
// workgroups x kNoallocRhs columns x 2 sums; the per-column sums go to the
// handle's pinned host buffer as in vtm_solve).  Every check writes all of what
// it then reads, so nothing needs clearing between calls.  Host code never passes this name to a kernel:
// it is a host-side stand-in; scratch_address() gives the device address.
constexpr int kNoallocRhs = 64;
constexpr size_t kNoallocDoubles = size_t(vtm::kResidBlocks) * kNoallocRhs * 2;
static __device__ __align__(256) double scratch[kNoallocDoubles];

namespace {

std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_addr;  // device -> address of its copy of `scratch`

// The address of `scratch` on device dev (which must be current), looked up
// once per device.
vtm_status scratch_address(int dev, double** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it == g_scratch_addr.end()) {
        void* p = nullptr;
        VTM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(VTM_E_HIP, "hipGetSymbolAddress returned no address for the static workspace");
        it = g_scratch_addr.emplace(dev, static_cast<double*>(p)).first;
    }
    *out = it->second;
    return VTM_OK;
}

}  // namespace

namespace {

// Launch shapes the autotuner chose, per process, keyed by the device and what
// the timing depends on: precision, right-hand sides, forced shape options and
// the plan's sizes.  A setup with the same key takes the cached shapes.
struct TuneKey {
    int device, precision, nrhs, rows, rc;
    int64_t S, n, nports, entries, port_entries;
    int max_ns, max_ports;
    bool operator<(const TuneKey& o) const {
        return std::tie(device, precision, nrhs, rows, rc, S, n, nports, entries, port_entries, max_ns, max_ports) <
               std::tie(o.device, o.precision, o.nrhs, o.rows, o.rc, o.S, o.n, o.nports, o.entries, o.port_entries,
                        o.max_ns, o.max_ports);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::array<int, 4>> g_tune;  // mfma variant, mfma rc, pp variant, pp rc

}  // namespace

struct vtm_handle_s {
    int device = 0;
    hipStream_t stream = nullptr;
    vtm_options opt{};
    vtm::Plan plan;
    int nrhs_max = 1;

    // untorn renumbered matrix, and its transpose when A is not symmetric
    DevBuf<int32_t> rowptr, col, rowptrT, colT;
    DevBuf<double> val, valT;
    // sub-circuits and ports
    DevBuf<int32_t> perm, iperm, sub_off, port_off, port_node, port_slot, port_twin, abi2port;
    DevBuf<int64_t> kofs;
    DevBuf<double> dmod;
    DevBuf<double> c64, beta64, gamma64;
    DevBuf<float> c32, beta32, gamma32;
    // stored inverses: column groups (K64 / K32), or MFMA tiles (K64 / Kbf) when tiles is set
    DevBuf<double> K64;
    DevBuf<float> K32;
    DevBuf<__bf16> Kbf;
    DevBuf<int64_t> mofs;
    bool tiles = false;
    // MFMA tiles of the transposed inverses (adjoint of an unsymmetric A)
    DevBuf<double> K64T;
    DevBuf<__bf16> KbfT;
    // the caller's A as passed to setup: row and column of every entry (vtm_grad's dL/dA)
    DevBuf<int32_t> erow, ecol;
    int64_t a_nnz = 0;
    // port-to-port operators (opt.local_form = 1): M_s per sub-circuit and h per solve
    bool pp = false;
    DevBuf<int64_t> pofs;
    DevBuf<double> M64, h64;
    DevBuf<float> M32, h32;
    // symmetric A: packed port-node operators instead of M
    bool pps = false;
    // any A: K^-1 over the port nodes (k x k) when that is smaller than M
    bool ppn = false;
    DevBuf<int64_t> nofs;
    DevBuf<double> N64, N64T;  // T: transposed, for the adjoint of an unsymmetric A
    DevBuf<float> N32, N32T;
    DevBuf<int32_t> pn_off, pn_node, pn_pfirst;
    // tearing at interfacial nodes: maps between plan rows and the caller's nodes, the
    // caller's A, and right-hand side / residual / solution in the caller's node order
    DevBuf<int32_t> vx_src, vr0, vr1, orow, ocol, oid, orowT, ocolT;
    DevBuf<double> vx_w, oval, ovalT, bo, ro, xo;
    const double* b_user = nullptr;
    // coupled lines: B = 2 W over the ports (CSR) and each port's plan row
    DevBuf<int32_t> brow, bcol, port_row;
    DevBuf<double> bval64;
    DevBuf<float> bval32;
    // residual checks from port quantities (port-to-port form): g and G - g per port
    DevBuf<double> pg64, pgd64;
    // batched port-to-port form (MFMA tiles): q x q operators in A-tile order
    bool ppb = false;
    int pp_variant = 0, pp_rc = 0;  // its launch shape (autotuned like the full batched sweep)
    DevBuf<int64_t> qmofs;
    DevBuf<__bf16> Mbt;
    DevBuf<double> M64t;
    DevBuf<int64_t> sofs;
    DevBuf<double> S64, W64p;
    DevBuf<float> S32, W32p;
    size_t lds_limit = 65536;
    int mfma_variant = 0;                 // chosen by the autotuner
    int mfma_rc = 0;
    // work vectors, [rows][nrhs]
    DevBuf<double> bp, xp, rp;            // FP64: permuted b, x, residual
    DevBuf<double> a64[2];                // FP64 waves
    DevBuf<float> b32, d32, a32[2];       // low-precision inner solve
    DevBuf<__bf16> b16;                   // its right-hand side in BF16 (batched BF16 form)
    DevBuf<double> partial;
    // where the residual reductions put their per-workgroup partial sums and
    // per-column sums: the handle's partial / norms, or the static workspace of
    // vtm_solve_noalloc for the duration of such a call
    double* red_partial = nullptr;
    double* red_norms = nullptr;          // device view of h_norms: the sums land in host memory
    DevBuf<int> flag;
    double* h_norms = nullptr;            // pinned, device-mapped and coherent: the residual kernels
                                          // write the per-column sums here directly (no copy)
    bool waves_set = false;               // next solve resumes from the stored waves
    // per-launch timing of the sweep kernel (opt.timing)
    std::vector<hipEvent_t> ev;
    std::vector<char> ev_tag;             // per event pair: 0 full sweep, 1 port-to-port sweep(s)
    std::vector<int> ev_count;            // per event pair: launches it brackets
    size_t ev_used = 0;
    // captured check intervals (opt.use_graph), keyed by everything their launches depend on
    std::map<std::array<int, 6>, hipGraphExec_t> graphs;
    bool capturing = false;               // no per-sweep timing events inside a capture
    hipStream_t gstream = nullptr;        // private non-blocking stream the graphs run on
    hipEvent_t gready = nullptr;          // orders it after the caller's stream

    ~vtm_handle_s() {
        if (h_norms) (void)hipHostFree(h_norms);
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        if (gready) (void)hipEventDestroy(gready);
        if (gstream) (void)hipStreamDestroy(gstream);
    }

    template <typename T>
    vtm::Coupling<T> coupling() const {
        vtm::Coupling<T> B;
        if (!plan.coupled) return B;
        B.row = brow.p;
        B.col = bcol.p;
        if constexpr (std::is_same_v<T, double>)
            B.val = bval64.p;
        else
            B.val = bval32.p;
        return B;
    }

    vtm::PortArrays ports() const {
        return vtm::PortArrays{port_off.p, port_node.p, port_slot.p, port_twin.p, plan.max_slot};
    }
};

namespace {

using Clock = std::chrono::steady_clock;

// FP64 residual of x against b (both [n][nrhs] renumbered): launches the
// residual and the copy of its per-column sums into pinned host memory.  With
// transpose set the residual is taken on A^T (the adjoint system).
template <typename TX>
vtm_status residual_launch(vtm_handle h, const double* b, const TX* x, int nrhs, double* r_out, bool transpose,
                           float* r32 = nullptr, __bf16* r16 = nullptr) {
    const vtm::Plan& P = h->plan;
    if (P.vertex) {
        // the untorn system in the caller's numbering: x of an interfacial node is the mean
        // of its twins; b is the solve's right-hand side, or the outer residual for an inner check
        const int no = int(P.n_orig);
        const double* bo = b == h->bp.p ? h->bo.p : h->ro.p;
        const bool oT = transpose && !P.osymmetric;  // the adjoint's residual is on A^T
        VTM_HIP(vtm::launch_restrict<TX>(no, nrhs, h->vr0.p, h->vr1.p, x, h->xo.p, false, h->stream));
        VTM_HIP(vtm::launch_residual<double>(no, nrhs, oT ? h->orowT.p : h->orow.p, oT ? h->ocolT.p : h->ocol.p,
                                             oT ? h->ovalT.p : h->oval.p, bo, h->xo.p, r_out ? h->ro.p : nullptr,
                                             nullptr, nullptr, h->red_partial, h->red_norms, h->stream));
        if (r_out)
            VTM_HIP(vtm::launch_expand(int(P.n), nrhs, no, h->vx_src.p, h->vx_w.p, h->ro.p, false, r_out, h->stream));
        const int64_t nv = P.n * nrhs;  // the low-precision copies from the expanded residual
        if (r_out && r32) VTM_HIP((vtm::launch_convert<double, float>(nv, r_out, r32, h->stream)));
        if (r_out && r16) VTM_HIP((vtm::launch_convert<double, __bf16>(nv, r_out, r16, h->stream)));
        return VTM_OK;
    }
    const bool useT = transpose && !P.symmetric;
    VTM_HIP(vtm::launch_residual<TX>(int(P.n), nrhs, useT ? h->rowptrT.p : h->rowptr.p,
                                     useT ? h->colT.p : h->col.p, useT ? h->valT.p : h->val.p, b, x, r_out, r32,
                                     r16, h->red_partial, h->red_norms, h->stream));
    return VTM_OK;
}

// waits for the stream, then relres per column from the copied sums
vtm_status residual_finish(vtm_handle h, int nrhs, std::vector<double>& rel) {
    VTM_HIP(hipStreamSynchronize(h->stream));
    rel.resize(nrhs);
    for (int r = 0; r < nrhs; ++r) {
        const double rr = h->h_norms[2 * r], bb = h->h_norms[2 * r + 1];
        rel[r] = bb > 0.0 ? std::sqrt(rr / bb) : std::sqrt(rr);
    }
    return VTM_OK;
}

template <typename TX>
vtm_status residual(vtm_handle h, const double* b, const TX* x, int nrhs, double* r_out,
                    std::vector<double>& rel, bool transpose, float* r32 = nullptr, __bf16* r16 = nullptr) {
    vtm_status st = residual_launch<TX>(h, b, x, nrhs, r_out, transpose, r32, r16);
    if (st != VTM_OK) return st;
    return residual_finish(h, nrhs, rel);
}

// Residual check from port quantities after a sweep that read waves cur and
// wrote cur ^ 1; per right-hand side r the sum of squares lands in h_norms[2 r].
vtm_status port_residual_launch(vtm_handle h, bool low, int cur, int nrhs) {
    const vtm::Plan& P = h->plan;
    const int64_t nn = int64_t(P.pn_pfirst.size()) - 1;
    if (!low)
        VTM_HIP(vtm::launch_port_residual<double>(nn, nrhs, h->pn_pfirst.p, h->port_twin.p, h->a64[cur].p,
                                                  h->a64[cur ^ 1].p, h->c64.p, h->beta64.p, h->gamma64.p,
                                                  h->pgd64.p, h->pg64.p, h->red_partial, h->red_norms, h->stream));
    else
        VTM_HIP(vtm::launch_port_residual<float>(nn, nrhs, h->pn_pfirst.p, h->port_twin.p, h->a32[cur].p,
                                                 h->a32[cur ^ 1].p, h->c64.p, h->beta64.p, h->gamma64.p,
                                                 h->pgd64.p, h->pg64.p, h->red_partial, h->red_norms, h->stream));
    return VTM_OK;
}

struct IterOut {
    int64_t sweeps = 0;
    int checks = 0;
    int outer = 0;
    double sweep_ms = 0.0;   // full sweeps (opt.timing)
    int64_t launches = 0;
    double pp_ms = 0.0;      // port-to-port sweeps (opt.timing)
    int64_t pp_launches = 0;
    std::vector<double> rel;
    vtm_status status = VTM_OK;
    // residual history: max over columns of the relative residual at each check of a
    // plain solve, or of the FP64 outer residual at each outer step of a refinement,
    // with the sweeps run by then
    std::vector<double> hist;
    std::vector<int64_t> hist_sweeps;
    void record() {
        hist.push_back(max_of_rel());
        hist_sweeps.push_back(sweeps);
    }
    double max_of_rel() const {
        double mx = 0.0;
        for (double v : rel) mx = std::isnan(v) ? v : std::max(mx, v);
        return mx;
    }
};

// Event around a sweep launch (opt.timing); pairs are reused per check interval.
vtm_status timing_event(vtm_handle h, hipEvent_t* out, char tag) {
    if (h->ev_used == h->ev.size()) {
        hipEvent_t e;
        VTM_HIP(hipEventCreate(&e));
        h->ev.push_back(e);
        h->ev_tag.push_back(0);
        h->ev_count.push_back(1);
    }
    h->ev_tag[h->ev_used] = tag;
    h->ev_count[h->ev_used] = 1;
    *out = h->ev[h->ev_used++];
    VTM_HIP(hipEventRecord(*out, h->stream));
    return VTM_OK;
}

// Sums the durations of the recorded event pairs and resets them (waits for the last).
vtm_status timing_collect(vtm_handle h, IterOut& out) {
    if (h->ev_used > 0) VTM_HIP(hipEventSynchronize(h->ev[h->ev_used - 1]));
    for (size_t k = 0; k + 1 < h->ev_used; k += 2) {
        float t = 0.f;
        VTM_HIP(hipEventElapsedTime(&t, h->ev[k], h->ev[k + 1]));
        if (h->ev_tag[k]) {
            out.pp_ms += t;
            out.pp_launches += h->ev_count[k];
        } else {
            out.sweep_ms += t;
            out.launches += h->ev_count[k];
        }
    }
    h->ev_used = 0;
    return VTM_OK;
}

vtm_status launch_one(vtm_handle h, bool low, int nrhs, const void* b, void* x, int cur, bool adjoint, int variant,
                      int rc, bool write_x, bool port_rows = false) {
    const vtm::Plan& P = h->plan;
    if (h->tiles) {
        // the adjoint's operator is K^-T: the same tiles when A is symmetric, else the transposed copy
        const bool kt = adjoint && !P.symmetric;
        if (!low)
            VTM_HIP(vtm::launch_sweep_mfma<double>(int(P.S), P.max_ns, P.max_ports, nrhs, variant, rc, h->lds_limit,
                                                   kt ? h->K64T.p : h->K64.p, h->mofs.p, h->sub_off.p, h->ports(), h->c64.p,
                                                   h->beta64.p, h->gamma64.p, static_cast<const double*>(b),
                                                   h->a64[cur].p, h->a64[cur ^ 1].p, static_cast<double*>(x), write_x,
                                                   h->stream, port_rows));
        else
            VTM_HIP(vtm::launch_sweep_mfma<__bf16>(int(P.S), P.max_ns, P.max_ports, nrhs, variant, rc, h->lds_limit,
                                                   kt ? h->KbfT.p : h->Kbf.p, h->mofs.p, h->sub_off.p, h->ports(), h->c32.p,
                                                   h->beta32.p, h->gamma32.p, h->b16.p, h->a32[cur].p,
                                                   h->a32[cur ^ 1].p, static_cast<float*>(x), write_x, h->stream,
                                                   port_rows));
        return VTM_OK;
    }
    if (!low) {
        VTM_HIP((vtm::launch_sweep<double, double>(int(P.S), P.max_ns, nrhs, h->K64.p, h->kofs.p, h->sub_off.p,
                                                   h->ports(), h->c64.p, h->beta64.p, h->gamma64.p,
                                                   static_cast<const double*>(b), h->a64[cur].p,
                                                   h->a64[cur ^ 1].p, static_cast<double*>(x), adjoint,
                                                   h->lds_limit, h->stream, port_rows)));
    } else {
        VTM_HIP((vtm::launch_sweep<float, float>(int(P.S), P.max_ns, nrhs, h->K32.p, h->kofs.p, h->sub_off.p,
                                                 h->ports(), h->c32.p, h->beta32.p, h->gamma32.p,
                                                 static_cast<const float*>(b), h->a32[cur].p, h->a32[cur ^ 1].p,
                                                 static_cast<float*>(x), adjoint, h->lds_limit, h->stream,
                                                 port_rows)));
    }
    return VTM_OK;
}

// One sweep on the FP64 or FP32/BF16 buffers; cur selects the wave buffer read.
// write_x: the sweep's x must be complete (the last sweep before a check).
// pp: a port-to-port sweep (waves only; needs h of this right-hand side).
// port_rows: a full sweep whose x is read on the port nodes only (the first sweep
// of a port-to-port run, whose x feeds h and is rebuilt later); kernels that can
// form those rows alone do so.
vtm_status sweep_once(vtm_handle h, bool low, int nrhs, const void* b, void* x, int cur, bool adjoint,
                      bool write_x, bool pp = false, bool port_rows = false) {
    hipEvent_t e0, e1;
    vtm_status st;
    // timing 1: events around every launch; 2: only full sweeps here (runs of
    // port-to-port sweeps get one pair in run_chunk)
    const bool timed = !h->capturing && (h->opt.timing == 1 || (h->opt.timing == 2 && !pp));
    if (timed && (st = timing_event(h, &e0, pp ? 1 : 0)) != VTM_OK) return st;
    if (pp && h->tiles) {
        const vtm::Plan& P = h->plan;
        if (!low)
            VTM_HIP(vtm::launch_sweep_mfma_pp<double>(int(P.S), P.max_ports, nrhs, h->pp_variant, h->pp_rc,
                                                      h->lds_limit, h->M64t.p, h->qmofs.p, h->port_off.p,
                                                      h->port_twin.p, h->h64.p, h->a64[cur].p, h->a64[cur ^ 1].p,
                                                      cur, h->stream));
        else
            VTM_HIP(vtm::launch_sweep_mfma_pp<__bf16>(int(P.S), P.max_ports, nrhs, h->pp_variant, h->pp_rc,
                                                      h->lds_limit, h->Mbt.p, h->qmofs.p, h->port_off.p,
                                                      h->port_twin.p, h->h32.p, h->a32[cur].p, h->a32[cur ^ 1].p,
                                                      cur, h->stream));
    } else if (pp && h->ppn) {
        const vtm::Plan& P = h->plan;
        if (!low)
            VTM_HIP((vtm::launch_sweep_ppn<double, double>(int(P.S), P.max_npn, P.max_ports,
                                                           adjoint && !P.symmetric ? h->N64T.p : h->N64.p, h->nofs.p,
                                                           h->pn_off.p, h->pn_pfirst.p, h->port_off.p, h->port_twin.p,
                                                           h->c64.p, h->beta64.p, h->gamma64.p, h->h64.p,
                                                           h->a64[cur].p, h->a64[cur ^ 1].p, h->stream)));
        else
            VTM_HIP((vtm::launch_sweep_ppn<float, float>(int(P.S), P.max_npn, P.max_ports,
                                                         adjoint && !P.symmetric ? h->N32T.p : h->N32.p, h->nofs.p,
                                                         h->pn_off.p, h->pn_pfirst.p, h->port_off.p, h->port_twin.p,
                                                         h->c32.p, h->beta32.p, h->gamma32.p, h->h32.p,
                                                         h->a32[cur].p, h->a32[cur ^ 1].p, h->stream)));
    } else if (pp && h->pps) {
        const vtm::Plan& P = h->plan;
        const double W = P.nwires ? P.wW[0] : 0.0;
        if (!low)
            VTM_HIP((vtm::launch_sweep_pps<double, double>(int(P.S), P.max_npn, P.max_ports, h->S64.p, h->sofs.p, h->pn_off.p,
                                                           h->pn_pfirst.p, h->port_off.p, h->port_twin.p, h->c64.p,
                                                           h->W64p.p, W, h->h64.p, h->a64[cur].p, h->a64[cur ^ 1].p,
                                                           cur, h->stream)));
        else
            VTM_HIP((vtm::launch_sweep_pps<float, float>(int(P.S), P.max_npn, P.max_ports, h->S32.p, h->sofs.p, h->pn_off.p,
                                                         h->pn_pfirst.p, h->port_off.p, h->port_twin.p, h->c32.p,
                                                         h->W32p.p, float(W), h->h32.p, h->a32[cur].p,
                                                         h->a32[cur ^ 1].p, cur, h->stream)));
    } else if (pp) {
        const vtm::Plan& P = h->plan;
        if (!low)
            VTM_HIP((vtm::launch_sweep_pp<double, double>(int(P.S), P.max_ports, h->M64.p, h->pofs.p, h->port_off.p,
                                                          h->port_twin.p, h->h64.p, h->a64[cur].p, h->a64[cur ^ 1].p,
                                                          h->stream)));
        else
            VTM_HIP((vtm::launch_sweep_pp<float, float>(int(P.S), P.max_ports, h->M32.p, h->pofs.p, h->port_off.p,
                                                        h->port_twin.p, h->h32.p, h->a32[cur].p, h->a32[cur ^ 1].p,
                                                        h->stream)));
    } else {
        if ((st = launch_one(h, low, nrhs, b, x, cur, adjoint, h->mfma_variant, h->mfma_rc, write_x, port_rows)) !=
            VTM_OK)
            return st;
        const vtm::Plan& P = h->plan;
        if (P.coupled) {  // the waves of coupled lines need W over the port rows of x
            if (!low)
                VTM_HIP(vtm::launch_wave_coupled<double>(int(P.nports), nrhs, h->coupling<double>(), h->port_row.p,
                                                         h->gamma64.p, h->port_twin.p, static_cast<const double*>(x),
                                                         h->a64[cur].p, h->a64[cur ^ 1].p, h->stream));
            else
                VTM_HIP(vtm::launch_wave_coupled<float>(int(P.nports), nrhs, h->coupling<float>(), h->port_row.p,
                                                        h->gamma32.p, h->port_twin.p, static_cast<const float*>(x),
                                                        h->a32[cur].p, h->a32[cur ^ 1].p, h->stream));
        }
    }
    if (timed) return timing_event(h, &e1, pp ? 1 : 0);
    return VTM_OK;
}

// h_p = beta_p x_i(p) from the x just computed (x = K^-1 b: the first sweep from zero waves)
vtm_status port_h(vtm_handle h, bool low, int nrhs) {
    const vtm::Plan& P = h->plan;
    if (!low)
        VTM_HIP(vtm::launch_port_h<double>(int(P.S), nrhs, h->sub_off.p, h->port_off.p, h->port_node.p, h->beta64.p,
                                           h->xp.p, h->h64.p, h->stream, h->coupling<double>()));
    else
        VTM_HIP(vtm::launch_port_h<float>(int(P.S), nrhs, h->sub_off.p, h->port_off.p, h->port_node.p, h->beta32.p,
                                          h->d32.p, h->h32.p, h->stream, h->coupling<float>()));
    return VTM_OK;
}

// Autotuner of the batched kernel: on this handle's own sub-circuits (zero
// vectors: timing does not depend on values), time every candidate launch
// shape -- row tiles per wavefront per pass (3 or 5) x right-hand sides per
// workgroup (64, 48, 32, 16) -- over three sweeps after one warm-up, keep the
// fastest.
vtm_status autotune(vtm_handle h) {
    const vtm::Plan& P = h->plan;
    const bool low = h->opt.precision != VTM_FP64;
    const int nrhs = h->nrhs_max;
    const void* b = low ? static_cast<const void*>(h->b32.p) : static_cast<const void*>(h->bp.p);
    void* x = low ? static_cast<void*>(h->d32.p) : static_cast<void*>(h->xp.p);
    if (low) {
        VTM_HIP(vtm::launch_fill<__bf16>(P.n * nrhs, __bf16(0.0f), h->b16.p, h->stream));
        VTM_HIP(vtm::launch_fill<float>(P.nports * nrhs, 0.0f, h->a32[0].p, h->stream));
        VTM_HIP(vtm::launch_fill<float>(P.nports * nrhs, 0.0f, h->a32[1].p, h->stream));
    } else {
        VTM_HIP(vtm::launch_fill<double>(P.n * nrhs, 0.0, h->bp.p, h->stream));
        VTM_HIP(vtm::launch_fill<double>(P.nports * nrhs, 0.0, h->a64[0].p, h->stream));
        VTM_HIP(vtm::launch_fill<double>(P.nports * nrhs, 0.0, h->a64[1].p, h->stream));
    }
    hipEvent_t t0, t1;
    VTM_HIP(hipEventCreate(&t0));
    VTM_HIP(hipEventCreate(&t1));
    float best = INFINITY;
    int bv = 0, brc = 0;
    vtm_status st = VTM_OK;
    const int v_lo = h->opt.batch_row_tiles == 5 ? 1 : 0, v_hi = h->opt.batch_row_tiles == 3 ? 0 : 1;
    // variants 0 and 1: 3 or 5 row tiles per pass; 2: one row tile (only when not forced)
    for (int variant = v_lo; variant <= (h->opt.batch_row_tiles > 0 ? v_hi : 2) && st == VTM_OK; ++variant)
        for (int rc = 64; rc >= 16 && st == VTM_OK; rc -= 16) {
            if (variant == 1 && v_hi == 0) continue;
            if (rc > 16 && rc >= nrhs + 16) continue;  // wider than the right-hand sides
            if (h->opt.batch_rhs_block > 0 && rc != h->opt.batch_rhs_block) continue;
            st = launch_one(h, low, nrhs, b, x, 0, false, variant, rc, false);
            if (st != VTM_OK) break;
            if (hipEventRecord(t0, h->stream) != hipSuccess) st = fail(VTM_E_HIP, "event record");
            for (int k = 0; k < 3 && st == VTM_OK; ++k)
                st = launch_one(h, low, nrhs, b, x, k & 1, false, variant, rc, false);
            if (st != VTM_OK) break;
            float ms = 0.f;
            if (hipEventRecord(t1, h->stream) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
                hipEventElapsedTime(&ms, t0, t1) != hipSuccess)
                st = fail(VTM_E_HIP, "autotune timing");
            else if (ms < best) {
                best = ms;
                h->mfma_variant = variant;
                h->mfma_rc = rc;
            }
        }
    // the batched port-to-port sweep: the same candidates on its q x q operators
    if (st == VTM_OK && h->ppb) {
        const int32_t timing = h->opt.timing;  // no per-launch events while tuning
        h->opt.timing = 0;
        if (low)
            VTM_HIP(vtm::launch_fill<float>(P.nports * nrhs, 0.0f, h->h32.p, h->stream));
        else
            VTM_HIP(vtm::launch_fill<double>(P.nports * nrhs, 0.0, h->h64.p, h->stream));
        float best_pp = INFINITY;
        // variants: bit 0 five row tiles, bit 1 eight wavefronts, bit 2 one row tile (bit 0 unused)
        const bool forced_rows = h->opt.batch_row_tiles > 0;
        for (int variant = 0; variant < 8 && st == VTM_OK; ++variant)
            for (int rc = 64; rc >= 16 && st == VTM_OK; rc -= 16) {
                if ((variant & 5) == 5 || (forced_rows && (variant & 4))) continue;
                if (!(variant & 4) && ((variant & 1) < v_lo || (variant & 1) > v_hi)) continue;
                if (rc > 16 && rc >= nrhs + 16) continue;
                if (h->opt.batch_rhs_block > 0 && rc != h->opt.batch_rhs_block) continue;
                h->pp_variant = variant;
                h->pp_rc = rc;
                st = sweep_once(h, low, nrhs, b, x, 0, false, false, true);
                if (st != VTM_OK) break;
                if (hipEventRecord(t0, h->stream) != hipSuccess) st = fail(VTM_E_HIP, "event record");
                for (int k = 0; k < 3 && st == VTM_OK; ++k) st = sweep_once(h, low, nrhs, b, x, k & 1, false, false, true);
                if (st != VTM_OK) break;
                float ms = 0.f;
                if (hipEventRecord(t1, h->stream) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
                    hipEventElapsedTime(&ms, t0, t1) != hipSuccess)
                    st = fail(VTM_E_HIP, "autotune timing");
                else if (ms < best_pp) {
                    best_pp = ms;
                    bv = variant;
                    brc = rc;
                }
            }
        h->pp_variant = bv;
        h->pp_rc = brc;
        h->opt.timing = timing;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    return st;
}

// One check interval: `chunk` sweeps from wave buffer `cur`, then the FP64
// residual check.  Plain form: b = bp, x = xp, check of b - A x.  Inner form
// (low precision): x = d32, check of r - A d.  pp: sweeps in between are
// port-to-port, the last one is a full sweep (it rebuilds x for the check);
// first: the interval starts the solve from zero waves, so its first sweep is
// a full one and yields h.  With opt.use_graph the interval is captured once
// per shape and replayed as one hipGraph launch.
// `chunk` sweeps from waves `cur`, then a residual check.  pp: the sweeps are
// port-to-port except the first of a solve (which also forms h) and, unless
// iface, the last (which rebuilds x for the residual on A).  iface: the check
// is the residual from port quantities, relative to sqrt(bb).
vtm_status run_chunk(vtm_handle h, bool low, int nrhs, bool adjoint, int64_t chunk, int cur,
                     std::vector<double>& rel, bool pp, bool first, bool iface = false,
                     const std::vector<double>* bb = nullptr) {
    const void* b = low ? (h->tiles ? static_cast<const void*>(h->b16.p) : static_cast<const void*>(h->b32.p))
                        : static_cast<const void*>(h->bp.p);
    void* x = low ? static_cast<void*>(h->d32.p) : static_cast<void*>(h->xp.p);
    auto enqueue = [&]() -> vtm_status {
        const bool bracket = h->opt.timing == 2 && !h->capturing;
        hipEvent_t r0 = nullptr, r1 = nullptr;
        size_t r0_slot = 0;
        int run = 0;  // port-to-port sweeps since r0
        auto close_run = [&]() -> vtm_status {
            if (run == 0) return VTM_OK;
            vtm_status st = timing_event(h, &r1, 1);
            if (st != VTM_OK) return st;
            h->ev_count[r0_slot] = run;
            run = 0;
            return VTM_OK;
        };
        for (int64_t k = 0; k < chunk; ++k) {
            const bool full = !pp || (k + 1 == chunk && !iface) || (first && k == 0);
            vtm_status st;
            if (bracket && full && (st = close_run()) != VTM_OK) return st;
            if (bracket && !full && run == 0) {
                r0_slot = h->ev_used;
                if ((st = timing_event(h, &r0, 1)) != VTM_OK) return st;
            }
            // the first sweep of a port-to-port run needs x on the port nodes only (for h),
            // unless it also ends a chunk whose check reads x on A
            const bool port_rows = full && pp && first && k == 0 && (iface || k + 1 < chunk);
            st = sweep_once(h, low, nrhs, b, x, (cur + int(k)) & 1, adjoint, k + 1 == chunk, !full, port_rows);
            if (st != VTM_OK) return st;
            if (!full) ++run;
            if (pp && first && k == 0 && (st = port_h(h, low, nrhs)) != VTM_OK) return st;
        }
        if (bracket) {
            vtm_status st = close_run();
            if (st != VTM_OK) return st;
        }
        if (iface) return port_residual_launch(h, low, (cur + int(chunk) - 1) & 1, nrhs);
        return low ? residual_launch<float>(h, h->rp.p, h->d32.p, nrhs, nullptr, adjoint)
                   : residual_launch<double>(h, h->bp.p, h->xp.p, nrhs, nullptr, adjoint);
    };
    auto finish = [&]() -> vtm_status {
        if (!iface) return residual_finish(h, nrhs, rel);
        VTM_HIP(hipStreamSynchronize(h->stream));
        rel.resize(nrhs);
        for (int r = 0; r < nrhs; ++r) {
            const double d = bb ? (*bb)[r] : 1.0, rr = h->h_norms[2 * r];
            rel[r] = d > 0.0 ? std::sqrt(rr / d) : std::sqrt(rr);
        }
        return VTM_OK;
    };
    if (!h->opt.use_graph) {
        vtm_status st = enqueue();
        if (st != VTM_OK) return st;
        return finish();
    }
    // graphs run on the handle's own non-blocking stream (the caller's may be the
    // legacy null stream, which cannot be captured), after the caller's work
    if (!h->gstream) {
        VTM_HIP(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
        VTM_HIP(hipEventCreateWithFlags(&h->gready, hipEventDisableTiming));
    }
    VTM_HIP(hipEventRecord(h->gready, h->stream));
    VTM_HIP(hipStreamWaitEvent(h->gstream, h->gready, 0));
    struct Swap {
        vtm_handle h;
        hipStream_t saved;
        ~Swap() { h->stream = saved; }
    } swap{h, h->stream};
    h->stream = h->gstream;
    const std::array<int, 6> key{int(low), nrhs, int(adjoint), int(chunk), cur,
                                 int(pp) * 4 + int(iface) * 2 + int(first)};
    auto it = h->graphs.find(key);
    if (it == h->graphs.end()) {
        VTM_HIP(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        h->capturing = true;
        vtm_status st = enqueue();
        h->capturing = false;
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(h->stream, &g);
        if (st != VTM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return fail(VTM_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) return fail(VTM_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
        it = h->graphs.emplace(key, ex).first;
    }
    VTM_HIP(hipGraphLaunch(it->second, h->stream));
    return finish();
}


// Where the next residual check goes.  With adaptive checks, once two checks
// show the residual falling, the per-sweep rate predicts the sweeps left to the
// target; the next check comes after half of them (a multiple of m, at most
// 64 m), so checks thin out far from the target and return to every m sweeps
// near it.
struct Cadence {
    int64_t m = 1;
    bool adaptive = false;
    double reach = 0.5;     // fraction of the predicted sweeps to the target before the next check
    int64_t cap = 64;       // at most this many m between checks
    int64_t s_prev = -1, s_last = -1;
    double r_prev = 0.0, r_last = 0.0;
    void record(int64_t s, double r) {
        s_prev = s_last;
        r_prev = r_last;
        s_last = s;
        r_last = r;
    }
    int64_t next(double target) const {
        if (!adaptive || s_prev < 0 || !(r_last < r_prev) || !(r_last > 0.0) || !(target > 0.0) ||
            !(r_last > target))
            return m;
        const double rate = std::log(r_last / r_prev) / double(s_last - s_prev);  // < 0
        const double left = std::log(target / r_last) / rate;                       // > 0
        const int64_t k = int64_t(reach * left / double(m)) * m;
        return std::min<int64_t>(std::max<int64_t>(k, m), cap * m);
    }
};

double max_of(const std::vector<double>& v) {
    double mx = 0.0;
    for (double x : v) mx = std::isnan(x) ? x : std::max(mx, x);
    return mx;
}

// With graphs, check intervals are m times a power of two (a few graphs cover them all).
int64_t graph_length(vtm_handle h, int64_t k) {
    if (!h->opt.use_graph) return k;
    const int64_t m = h->opt.check_every;
    int64_t len = m;
    while (2 * len <= k) len *= 2;
    return len;
}

// Plain FP64 VTM on (bp -> xp).  Waves start at zero unless resume is set.
vtm_status run_fp64(vtm_handle h, int nrhs, double tol, bool adjoint, bool resume, IterOut& out) {
    const vtm::Plan& P = h->plan;
    const int64_t np = P.nports * nrhs;
    Cadence cad;
    cad.m = h->opt.check_every;
    cad.adaptive = h->opt.adaptive_checks != 0;
    int cur = 0;
    if (!resume) VTM_HIP(vtm::launch_fill<double>(np, 0.0, h->a64[0].p, h->stream));
    VTM_HIP(vtm::launch_fill<double>(P.n * nrhs, 0.0, h->xp.p, h->stream));
    // x^0 = 0: the check before any sweep (b = 0 converges at once)
    vtm_status st = residual<double>(h, h->bp.p, h->xp.p, nrhs, nullptr, out.rel, adjoint);
    if (st != VTM_OK) return st;
    ++out.checks;
    out.record();
    auto done = [&](const std::vector<double>& rel) {
        for (double v : rel)
            if (!(v <= tol)) return false;
        return true;
    };
    if (done(out.rel)) return VTM_OK;
    if (!resume) cad.record(0, max_of(out.rel));
    std::vector<double> bb(nrhs);  // ||b||^2 per right-hand side, for the port-residual checks
    for (int r = 0; r < nrhs; ++r) bb[r] = h->h_norms[2 * r + 1];
    const bool pp = ((h->pp && nrhs == 1) || h->ppb) && (!adjoint || P.symmetric || h->ppn) && !resume;
    // port-to-port sweeps check the residual from port quantities; once it passes
    // (and at the end), x^k is rebuilt by a full sweep from the same waves and
    // the residual on A decides
    const bool iface = pp && !P.vertex;  // the port identity holds for cut branches only
    auto rebuild = [&]() -> vtm_status {
        vtm_status s2 = sweep_once(h, false, nrhs, h->bp.p, h->xp.p, cur ^ 1, adjoint, true, false);
        if (s2 != VTM_OK) return s2;
        if ((s2 = residual<double>(h, h->bp.p, h->xp.p, nrhs, nullptr, out.rel, adjoint)) != VTM_OK) return s2;
        ++out.checks;
        out.record();
        return timing_collect(h, out);
    };
    while (true) {
        const int64_t chunk = std::min<int64_t>(graph_length(h, cad.next(tol)), h->opt.max_sweeps - out.sweeps);
        st = run_chunk(h, false, nrhs, adjoint, chunk, cur, out.rel, pp, out.sweeps == 0, iface, &bb);
        if (st != VTM_OK) return st;
        cur ^= int(chunk & 1);
        out.sweeps += chunk;
        ++out.checks;
        out.record();
        if ((st = timing_collect(h, out)) != VTM_OK) return st;
        bool bad = false;
        for (double v : out.rel)
            if (!std::isfinite(v) || v > h->opt.divergence) bad = true;
        if (bad) {
            if (iface && (st = rebuild()) != VTM_OK) return st;
            out.status = VTM_E_DIVERGED;
            break;
        }
        if (done(out.rel)) {
            if (!iface) break;
            if ((st = rebuild()) != VTM_OK) return st;
            if (done(out.rel)) break;
        }
        if (out.sweeps >= h->opt.max_sweeps) {
            if (iface && (st = rebuild()) != VTM_OK) return st;
            out.status = VTM_E_MAXITER;
            break;
        }
        cad.record(out.sweeps, max_of(out.rel));
    }
    // leave the latest waves in buffer 0 for export / resume
    if (cur == 1)
        VTM_HIP(hipMemcpyAsync(h->a64[0].p, h->a64[1].p, sizeof(double) * np, hipMemcpyDeviceToDevice,
                               h->stream));
    return VTM_OK;
}

// Mixed precision: FP64 outer refinement around an FP32 inner VTM.
// Algorithmic bytes of one port-to-port sweep of nrhs right-hand sides: operator
// entries once (without layout padding); per port the wave in, h in, wave out
// (and c for the packed form) plus the twin index; per port node its first port;
// per sub-circuit its offsets.  0 without a port-to-port form.
int64_t pp_sweep_bytes(const vtm_handle_s* h, int64_t nrhs) {
    const vtm::Plan& P = h->plan;
    const int64_t esize = h->opt.precision == VTM_FP64 ? 8 : (h->opt.precision == VTM_FP32_REFINE ? 4 : 2);
    const int64_t tv = h->opt.precision == VTM_FP64 ? 8 : 4;  // waves (FP32 for the BF16 form)
    if (h->ppb) return P.sq_entries * esize + P.nports * (4 + nrhs * 3 * tv) + P.S * 16;
    if (h->ppn)
        return P.sqn_entries * esize + P.nports * (6 * esize + 4) + int64_t(P.pn_node.size()) * 4 + P.S * 16;
    if (h->pps)
        return P.tri_entries * esize + P.nports * (4 * esize + 4 + (P.uniform_W ? 0 : esize)) +
               int64_t(P.pn_node.size()) * 4 + P.S * 16;
    if (h->pp) return P.sq_entries * esize + P.nports * (3 * esize + 4) + P.S * 12;
    return 0;
}

// How far towards the predicted target an inner solve's next check goes: the
// next check comes after this fraction of the predicted sweeps.  Far (0.9) when a
// check costs more than a sweep, so that few checks are spent; halfway (0.5)
// when sweeps cost more, so that little is overshot.  Costs from the bytes each
// moves: a sweep streams its operator and vectors (plus ~4 us of launch, 20 MB at
// 5 TB/s); a check reads per port its waves and its twin's with six
// coefficients (port form) or A, b and x (CSR form), at about half a sweep's
// rate (gathers), and waits for the host (~25 us, 125 MB).
double inner_reach(const vtm_handle_s* h, int nrhs, bool pp) {
    const vtm::Plan& P = h->plan;
    const int64_t tv = h->opt.precision == VTM_FP64 ? 8 : 4;
    const int64_t esize = h->opt.precision == VTM_FP64 ? 8 : (h->opt.precision == VTM_FP32_REFINE ? 4 : 2);
    double sweep, check;
    if (pp) {
        sweep = double(pp_sweep_bytes(h, nrhs));
        check = double(P.nports) * (3.0 * nrhs * tv + 44.0) + double(P.pn_node.size()) * (nrhs * tv + 8.0);
    } else {
        sweep = double(h->tiles ? P.mofs[P.S] : P.kofs[P.S]) * esize + double(P.n) * nrhs * 2.0 * tv;
        check = double(P.col.size()) * 12.0 + double(P.n) * nrhs * (16.0 + tv);
    }
    const double c = (2.0 * check + 125e6) / (sweep + 20e6);
    return c > 1.0 ? 0.9 : 0.5;
}

vtm_status run_refine(vtm_handle h, int nrhs, double tol, bool adjoint, IterOut& out) {
    const vtm::Plan& P = h->plan;
    const int64_t nv = P.n * nrhs, np = P.nports * nrhs;
    double drop = h->opt.inner_drop;
    if (!(drop > 0.0)) drop = h->opt.precision == VTM_BF16_REFINE ? 1e-2 : 1e-5;
    VTM_HIP(vtm::launch_fill<double>(nv, 0.0, h->xp.p, h->stream));
    std::vector<double> rel, e, target(nrhs);
    const bool pp = ((h->pp && nrhs == 1) || h->ppb) && (!adjoint || P.symmetric || h->ppn);
    auto all_le = [](const std::vector<double>& v, const std::vector<double>& t) {
        for (size_t i = 0; i < v.size(); ++i)
            if (!(v[i] <= t[i])) return false;
        return true;
    };
    // the inner checks: ||r - A d|| from port quantities (then r itself is not read
    // again), else on A with the FP64 r kept by the outer residual
    const bool iface = pp && !P.vertex;
    for (int outer = 0;; ++outer) {
        // r = b - A x (FP64) and its BF16 or FP32 copy (the inner right-hand side),
        // written by the same pass
        vtm_status st = residual<double>(h, h->bp.p, h->xp.p, nrhs, iface ? nullptr : h->rp.p, rel, adjoint,
                                         h->tiles ? nullptr : h->b32.p, h->tiles ? h->b16.p : nullptr);
        if (st != VTM_OK) return st;
        ++out.checks;
        out.rel = rel;
        out.record();
        for (double v : rel)
            if (!std::isfinite(v) || v > h->opt.divergence) {
                out.status = VTM_E_DIVERGED;
                return VTM_OK;
            }
        if (all_le(rel, std::vector<double>(nrhs, tol))) return VTM_OK;
        if (outer >= h->opt.max_outer) {
            out.status = VTM_E_MAXITER;
            return VTM_OK;
        }
        // inner target relative to ||r||: enough for the outer tolerance, at most drop
        for (int r = 0; r < nrhs; ++r) target[r] = rel[r] > 0.0 ? std::max(drop, 0.5 * tol / rel[r]) : 1.0;
        std::vector<double> rr(nrhs);  // ||r||^2 per right-hand side, for the port-residual inner checks
        for (int r = 0; r < nrhs; ++r) rr[r] = h->h_norms[2 * r];
        VTM_HIP(vtm::launch_fill<float>(np, 0.0f, h->a32[0].p, h->stream));
        Cadence cad;
        cad.m = h->opt.check_every;
        cad.adaptive = h->opt.adaptive_checks != 0;
        cad.reach = inner_reach(h, nrhs, pp);
        cad.cap = 4;
        cad.record(0, 1.0);
        double goal = 1.0;
        for (int r = 0; r < nrhs; ++r) goal = std::min(goal, target[r]);
        int cur = 0;
        int64_t inner = 0;
        std::vector<double> best(nrhs, INFINITY);
        int since = 0;
        while (true) {
            // an inner solve may stall above its target (the low-precision inverse
            // bounds the reachable reduction), so its checks are at most 4 m apart
            const int64_t chunk =
                std::min<int64_t>(graph_length(h, cad.next(goal)), h->opt.max_sweeps - inner);
            // sweeps, then ||r - A d|| / ||r|| in FP64 (from port quantities with pp)
            st = run_chunk(h, true, nrhs, adjoint, chunk, cur, e, pp, inner == 0, iface, &rr);
            if (st != VTM_OK) return st;
            cur ^= int(chunk & 1);
            inner += chunk;
            ++out.checks;
            if ((st = timing_collect(h, out)) != VTM_OK) return st;
            // progress: some column fell by at least 20% since its best check
            bool improved = false, bad = false;
            for (int r = 0; r < nrhs; ++r) {
                if (!std::isfinite(e[r])) bad = true;
                if (e[r] < 0.8 * best[r]) improved = true;
                best[r] = std::min(best[r], e[r]);
            }
            if (bad) {
                out.sweeps += inner;
                out.status = VTM_E_DIVERGED;
                return VTM_OK;
            }
            since = improved ? 0 : since + 1;
            if (all_le(e, target) || since >= 2 || inner >= h->opt.max_sweeps) break;
            cad.record(inner, max_of(e));
        }
        out.sweeps += inner;
        if (pp && !P.vertex) {  // d from the last sweep's waves, by a full sweep
            const void* bl = h->tiles ? static_cast<const void*>(h->b16.p) : static_cast<const void*>(h->b32.p);
            if ((st = sweep_once(h, true, nrhs, bl, h->d32.p, cur ^ 1, adjoint, true, false)) != VTM_OK)
                return st;
            if ((st = timing_collect(h, out)) != VTM_OK) return st;
        }
        VTM_HIP(vtm::launch_add<float>(nv, h->d32.p, h->xp.p, h->stream));
        ++out.outer;
    }
}

vtm_status solve_common(vtm_handle h, const double* b, double* x, int32_t nrhs, double tol, vtm_report* rep,
                        bool adjoint) {
    const auto t0 = Clock::now();
    if (!h) return fail(VTM_E_ARG, "null handle");
    h->ev_used = 0;
    if (!b || !x) return fail(VTM_E_ARG, "null vector");
    if (nrhs < 1 || nrhs > h->nrhs_max) return fail(VTM_E_ARG, "nrhs outside 1..nrhs_max");
    if (!(tol > 0.0)) return fail(VTM_E_ARG, "tol must be positive");
    VTM_HIP(hipSetDevice(h->device));
    const vtm::Plan& P = h->plan;
    if (P.vertex) {
        // interfacial sources split between the twins; b also kept in node order for the residual
        VTM_HIP(vtm::launch_expand(int(P.n), nrhs, int(P.n_orig), h->vx_src.p, h->vx_w.p, b, true, h->bp.p,
                                   h->stream));
        VTM_HIP(vtm::launch_gather(int(P.n_orig), nrhs, h->oid.p, b, h->bo.p, h->stream));
    } else {
        VTM_HIP(vtm::launch_gather(int(P.n), nrhs, h->perm.p, b, h->bp.p, h->stream));
    }
    IterOut out;
    vtm_status st;
    if (h->opt.precision == VTM_FP64) {
        st = run_fp64(h, nrhs, tol, adjoint, h->waves_set, out);
    } else {
        st = run_refine(h, nrhs, tol, adjoint, out);
    }
    h->waves_set = false;
    if (st != VTM_OK) return st;
    if (P.vertex)
        VTM_HIP(vtm::launch_restrict<double>(int(P.n_orig), nrhs, h->vr0.p, h->vr1.p, h->xp.p, x, true, h->stream));
    else
        VTM_HIP(vtm::launch_scatter(int(P.n), nrhs, h->iperm.p, h->xp.p, x, h->stream));
    VTM_HIP(hipStreamSynchronize(h->stream));
    if (rep) {
        rep->sweeps = out.sweeps;
        rep->outer = out.outer;
        rep->checks = out.checks;
        rep->relres_max = max_of(out.rel);
        rep->solve_ms = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
        rep->sweep_kernel_ms = out.sweep_ms;
        rep->sweep_launches = out.launches;
        rep->pp_kernel_ms = out.pp_ms;
        rep->pp_launches = out.pp_launches;
        rep->batch_row_tiles = h->tiles ? (h->mfma_variant == 1 ? 5 : (h->mfma_variant == 2 ? 1 : 3)) : 0;
        rep->batch_rhs_block = h->tiles ? h->mfma_rc : 0;
        // pp variant bits: 0 five row tiles, 1 eight wavefronts, 2 one row tile
        const int ppv = h->pp_variant;
        rep->pp_shape[0] = h->ppb ? ((ppv & 4) ? 1 : (ppv & 1) ? 5 : 3) : 0;
        rep->pp_shape[1] = h->ppb ? std::min(h->pp_rc, (nrhs + 15) / 16 * 16) : 0;
        rep->pp_shape[2] = h->ppb ? ((ppv & 2) ? 8 : 4) : 0;
        if (rep->relres)
            for (int r = 0; r < nrhs; ++r) rep->relres[r] = out.rel[r];
        const int64_t len = std::min<int64_t>(int64_t(out.hist.size()), std::max(rep->history_cap, 0));
        for (int64_t k = 0; k < len; ++k) {
            if (rep->history) rep->history[k] = out.hist[k];
            if (rep->history_sweeps) rep->history_sweeps[k] = out.hist_sweeps[k];
        }
        rep->history_len = int32_t(len);
        rep->history_total = int32_t(out.hist.size());
    }
    if (out.status == VTM_E_DIVERGED) return fail(VTM_E_DIVERGED, "the iteration diverged");
    if (out.status == VTM_E_MAXITER) return fail(VTM_E_MAXITER, "no convergence within the sweep limit");
    return VTM_OK;
}

}  // namespace

extern "C" {

static vtm_status check_options(const vtm_options& o);
static vtm_status setup_from_plan(std::unique_ptr<vtm_handle_s> h, vtm_handle* out);

// Row and column of every entry of the caller's A, in the caller's entry order
// (vtm_grad's dL/dA); A was validated by the planner.
static vtm_status keep_pattern(vtm_handle_s* h, const vtm_csr* A) {
    std::vector<int32_t> row(A->nnz), col(A->col, A->col + A->nnz);
    for (int64_t i = 0; i < A->n; ++i)
        for (int64_t q = A->rowptr[i]; q < A->rowptr[i + 1]; ++q) row[q] = int32_t(i);
    VTM_HIP(h->erow.upload(row, h->stream));
    VTM_HIP(h->ecol.upload(col, h->stream));
    VTM_HIP(hipStreamSynchronize(h->stream));
    h->a_nnz = A->nnz;
    return VTM_OK;
}

vtm_status vtm_setup(const vtm_csr* A, const int32_t* part, const double* Z, int64_t nZ,
                     const vtm_options* opt, void* stream, vtm_handle* out) {
    return vtm::guarded([&]() -> vtm_status {
        if (!out) return fail(VTM_E_ARG, "null output handle");
        *out = nullptr;
        vtm_options o;
        vtm_default_options(&o);
        if (opt) o = *opt;
        vtm_status st = check_options(o);
        if (st != VTM_OK) return st;
        auto h = std::make_unique<vtm_handle_s>();
        h->opt = o;
        h->nrhs_max = o.nrhs_max;
        h->stream = static_cast<hipStream_t>(stream);
        std::string err;
        st = vtm::build_plan(A, part, Z, nZ, h->plan, err);
        if (st != VTM_OK) return fail(st, err);
        if ((st = keep_pattern(h.get(), A)) != VTM_OK) return st;
        return setup_from_plan(std::move(h), out);
    });
}

static vtm_status setup_vertex_common(const vtm_csr* A, const int32_t* label, const int32_t* iface, const int32_t* sides,
                               int64_t n_iface, const double* W, int64_t nW, const vtm_csr* Wc,
                               const vtm_options* opt, void* stream, vtm_handle* out);

vtm_status vtm_setup_vertex(const vtm_csr* A, const int32_t* label, const int32_t* iface, const int32_t* sides,
                            int64_t n_iface, const double* W, int64_t nW, const vtm_options* opt, void* stream,
                            vtm_handle* out) {
    return vtm::guarded([&]() -> vtm_status {
        return setup_vertex_common(A, label, iface, sides, n_iface, W, nW, nullptr, opt, stream, out);
    });
}

static vtm_status setup_vertex_common(const vtm_csr* A, const int32_t* label, const int32_t* iface, const int32_t* sides,
                               int64_t n_iface, const double* W, int64_t nW, const vtm_csr* Wc,
                               const vtm_options* opt, void* stream, vtm_handle* out) {
    if (!out) return fail(VTM_E_ARG, "null output handle");
    *out = nullptr;
    vtm_options o;
    vtm_default_options(&o);
    if (opt) o = *opt;
    vtm_status st = check_options(o);
    if (st != VTM_OK) return st;
    auto h = std::make_unique<vtm_handle_s>();
    h->opt = o;
    h->nrhs_max = o.nrhs_max;
    h->stream = static_cast<hipStream_t>(stream);
    std::string err;
    st = vtm::build_plan_vertex(A, label, iface, sides, n_iface, W, nW, h->plan, err, Wc);
    if (st != VTM_OK) return fail(st, err);
    if ((st = keep_pattern(h.get(), A)) != VTM_OK) return st;
    const vtm::Plan& P = h->plan;
    hipStream_t s = h->stream;
    VTM_HIP(hipGetDevice(&h->device));
    std::vector<int32_t> id(P.n_orig);
    std::iota(id.begin(), id.end(), 0);
    const int64_t no = P.n_orig * o.nrhs_max;
    VTM_HIP(h->vx_src.upload(P.vx_src, s));
    VTM_HIP(h->vx_w.upload(P.vx_w, s));
    VTM_HIP(h->vr0.upload(P.vr0, s));
    VTM_HIP(h->vr1.upload(P.vr1, s));
    VTM_HIP(h->orow.upload(P.orow, s));
    VTM_HIP(h->ocol.upload(P.ocol, s));
    VTM_HIP(h->oval.upload(P.oval, s));
    VTM_HIP(h->oid.upload(id, s));
    if (!P.osymmetric) {
        VTM_HIP(h->orowT.upload(P.orowT, s));
        VTM_HIP(h->ocolT.upload(P.ocolT, s));
        VTM_HIP(h->ovalT.upload(P.ovalT, s));
    }
    VTM_HIP(h->bo.alloc(no));
    VTM_HIP(h->ro.alloc(no));
    VTM_HIP(h->xo.alloc(no));
    VTM_HIP(hipStreamSynchronize(s));
    return setup_from_plan(std::move(h), out);
}

vtm_status vtm_setup_vertex_coupled(const vtm_csr* A, const int32_t* label, const int32_t* iface,
                                    const int32_t* sides, int64_t n_iface, const vtm_csr* W, const vtm_options* opt,
                                    void* stream, vtm_handle* out) {
    return vtm::guarded([&]() -> vtm_status {
        if (!W) return fail(VTM_E_ARG, "null W");
        return setup_vertex_common(A, label, iface, sides, n_iface, nullptr, 0, W, opt, stream, out);
    });
}

static vtm_status check_options(const vtm_options& o) {
    if (o.precision < VTM_FP64 || o.precision > VTM_BF16_REFINE)
        return fail(VTM_E_ARG, "unknown precision");
    if (o.nrhs_max < 1 || o.nrhs_max > 256) return fail(VTM_E_ARG, "nrhs_max outside 1..256");
    if (o.check_every < 1 || o.max_sweeps < 1 || o.max_outer < 0 || !(o.divergence > 0.0))
        return fail(VTM_E_ARG, "bad iteration limits");
    if (o.local_form < 0 || o.local_form > 2) return fail(VTM_E_ARG, "local_form must be 0, 1 or 2");
    if (o.timing < 0 || o.timing > 2) return fail(VTM_E_ARG, "timing must be 0, 1 or 2");
    if ((o.batch_row_tiles != 0 && o.batch_row_tiles != 3 && o.batch_row_tiles != 5) ||
        (o.batch_rhs_block != 0 && (o.batch_rhs_block % 16 != 0 || o.batch_rhs_block > 64 || o.batch_rhs_block < 0)))
        return fail(VTM_E_ARG, "bad batched kernel shape");
    return VTM_OK;
}

// Everything of a handle that depends on the values of A and on the line
// admittances: the uploaded values and port coefficients, the inverses and the
// port-to-port operators.  Setup runs it once; vtm_refresh runs it again on the
// same pattern and partition, so every buffer keeps its size and the same
// kernels run on the same layout.
static vtm_status build_values(vtm_handle_s* h) {
    const vtm_options& o = h->opt;
    const vtm::Plan& P = h->plan;
    hipStream_t s = h->stream;
    const int64_t nk = P.kofs[P.S], nm = P.mofs[P.S];
    VTM_HIP(h->val.upload(P.val, s));
    if (!P.symmetric) {
        std::vector<int32_t> rT, cT;
        std::vector<double> vT;
        vtm::transpose_csr(P, rT, cT, vT);
        VTM_HIP(h->rowptrT.upload(rT, s));
        VTM_HIP(h->colT.upload(cT, s));
        VTM_HIP(h->valT.upload(vT, s));
        VTM_HIP(hipStreamSynchronize(s));
    }
    VTM_HIP(h->dmod.upload(P.dmod, s));
    VTM_HIP(vtm::launch_fill<int>(1, 0, h->flag.p, s));
    DevBuf<double> inv64, panel;  // FP64 inverses, and the elimination's panels
    DevBuf<int32_t> ipiv;
    if (h->tiles || P.max_ns > vtm::kLdsSetupMax) VTM_HIP(inv64.alloc(nk));
    if (P.max_ns > vtm::kLdsSetupMax) {
        VTM_HIP(panel.alloc(vtm::setup_panel_doubles(P.n, P.max_ns)));
        VTM_HIP(ipiv.alloc(P.n));
    }
    // The inversion reads none of the port coefficients: their uploads (staged
    // through host memory by this thread) go on a second stream while its kernels
    // run.  That stream first waits for the work the handle's stream holds before
    // the inversion (nothing still reads the old coefficients then), and the
    // handle's stream waits for the uploads before anything reads them.
    struct Side {
        hipStream_t st = nullptr;
        hipEvent_t before = nullptr, done = nullptr;
        ~Side() {
            if (before) (void)hipEventDestroy(before);
            if (done) (void)hipEventDestroy(done);
            if (st) (void)hipStreamDestroy(st);
        }
    } side;
    VTM_HIP(hipStreamCreateWithFlags(&side.st, hipStreamNonBlocking));
    VTM_HIP(hipEventCreateWithFlags(&side.before, hipEventDisableTiming));
    VTM_HIP(hipEventCreateWithFlags(&side.done, hipEventDisableTiming));
    VTM_HIP(hipEventRecord(side.before, s));
    VTM_HIP(hipStreamWaitEvent(side.st, side.before, 0));
    if (o.precision == VTM_FP64) {
        if (h->tiles) {
            VTM_HIP(h->K64.alloc(nm));
            if (!P.symmetric) VTM_HIP(h->K64T.alloc(nm));
            VTM_HIP(vtm::launch_setup_tiles<double>(int(P.S), P.max_ns, h->sub_off.p, h->kofs.p, h->mofs.p,
                                                    h->rowptr.p, h->col.p, h->val.p, h->dmod.p, h->K64.p, inv64.p,
                                                    panel.p, ipiv.p, h->flag.p, s, h->K64T.p));
        } else {
            VTM_HIP(h->K64.alloc(nk));
            VTM_HIP(vtm::launch_setup<double>(int(P.S), P.max_ns, h->sub_off.p, h->kofs.p, h->rowptr.p, h->col.p,
                                              h->val.p, h->dmod.p, h->K64.p, inv64.p, panel.p, ipiv.p, h->flag.p,
                                              s));
        }
    } else {
        if (h->tiles) {
            VTM_HIP(h->Kbf.alloc(nm));
            if (!P.symmetric) VTM_HIP(h->KbfT.alloc(nm));
            VTM_HIP(vtm::launch_setup_tiles<__bf16>(int(P.S), P.max_ns, h->sub_off.p, h->kofs.p, h->mofs.p,
                                                    h->rowptr.p, h->col.p, h->val.p, h->dmod.p, h->Kbf.p, inv64.p,
                                                    panel.p, ipiv.p, h->flag.p, s, h->KbfT.p));
        } else {
            VTM_HIP(h->K32.alloc(nk));
            VTM_HIP(vtm::launch_setup<float>(int(P.S), P.max_ns, h->sub_off.p, h->kofs.p, h->rowptr.p, h->col.p,
                                             h->val.p, h->dmod.p, h->K32.p, inv64.p, panel.p, ipiv.p, h->flag.p,
                                             s));
        }
    }
    {
        hipStream_t s2 = side.st;
        VTM_HIP(h->c64.upload(P.pc, s2));
        VTM_HIP(h->beta64.upload(P.pbeta, s2));
        VTM_HIP(h->gamma64.upload(P.pgamma, s2));
        if (P.coupled) {
            VTM_HIP(h->bval64.upload(P.bval, s2));
            if (o.precision != VTM_FP64) VTM_HIP(h->bval32.upload(to_float(P.bval), s2));
        }
        if (o.precision != VTM_FP64) {
            VTM_HIP(h->c32.upload(to_float(P.pc), s2));
            VTM_HIP(h->beta32.upload(to_float(P.pbeta), s2));
            VTM_HIP(h->gamma32.upload(to_float(P.pgamma), s2));
        }
        if (h->pp || h->ppb) {
            VTM_HIP(h->pg64.upload(P.pg, s2));
            VTM_HIP(h->pgd64.upload(P.pgd, s2));
        }
        VTM_HIP(hipEventRecord(side.done, s2));
        VTM_HIP(hipStreamWaitEvent(s, side.done, 0));
    }
    VTM_HIP(hipStreamSynchronize(s));
    int flag = 0;
    VTM_HIP(hipMemcpyAsync(&flag, h->flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    VTM_HIP(hipStreamSynchronize(s));
    if (flag & 1) return fail(VTM_E_SINGULAR, "a sub-circuit matrix is singular");
    // port-to-port operators from the inverses
    if (h->ppb) {  // batched form: in tile order, from the FP64 inverses in inv64
        const int64_t nq = P.qmofs[P.S];
        if (o.precision == VTM_FP64) {
            VTM_HIP(h->M64t.alloc(nq));
            VTM_HIP(vtm::launch_port_matrix_tiles<double>(int(P.S), h->sub_off.p, h->kofs.p, h->port_off.p,
                                                          h->port_node.p, h->c64.p, h->beta64.p, h->gamma64.p,
                                                          inv64.p, h->qmofs.p, h->M64t.p, s, h->coupling<double>()));
        } else {
            VTM_HIP(h->Mbt.alloc(nq));
            VTM_HIP(vtm::launch_port_matrix_tiles<__bf16>(int(P.S), h->sub_off.p, h->kofs.p, h->port_off.p,
                                                          h->port_node.p, h->c64.p, h->beta64.p, h->gamma64.p,
                                                          inv64.p, h->qmofs.p, h->Mbt.p, s, h->coupling<double>()));
        }
        VTM_HIP(hipStreamSynchronize(s));
    }
    if (h->ppn) {
        const int64_t nn = P.nofs[P.S];
        if (o.precision == VTM_FP64) {
            VTM_HIP(h->N64.alloc(nn));
            VTM_HIP(vtm::launch_port_node_dense<double>(int(P.S), h->sub_off.p, h->kofs.p, h->pn_off.p, h->pn_node.p,
                                                        h->K64.p, h->nofs.p, h->N64.p, false, s));
            if (!P.symmetric) {
                VTM_HIP(h->N64T.alloc(nn));
                VTM_HIP(vtm::launch_port_node_dense<double>(int(P.S), h->sub_off.p, h->kofs.p, h->pn_off.p,
                                                            h->pn_node.p, h->K64.p, h->nofs.p, h->N64T.p, true, s));
            }
        } else {
            VTM_HIP(h->N32.alloc(nn));
            VTM_HIP(vtm::launch_port_node_dense<float>(int(P.S), h->sub_off.p, h->kofs.p, h->pn_off.p, h->pn_node.p,
                                                       h->K32.p, h->nofs.p, h->N32.p, false, s));
            if (!P.symmetric) {
                VTM_HIP(h->N32T.alloc(nn));
                VTM_HIP(vtm::launch_port_node_dense<float>(int(P.S), h->sub_off.p, h->kofs.p, h->pn_off.p,
                                                           h->pn_node.p, h->K32.p, h->nofs.p, h->N32T.p, true, s));
            }
        }
        VTM_HIP(hipStreamSynchronize(s));
    } else if (h->pps) {
        std::vector<double> Wp;
        if (!P.uniform_W) {  // line admittance per port (both ports of a wire share it)
            Wp.resize(P.nports);
            for (int64_t q = 0; q < P.nports; ++q) Wp[P.abi2port[q]] = P.wW[q / 2];
        }
        const int64_t nsp = P.sofs[P.S];
        if (o.precision == VTM_FP64) {
            VTM_HIP(h->S64.alloc(nsp));
            if (!P.uniform_W)
                VTM_HIP(h->W64p.upload(Wp, s));
            else
                h->W64p.reset();  // one W for every port: the kernel takes it as a scalar
            VTM_HIP(vtm::launch_fill<double>(nsp, double(0), h->S64.p, s));  // pads stay zero
            VTM_HIP(vtm::launch_port_node_matrix<double>(int(P.S), h->sub_off.p, h->kofs.p, h->pn_off.p,
                                                         h->pn_node.p, h->K64.p, h->sofs.p, h->S64.p, s));
        } else {
            VTM_HIP(h->S32.alloc(nsp));
            if (!P.uniform_W)
                VTM_HIP(h->W32p.upload(to_float(Wp), s));
            else
                h->W32p.reset();
            VTM_HIP(vtm::launch_fill<float>(nsp, float(0), h->S32.p, s));  // pads stay zero
            VTM_HIP(vtm::launch_port_node_matrix<float>(int(P.S), h->sub_off.p, h->kofs.p, h->pn_off.p,
                                                        h->pn_node.p, h->K32.p, h->sofs.p, h->S32.p, s));
        }
        VTM_HIP(hipStreamSynchronize(s));
    } else if (h->pp) {
        const int64_t npm = P.pofs[P.S];
        if (o.precision == VTM_FP64) {
            VTM_HIP(h->M64.alloc(npm));
            VTM_HIP(vtm::launch_port_matrix<double>(int(P.S), h->sub_off.p, h->kofs.p, h->port_off.p, h->port_node.p,
                                                    h->c64.p, h->beta64.p, h->gamma64.p, h->K64.p, h->pofs.p,
                                                    h->M64.p, s, h->coupling<double>()));
        } else {
            VTM_HIP(h->M32.alloc(npm));
            VTM_HIP(vtm::launch_port_matrix<float>(int(P.S), h->sub_off.p, h->kofs.p, h->port_off.p, h->port_node.p,
                                                   h->c64.p, h->beta64.p, h->gamma64.p, h->K32.p, h->pofs.p,
                                                   h->M32.p, s, h->coupling<double>()));
        }
        VTM_HIP(hipStreamSynchronize(s));
    }
    return VTM_OK;
}

// The handle's structure (index arrays, work buffers, which local forms run),
// then its values (build_values), then the batched kernels' launch shapes.
static vtm_status setup_from_plan(std::unique_ptr<vtm_handle_s> h, vtm_handle* out) {
    const vtm_options& o = h->opt;
    vtm_status st = VTM_OK;
    VTM_HIP(hipGetDevice(&h->device));
    const vtm::Plan& P = h->plan;
    hipStream_t s = h->stream;

    VTM_HIP(h->rowptr.upload(P.rowptr, s));
    VTM_HIP(h->col.upload(P.col, s));
    VTM_HIP(h->perm.upload(P.perm, s));
    VTM_HIP(h->iperm.upload(P.iperm, s));
    VTM_HIP(h->sub_off.upload(P.sub_off, s));
    VTM_HIP(h->kofs.upload(P.kofs, s));
    VTM_HIP(h->port_off.upload(P.port_off, s));
    VTM_HIP(h->port_node.upload(P.port_node, s));
    VTM_HIP(h->port_slot.upload(P.port_slot, s));
    VTM_HIP(h->port_twin.upload(P.port_twin, s));
    VTM_HIP(h->abi2port.upload(P.abi2port, s));
    VTM_HIP(h->flag.alloc(1));

    const int nr = h->nrhs_max;
    VTM_HIP(h->bp.alloc(P.n * nr));
    VTM_HIP(h->xp.alloc(P.n * nr));
    VTM_HIP(h->partial.alloc(size_t(vtm::kResidBlocks) * nr * 2));
    // the per-column sums of every check go straight to pinned host memory that the
    // device writes over the fabric (a 1 KiB copy through a blit kernel cost ~20 us a check)
    VTM_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->h_norms), sizeof(double) * 2 * nr,
                          hipHostMallocMapped | hipHostMallocCoherent));
    VTM_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&h->red_norms), h->h_norms, 0));
    h->red_partial = h->partial.p;
    int lds = 0;
    VTM_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
    h->lds_limit = size_t(lds > 0 ? lds : 65536);
    // a full sweep stages a sub-circuit's right-hand side in LDS (and its x where both fit)
    if (size_t(P.max_ns) * (o.precision == VTM_FP64 ? 8 : 4) > h->lds_limit)
        return fail(VTM_E_UNSUPPORTED, "a sub-circuit is too large for the sweep's LDS staging of its right-hand side");
    // batched form: MFMA tiles for BF16, and for FP64 handles sized for 16+ right-hand sides
    // when a 16-column block of the largest sub-circuit fits the LDS staging of the batched
    // sweep (else FP64 keeps the column-group layout; BF16 has no other form)
    const int npad = vtm::tile_pad(P.max_ns);
    const size_t mfma_extra = size_t(P.max_ports) * 4 + size_t(npad) * 3 + 4;
    const bool fits64 = vtm::tile_lds_bytes<double>(npad, 16) + mfma_extra <= h->lds_limit;
    const bool fits16 = vtm::tile_lds_bytes<__bf16>(npad, 16) + mfma_extra <= h->lds_limit;
    if (o.precision == VTM_BF16_REFINE && !fits16)
        return fail(VTM_E_UNSUPPORTED, "BF16 path: a sub-circuit is too large for the batched sweep's LDS staging");
    h->tiles = o.precision == VTM_BF16_REFINE || (o.precision == VTM_FP64 && nr >= 16 && fits64);
    if (h->tiles) {
        if (nr > 64 && o.precision == VTM_BF16_REFINE) return fail(VTM_E_UNSUPPORTED, "BF16 path takes at most 64 RHS");
        VTM_HIP(h->mofs.upload(P.mofs, s));
    }
    if (P.coupled) {
        VTM_HIP(h->brow.upload(P.brow, s));
        VTM_HIP(h->bcol.upload(P.bcol, s));
        VTM_HIP(h->port_row.upload(P.port_row, s));
    }
    if (o.precision == VTM_FP64) {
        VTM_HIP(h->a64[0].alloc(P.nports * nr));
        VTM_HIP(h->a64[1].alloc(P.nports * nr));
        VTM_HIP(vtm::launch_fill<double>(P.nports * nr, 0.0, h->a64[0].p, s));
    } else {
        VTM_HIP(h->a32[0].alloc(P.nports * nr));
        VTM_HIP(h->a32[1].alloc(P.nports * nr));
        VTM_HIP(vtm::launch_fill<float>(P.nports * nr, 0.0f, h->a32[0].p, s));
        VTM_HIP(h->rp.alloc(P.n * nr));
        if (h->tiles)
            VTM_HIP(h->b16.alloc(P.n * nr));
        else
            VTM_HIP(h->b32.alloc(P.n * nr));
        VTM_HIP(h->d32.alloc(P.n * nr));
    }
    // which port-to-port operators the handle keeps (they depend on the pattern only)
    h->pp = o.local_form >= 1 && !h->tiles && P.nports > 0;
    // the port-node forms assume diagonal lines (beta and gamma per port)
    h->pps = h->pp && !P.coupled && o.local_form == 1 && P.symmetric && P.max_npn <= 64 && P.max_ports <= 64;
    const size_t ppn_lds = 2 * size_t(P.max_npn) * (o.precision == VTM_FP64 ? 8 : 4) + size_t(P.max_ports) * 4;
    h->ppn = h->pp && !h->pps && !P.coupled && o.local_form == 1 && P.sqn_entries < P.sq_entries &&
             ppn_lds <= 65536;
    const int qpad = vtm::tile_pad(P.max_ports);
    h->ppb = o.local_form >= 1 && h->tiles && P.nports > 0 &&
             (o.precision == VTM_FP64 ? vtm::pp_lds_bytes<double>(qpad, 16, false)
                                      : vtm::pp_lds_bytes<__bf16>(qpad, 16, false)) <= h->lds_limit;
    const bool fp64 = o.precision == VTM_FP64;
    if (h->ppb) {
        VTM_HIP(h->qmofs.upload(P.qmofs, s));
        VTM_HIP(fp64 ? h->h64.alloc(P.nports * nr) : h->h32.alloc(P.nports * nr));
    }
    if (h->pp || h->ppb) VTM_HIP(h->pn_pfirst.upload(P.pn_pfirst, s));
    if (h->ppn || h->pps) {
        VTM_HIP(h->pn_off.upload(P.pn_off, s));
        VTM_HIP(h->pn_node.upload(P.pn_node, s));
        VTM_HIP(h->ppn ? h->nofs.upload(P.nofs, s) : h->sofs.upload(P.sofs, s));
    } else if (h->pp) {
        VTM_HIP(h->pofs.upload(P.pofs, s));
    }
    if (h->pp) VTM_HIP(fp64 ? h->h64.alloc(P.nports) : h->h32.alloc(P.nports));

    if ((st = build_values(h.get())) != VTM_OK) return st;
    if (h->tiles) {
        const TuneKey key{h->device, o.precision, nr, o.batch_row_tiles, o.batch_rhs_block, P.S, P.n, P.nports,
                          P.mofs[P.S], P.qmofs[P.S], P.max_ns, P.max_ports};
        std::array<int, 4> shape{};
        bool cached = false;
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            auto it = g_tune.find(key);
            if (it != g_tune.end()) {
                shape = it->second;
                cached = true;
            }
        }
        if (cached) {
            h->mfma_variant = shape[0];
            h->mfma_rc = shape[1];
            h->pp_variant = shape[2];
            h->pp_rc = shape[3];
        } else {
            st = autotune(h.get());
            if (st != VTM_OK) return st;
            VTM_HIP(hipStreamSynchronize(s));
            std::lock_guard<std::mutex> lock(g_tune_mu);
            g_tune[key] = {h->mfma_variant, h->mfma_rc, h->pp_variant, h->pp_rc};
        }
    }
    *out = h.release();
    return VTM_OK;
}

vtm_status vtm_solve(vtm_handle h, const double* b, double* x, int32_t nrhs, double tol, vtm_report* rep) {
    return vtm::guarded([&]() -> vtm_status {
        return solve_common(h, b, x, nrhs, tol, rep, false);
    });
}

vtm_status vtm_solve_adjoint(vtm_handle h, const double* g, double* lambda, int32_t nrhs, double tol,
                             vtm_report* rep) {
    return vtm::guarded([&]() -> vtm_status {
        return solve_common(h, g, lambda, nrhs, tol, rep, true);
    });
}

vtm_status vtm_solve_noalloc(vtm_handle h, const double* b, double* x, int32_t nrhs, double tol, vtm_report* rep) {
    return vtm::guarded([&]() -> vtm_status {
        if (!h) return fail(VTM_E_ARG, "null handle");
        if (nrhs > kNoallocRhs)
            return fail(VTM_E_UNSUPPORTED, "vtm_solve_noalloc takes at most 64 right-hand sides (its static workspace "
                                           "holds the residual sums of 64 columns)");
        if (h->opt.use_graph || h->opt.timing)
            return fail(VTM_E_UNSUPPORTED, "vtm_solve_noalloc needs use_graph = 0 and timing = 0 (graphs and timing "
                                           "events are runtime objects created on first use)");
        VTM_HIP(hipSetDevice(h->device));
        double* ws = nullptr;
        vtm_status st = scratch_address(h->device, &ws);
        if (st != VTM_OK) return st;
        h->red_partial = ws;
        st = solve_common(h, b, x, nrhs, tol, rep, false);
        h->red_partial = h->partial.p;
        return st;
    });
}

vtm_status vtm_grad(vtm_handle h, const double* x, const double* lambda, int32_t nrhs, const int32_t* branch_ij,
                    int64_t m, double* dL_dg, double* dL_dA_or_null) {
    return vtm::guarded([&]() -> vtm_status {
        if (!h) return fail(VTM_E_ARG, "null handle");
        if (m < 0 || nrhs < 1 || ((m > 0 || dL_dA_or_null) && (!x || !lambda)) || (m > 0 && (!branch_ij || !dL_dg)))
            return fail(VTM_E_ARG, "bad gradient arguments");
        VTM_HIP(hipSetDevice(h->device));
        const int64_t nn = h->plan.vertex ? h->plan.n_orig : h->plan.n;  // the caller's nodes
        if (m > 0) VTM_HIP(vtm::launch_grad(m, int(nn), nrhs, x, lambda, branch_ij, dL_dg, h->stream));
        if (dL_dA_or_null)
            VTM_HIP(vtm::launch_grad_entries(h->a_nnz, int(nn), nrhs, x, lambda, h->erow.p, h->ecol.p, dL_dA_or_null,
                                             h->stream));
        VTM_HIP(hipStreamSynchronize(h->stream));
        return VTM_OK;
    });
}

vtm_status vtm_refresh(vtm_handle h, const double* val, const double* Z, int64_t nZ) {
    return vtm::guarded([&]() -> vtm_status {
        if (!h) return fail(VTM_E_ARG, "null handle");
        VTM_HIP(hipSetDevice(h->device));
        VTM_HIP(hipStreamSynchronize(h->stream));
        std::string err;
        vtm_status st = vtm::refresh_plan(h->plan, val, h->a_nnz, Z, Z ? nZ : 0, err);
        if (st != VTM_OK) return fail(st, err);
        // captured check intervals hold kernel arguments, some of which (the per-port W of
        // the packed form) may now live elsewhere: capture them again when next needed
        for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
        h->graphs.clear();
        h->waves_set = false;
        return build_values(h);
    });
}

vtm_status vtm_get_waves(vtm_handle h, double* waves, int32_t nrhs) {
    return vtm::guarded([&]() -> vtm_status {
        if (!h || !waves || nrhs < 1 || nrhs > h->nrhs_max) return fail(VTM_E_ARG, "bad wave arguments");
        if (h->opt.precision != VTM_FP64)
            return fail(VTM_E_UNSUPPORTED, "checkpoint and resume of the waves need the FP64 precision");
        VTM_HIP(hipSetDevice(h->device));
        VTM_HIP(vtm::launch_waves_io<double>(h->plan.nports, nrhs, h->abi2port.p, h->a64[0].p, waves, true,
                                             h->stream));
        VTM_HIP(hipStreamSynchronize(h->stream));
        return VTM_OK;
    });
}

vtm_status vtm_set_waves(vtm_handle h, const double* waves, int32_t nrhs) {
    return vtm::guarded([&]() -> vtm_status {
        if (!h || !waves || nrhs < 1 || nrhs > h->nrhs_max) return fail(VTM_E_ARG, "bad wave arguments");
        if (h->opt.precision != VTM_FP64)
            return fail(VTM_E_UNSUPPORTED, "checkpoint and resume of the waves need the FP64 precision");
        VTM_HIP(hipSetDevice(h->device));
        VTM_HIP(vtm::launch_waves_io<double>(h->plan.nports, nrhs, h->abi2port.p, h->a64[0].p,
                                             const_cast<double*>(waves), false, h->stream));
        VTM_HIP(hipStreamSynchronize(h->stream));
        h->waves_set = true;
        return VTM_OK;
    });
}

vtm_status vtm_info(vtm_handle h, int64_t* n, int64_t* n_sub, int64_t* n_wires, int64_t* inverse_bytes,
                    int64_t* port_operator_bytes, int64_t* port_sweep_bytes) {
    return vtm::guarded([&]() -> vtm_status {
        if (!h) return fail(VTM_E_ARG, "null handle");
        const vtm::Plan& P = h->plan;
        const int64_t esize = h->opt.precision == VTM_FP64 ? 8 : (h->opt.precision == VTM_FP32_REFINE ? 4 : 2);
        if (n) *n = P.n;
        if (n_sub) *n_sub = P.S;
        if (n_wires) *n_wires = P.nwires;
        if (inverse_bytes) *inverse_bytes = (h->tiles ? P.mofs[P.S] : P.kofs[P.S]) * esize;
        const int64_t op = h->ppb   ? P.qmofs[P.S] * esize
                           : h->ppn ? P.nofs[P.S] * esize
                           : h->pps ? P.sofs[P.S] * esize
                           : h->pp  ? P.pofs[P.S] * esize
                                    : 0;
        if (port_operator_bytes) *port_operator_bytes = op;
        if (port_sweep_bytes) *port_sweep_bytes = pp_sweep_bytes(h, h->nrhs_max);
        return VTM_OK;
    });
}

void vtm_destroy(vtm_handle h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

}  // extern "C"
