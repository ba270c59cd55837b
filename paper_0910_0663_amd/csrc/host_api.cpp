// C ABI calls that run on the host only: options, status strings, the last
// error, the tearing plan, the torn system of tearing at nodes and the line
// admittance rules of Section VIII.  Plain C++ (no device code), so that a
// CPU build with sanitizers can exercise them.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "plan.hpp"
#include "status.hpp"
#include "vtm.h"

namespace vtm {

namespace {
thread_local std::string g_err;
}  // namespace

vtm_status fail(vtm_status s, const std::string& msg) noexcept {
    try {
        g_err = msg;
    } catch (...) {  // no memory for the message: keep the status
        g_err.clear();
    }
    return s;
}

vtm_status fail(vtm_status s, const char* msg) noexcept {
    try {
        g_err = msg;
    } catch (...) {
        g_err.clear();
    }
    return s;
}

const char* last_error() { return g_err.c_str(); }

}  // namespace vtm

using vtm::fail;

extern "C" {

void vtm_default_options(vtm_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = VTM_FP64;
    opt->nrhs_max = 1;
    opt->check_every = 8;
    opt->max_outer = 30;
    opt->max_sweeps = 1000000;
    opt->divergence = 1e6;
    opt->inner_drop = 0.0;
    opt->use_graph = 0;
    opt->timing = 0;
    opt->adaptive_checks = 1;
    opt->batch_row_tiles = 0;
    opt->batch_rhs_block = 0;
    opt->local_form = 1;
}

const char* vtm_status_str(vtm_status s) {
    switch (s) {
        case VTM_OK: return "VTM_OK";
        case VTM_E_ARG: return "VTM_E_ARG";
        case VTM_E_UNTEARABLE: return "VTM_E_UNTEARABLE";
        case VTM_E_SINGULAR: return "VTM_E_SINGULAR";
        case VTM_E_DIVERGED: return "VTM_E_DIVERGED";
        case VTM_E_MAXITER: return "VTM_E_MAXITER";
        case VTM_E_HIP: return "VTM_E_HIP";
        case VTM_E_OOM: return "VTM_E_OOM";
        case VTM_E_UNSUPPORTED: return "VTM_E_UNSUPPORTED";
    }
    return "VTM_E_UNKNOWN";
}

const char* vtm_last_error(void) { return vtm::last_error(); }

vtm_status vtm_plan(const vtm_csr* A, const int32_t* part, const double* Z, int64_t nZ, int64_t* n_sub,
                    int64_t* n_wires, int32_t* wires, double* coef) {
    return vtm::guarded([&]() -> vtm_status {
        vtm::Plan P;
        std::string err;
        vtm_status st = vtm::build_plan(A, part, Z, nZ, P, err);
        if (st != VTM_OK) return fail(st, err);
        if (n_sub) *n_sub = P.S;
        if (n_wires) *n_wires = P.nwires;
        for (int64_t e = 0; e < P.nwires; ++e) {
            if (wires) {
                wires[2 * e] = P.wi[e];
                wires[2 * e + 1] = P.wj[e];
            }
            if (coef) {
                const vtm::PortCoef k = vtm::port_coef(P.wg[e], P.wW[e]);
                coef[4 * e + 0] = k.G;
                coef[4 * e + 1] = k.c;
                coef[4 * e + 2] = k.beta;
                coef[4 * e + 3] = k.gamma;
            }
        }
        return VTM_OK;
    });
}

vtm_status vtm_split_vertex(const vtm_csr* A, const int32_t* label, const int32_t* iface, const int32_t* sides,
                            int64_t n_iface, int64_t* n_torn, int64_t* nnz, int64_t* rowptr, int32_t* col,
                            double* val, int32_t* part) {
    return vtm::guarded([&]() -> vtm_status {
        vtm::VertexSplit X;
        std::string err;
        vtm_status st = vtm::split_at_vertices(A, label, iface, sides, n_iface, X, err);
        if (st != VTM_OK) return fail(st, err);
        if (n_torn) *n_torn = X.n + X.L;
        if (nnz) *nnz = int64_t(X.col.size());
        if (rowptr) std::copy(X.rowptr.begin(), X.rowptr.end(), rowptr);
        if (col) std::copy(X.col.begin(), X.col.end(), col);
        if (val) std::copy(X.val.begin(), X.val.end(), val);
        if (part) std::copy(X.part.begin(), X.part.end(), part);
        return VTM_OK;
    });
}

// mean conductance of A's two-terminal branches (symmetric negative off-diagonal
// pairs, each counted once); false when there is none
static bool mean_branch(const vtm_csr* A, double& mean) {
    double sum = 0.0;
    int64_t cnt = 0;
    for (int64_t i = 0; i < A->n; ++i)
        for (int64_t q = A->rowptr[i]; q < A->rowptr[i + 1]; ++q) {
            const int64_t j = A->col[q];
            const double v = A->val[q];
            if (j <= i || !(v < 0.0)) continue;
            double vt = 0.0;
            for (int64_t r = A->rowptr[j]; r < A->rowptr[j + 1]; ++r)
                if (A->col[r] == i) vt += A->val[r];
            if (vt == v) {
                sum += -v;
                ++cnt;
            }
        }
    if (cnt == 0) return false;
    mean = sum / double(cnt);
    return true;
}

vtm_status vtm_line_admittance(const vtm_csr* A, const int32_t* part, int32_t kind, double alpha, double* W,
                               int64_t n_wires) {
    return vtm::guarded([&]() -> vtm_status {
        if (!W) return fail(VTM_E_ARG, "null output");
        if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(VTM_E_ARG, "alpha must be positive");
        if (kind < VTM_W_SCALED_MEAN || kind > VTM_W_DIAG) return fail(VTM_E_ARG, "unknown admittance rule");
        vtm::Plan P;
        std::string err;
        const double one = 1.0;
        vtm_status st = vtm::build_plan(A, part, &one, 1, P, err);
        if (st != VTM_OK) return fail(st, err);
        if (n_wires != P.nwires) return fail(VTM_E_ARG, "n_wires does not match the partition's cut wires");
        double mean = 0.0;
        if (kind == VTM_W_SCALED_MEAN && !mean_branch(A, mean)) return fail(VTM_E_ARG, "A has no two-terminal branch");
        for (int64_t e = 0; e < P.nwires; ++e) {
            const double g = P.wg[e];
            switch (kind) {
                case VTM_W_SCALED_MEAN: W[e] = alpha * mean; break;
                case VTM_W_IDENTITY: W[e] = alpha; break;
                case VTM_W_OB:
                case VTM_W_DIAG: W[e] = 2.0 * g; break;
                default: W[e] = alpha * 2.0 * g; break;
            }
        }
        return VTM_OK;
    });
}

vtm_status vtm_vertex_sca(const vtm_csr* A, const int32_t* label, const int32_t* iface, const int32_t* sides,
                          int64_t n_iface, int32_t side, int32_t depth, double drop, int64_t* nnz, int64_t* rowptr,
                          int32_t* col, double* val) {
    return vtm::guarded([&]() -> vtm_status {
        if (side != 0 && side != 1) return fail(VTM_E_ARG, "side must be 0 or 1");
        if (!(drop >= 0.0) || !std::isfinite(drop)) return fail(VTM_E_ARG, "drop must be finite and non-negative");
        vtm::VertexSplit X;
        std::string err;
        vtm_status st = vtm::split_at_vertices(A, label, iface, sides, n_iface, X, err);
        if (st != VTM_OK) return fail(st, err);
        std::vector<std::vector<std::pair<int32_t, double>>> W;
        st = vtm::partial_schur_vertex(X, iface, sides, side, depth, drop, W, err);
        if (st != VTM_OK) return fail(st, err);
        int64_t k = 0;
        if (rowptr) rowptr[0] = 0;
        for (int64_t l = 0; l < n_iface; ++l) {
            for (const auto& e : W[l]) {
                if (col) col[k] = e.first;
                if (val) val[k] = e.second;
                ++k;
            }
            if (rowptr) rowptr[l + 1] = k;
        }
        if (nnz) *nnz = k;
        return VTM_OK;
    });
}

vtm_status vtm_vertex_admittance(const vtm_csr* A, const int32_t* label, const int32_t* iface, const int32_t* sides,
                                 int64_t n_iface, int32_t kind, double alpha, int32_t side, int64_t* nnz,
                                 int64_t* rowptr, int32_t* col, double* val) {
    return vtm::guarded([&]() -> vtm_status {
        if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(VTM_E_ARG, "alpha must be positive");
        if (kind < VTM_W_SCALED_MEAN || kind > VTM_W_DIAG) return fail(VTM_E_ARG, "unknown admittance rule");
        if (side != 0 && side != 1) return fail(VTM_E_ARG, "side must be 0 or 1");
        vtm::VertexSplit X;
        std::string err;
        vtm_status st = vtm::split_at_vertices(A, label, iface, sides, n_iface, X, err);
        if (st != VTM_OK) return fail(st, err);
        const int64_t n = X.n, L = n_iface;
        // C: the block of the torn matrix over the twins on the chosen side (line ids),
        // symmetrized (W must be symmetric; C is when A is)
        std::vector<std::map<int32_t, double>> C(L);
        if (kind == VTM_W_SCALED_MEAN || kind == VTM_W_IDENTITY) {
            double mean = 1.0;
            if (kind == VTM_W_SCALED_MEAN && !mean_branch(A, mean)) return fail(VTM_E_ARG, "A has no two-terminal branch");
            for (int64_t l = 0; l < L; ++l) C[l][int32_t(l)] = alpha * mean;
        } else {
            std::vector<int64_t> line_of(n + L, -1);
            for (int64_t l = 0; l < L; ++l) line_of[side ? n + l : iface[l]] = l;
            for (int64_t l = 0; l < L; ++l) {
                const int64_t r = side ? n + l : iface[l];
                for (int64_t q = X.rowptr[r]; q < X.rowptr[r + 1]; ++q) {
                    const int64_t m = line_of[X.col[q]];
                    if (m < 0 || (kind == VTM_W_DIAG && m != l)) continue;
                    const double w = (kind == VTM_W_WOB ? alpha : 1.0) * 0.5 * X.val[q];
                    C[l][int32_t(m)] += w;
                    C[m][int32_t(l)] += w;
                }
            }
            for (int64_t l = 0; l < L; ++l)
                if (!(C[l][int32_t(l)] > 0.0)) return fail(VTM_E_ARG, "the interface block has a non-positive diagonal");
        }
        int64_t k = 0;
        if (rowptr) rowptr[0] = 0;
        for (int64_t l = 0; l < L; ++l) {
            for (const auto& e : C[l]) {
                if (col) col[k] = e.first;
                if (val) val[k] = e.second;
                ++k;
            }
            if (rowptr) rowptr[l + 1] = k;
        }
        if (nnz) *nnz = k;
        return VTM_OK;
    });
}

}  // extern "C"
