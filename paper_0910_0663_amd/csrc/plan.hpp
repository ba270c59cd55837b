// Host tearing planner: turns (A, node partition, Z) into the per-sub-circuit
// data the device kernels consume.  Integer work plus the per-wire port
// coefficients; no device calls.
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "vtm.h"

namespace vtm {

// An allocator whose value-initialization is default-initialization, so that
// resize() leaves trivial elements unwritten: for large buffers that host threads
// then fill whole (their pages are first touched by those threads instead of
// being zeroed on one).
template <typename T>
struct NoInit : std::allocator<T> {
    using std::allocator<T>::allocator;
    template <typename U>
    struct rebind {
        using other = NoInit<U>;
    };
    template <typename U>
    void construct(U* p) noexcept {
        ::new (static_cast<void*>(p)) U;
    }
    template <typename U, typename... Args>
    void construct(U* p, Args&&... args) {
        ::new (static_cast<void*>(p)) U(std::forward<Args>(args)...);
    }
};
template <typename T>
using scratch_vec = std::vector<T, NoInit<T>>;

struct Plan {
    int64_t n = 0;        // nodes
    int64_t S = 0;        // sub-circuits
    int64_t nwires = 0;   // cut wires
    int64_t nports = 0;   // 2 * nwires
    int32_t max_ns = 0;   // largest sub-circuit
    int32_t max_slot = 0; // most ports on one node, minus one
    bool symmetric = false;

    // Sub-circuit-major renumbering: inside each sub-circuit its port nodes (the
    // ends of its lines) first, then its other nodes, ascending old id in each group.
    std::vector<int32_t> perm;     // new -> old
    std::vector<int32_t> iperm;    // old -> new
    std::vector<int32_t> sub_off;  // [S + 1] first new id of each sub-circuit
    std::vector<int64_t> kofs;     // [S + 1] element offset of each dense inverse
    std::vector<int64_t> mofs;     // [S + 1] element offset of each padded MFMA tile block
    std::vector<int64_t> pofs;     // [S + 1] element offset of each port-to-port operator (q_s x q_s)
    std::vector<int64_t> qmofs;    // [S + 1] element offset of each port operator in MFMA tiles (padded q_s)
    // Port nodes: the distinct nodes carrying ports, per sub-circuit in port order.
    std::vector<int32_t> pn_off;    // [S + 1] first port node of each sub-circuit
    std::vector<int32_t> pn_node;   // local node of each port node
    std::vector<int32_t> pn_pfirst; // [n_port_nodes + 1] first port of each port node (ports of one
                                    // node are consecutive; the last entry is nports)
    std::vector<int64_t> sofs;      // [S + 1] element offset of each packed symmetric block
    int32_t max_npn = 0;            // most port nodes on one sub-circuit
    int64_t tri_entries = 0;        // sum over sub-circuits of k (k + 1) / 2 (packed triangles, no padding)
    int64_t sq_entries = 0;         // sum over sub-circuits of q^2 (dense port operators, no padding)
    int64_t sqn_entries = 0;        // sum over sub-circuits of k^2 (port-node operators, no padding)
    std::vector<int64_t> nofs;      // [S + 1] element offset of each k x k port-node operator
    bool uniform_W = true;          // one line admittance for every wire

    int32_t max_ports = 0;         // most ports on one sub-circuit

    // Cut wires in canonical order (lower node, then upper node, ascending; old ids).
    std::vector<int32_t> wi, wj;
    std::vector<double> wg;        // branch conductance g = -A_ij
    std::vector<double> wW;        // line admittance W = 1 / Z

    // Ports: two per wire, grouped by sub-circuit, inside one by (local node, wire).
    std::vector<int32_t> port_off;   // [S + 1]
    scratch_vec<int32_t> port_node;  // local node index inside its sub-circuit
    scratch_vec<int32_t> port_slot;  // rank among the ports of the same node
    scratch_vec<int32_t> port_twin;  // the other port of the same wire
    scratch_vec<int32_t> abi2port;   // [2 * nwires]: ABI port (2e lower, 2e+1 upper) -> port
    scratch_vec<double> pc, pbeta, pgamma;  // per port: c, beta, gamma
    scratch_vec<double> pg, pgd;            // per port: wire conductance g and G - g

    std::vector<double> dmod;      // per new node: sum over its ports of (G - g)

    // The untorn A renumbered (rows and columns), duplicates merged, columns sorted.
    std::vector<int32_t> rowptr;
    scratch_vec<int32_t> col;
    scratch_vec<double> val;
    // a refresh merges new values here and swaps it with val once they pass every
    // check (kept between refreshes, so its pages are not faulted in again)
    scratch_vec<double> val_spare;
    // How the caller's entries became it (not for tearing at nodes): the caller's
    // entry indices in the order they are summed, per position a flag (bit 0: first
    // entry of a merged entry, bit 1: a diagonal one) and the renumbered entry the
    // sum goes to (-1: an explicit zero off the diagonal, dropped).
    scratch_vec<int32_t> src_ent, src_dst;
    scratch_vec<uint8_t> src_flag;
    // For the refresh's checks (same plans): per renumbered entry (r, c) the position
    // of (c, r), -1 if the pattern lacks it; per cut wire e the positions of its two
    // entries (r, c) and (c, r), at 2 e and 2 e + 1.
    scratch_vec<int32_t> tpos, wpos;

    // Tearing at interfacial nodes (build_plan_vertex): the plan above describes the
    // expanded system (every interfacial node replaced by two twins); these map it
    // to and from the caller's n_orig nodes.
    bool vertex = false;
    int64_t n_orig = 0;
    std::vector<int32_t> vx_src;   // per plan row: the original node it comes from
    std::vector<double> vx_w;      // per plan row: its share of that node's source (1 or 1/2)
    std::vector<int32_t> vr0, vr1; // per original node: its plan row(s); vr1 = -1 unless a twin pair
    std::vector<int32_t> orow, ocol;  // the caller's A, duplicates merged (residual on the untorn system)
    std::vector<double> oval;
    bool osymmetric = true;            // the caller's A is symmetric; else its transpose follows
    std::vector<int32_t> orowT, ocolT; // (for the adjoint's residual)
    std::vector<double> ovalT;

    // Coupled lines (a non-diagonal W over the interfacial nodes, eqs. 4-5): W is
    // part of the torn matrix (added between the twins of each side), so the
    // ports add no conductance (G = 0, c = 1, gamma = -1), and the outgoing wave
    // of port p is sum_m B_pm u_node(m) - a_p with B = 2 W, rows and columns
    // over the plan's ports (m in p's sub-circuit).  pbeta keeps B's diagonal.
    bool coupled = false;
    std::vector<int32_t> brow, bcol;  // CSR of B over plan ports
    std::vector<double> bval;
    std::vector<int32_t> port_row;    // plan row of every port's node
};

// Largest sub-circuit a plan accepts (its FP64 inverse is 2 GiB; a single
// right-hand side's full sweep stages 8 bytes per node in LDS, within gfx950's
// 160 KiB per workgroup; several right-hand sides or the adjoint need 16 bytes
// per node per right-hand side, so at most 10,240 nodes).
constexpr int64_t kMaxSubCircuit = 16384;

// Builds the plan; on failure returns the status and sets err.  With lines
// (line_a, line_b: n_lines pairs of nodes in different sub-circuits, not coupled
// by A) the lines are those pairs, each a line with no branch (vertex tearing),
// and A may couple no two sub-circuits; without, the lines are A's cut branches.
vtm_status build_plan(const vtm_csr* A, const int32_t* part, const double* Z, int64_t nZ,
                      Plan& plan, std::string& err, const int32_t* line_a = nullptr,
                      const int32_t* line_b = nullptr, int64_t n_lines = 0);

// The system torn at interfacial nodes, before renumbering: nodes 0..n-1 keep
// their ids (an interfacial node's id now names its twin in sides[2l]); node n + l
// is the twin of iface[l] in sides[2l + 1].
struct VertexSplit {
    int64_t n = 0, L = 0;
    std::vector<int64_t> rowptr;   // n + L + 1
    std::vector<int32_t> col;
    std::vector<double> val;
    std::vector<int32_t> part;     // n + L sub-circuit labels
    std::vector<int32_t> orow, ocol;  // the caller's A, duplicates merged, columns sorted
    std::vector<double> oval;
};

// Steps 2-3 of the vertex tearing below (no lines yet); err set on failure.
vtm_status split_at_vertices(const vtm_csr* A, const int32_t* label, const int32_t* iface,
                             const int32_t* sides, int64_t n_iface, VertexSplit& out, std::string& err);

// Rule 5 of Section VIII on a torn system: per group of lines whose twins lie
// in the same two sub-circuits (same order), W = C - E~ D~^-1 F~ over the twins
// of one side, D~ the inner nodes of that side's sub-circuit within `depth`
// hops of them (depth < 0: all), symmetrized, off-diagonal entries below
// drop * sqrt(|w_ii w_jj|) dropped.  Rows (lines) of sorted (line, value).
vtm_status partial_schur_vertex(const VertexSplit& X, const int32_t* iface, const int32_t* sides, int side,
                                int depth, double drop, std::vector<std::vector<std::pair<int32_t, double>>>& W,
                                std::string& err);

// Tearing at interfacial nodes (Section V, Steps 1-4, as the paper tears):
// every node iface[l] is split into two twins, one in each of the sub-circuits
// sides[2l] and sides[2l + 1], joined by a line of admittance W[l] (nW == 1: one
// W for all).  Other nodes keep label[i].  The plan describes the expanded
// system and carries the maps back to the caller's nodes.
// With Wc (an n_iface x n_iface CSR, symmetric, positive diagonal, coupling
// only lines whose twins lie in the same two sub-circuits, in the same order)
// the lines are coupled and W, nW are ignored.
vtm_status build_plan_vertex(const vtm_csr* A, const int32_t* label, const int32_t* iface,
                             const int32_t* sides, int64_t n_iface, const double* W, int64_t nW,
                             Plan& plan, std::string& err, const vtm_csr* Wc = nullptr);

// New values for the caller's A on the same pattern (val: nnz values in the
// caller's entry order) and optionally new line impedances (nZ 0: keep; 1 or
// n_wires as for build_plan): updates the renumbered values, the cut wires'
// conductances, the port coefficients and the diagonal changes exactly as
// build_plan would form them.  Errors: a pattern change (an off-diagonal entry
// becoming or ceasing to be zero), a change of symmetry, an untearable cut, a
// plan built for tearing at nodes; the plan is unchanged then.
vtm_status refresh_plan(Plan& plan, const double* val, int64_t nnz, const double* Z, int64_t nZ, std::string& err);

// Renumbered A^T in compressed rows (columns sorted).
void transpose_csr(const Plan& plan, std::vector<int32_t>& rowptr, std::vector<int32_t>& col,
                   std::vector<double>& val);

// Port coefficients of a cut wire with conductance g and line admittance W.
struct PortCoef {
    double G, c, beta, gamma;
};
PortCoef port_coef(double g, double W);

}  // namespace vtm
