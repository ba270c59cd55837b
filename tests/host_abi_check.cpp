// Host-only parts of the library under AddressSanitizer / UndefinedBehaviorSanitizer
// and ThreadSanitizer (built with g++ by tests/test_host_sanitizers.py): the
// tearing planner (with a circuit large enough for its passes to run on several
// host threads) and its refresh, and the host-only C ABI calls (vtm_plan, vtm_split_vertex,
// vtm_line_admittance, vtm_vertex_admittance, vtm_vertex_sca, status strings,
// options) on valid circuits and on malformed input.  Exit status 0 when every
// check holds; a sanitizer report aborts the run.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <map>
#include <random>
#include <string>
#include <vector>

#include "plan.hpp"
#include "vtm.h"

namespace {

int g_failures = 0;

void check(bool ok, const std::string& what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (last error: %s)\n", what.c_str(), vtm_last_error());
        ++g_failures;
    }
}

// A resistor grid (ny x nx, 5-point) with random branch conductances and 0.01 S
// to ground, assembled as COO rows, optionally with a duplicated diagonal half
// and rows in reverse column order.
struct Csr {
    int64_t n = 0;
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col;
    std::vector<double> val;
    vtm_csr view() const { return vtm_csr{n, int64_t(col.size()), rowptr.data(), col.data(), val.data()}; }
};

Csr grid(int ny, int nx, unsigned seed, bool duplicates, double vccs_gain = 0.0) {
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> g(0.5, 2.0);
    const int n = ny * nx;
    std::vector<std::vector<std::pair<int32_t, double>>> rows(n);
    std::vector<double> diag(n, 0.01);
    auto branch = [&](int i, int j) {
        const double v = g(rng);
        rows[i].push_back({j, -v});
        rows[j].push_back({i, -v});
        diag[i] += v;
        diag[j] += v;
    };
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (x + 1 < nx) branch(y * nx + x, y * nx + x + 1);
            if (y + 1 < ny) branch(y * nx + x, (y + 1) * nx + x);
        }
    if (vccs_gain != 0.0) rows[1].push_back({int32_t(nx + 1), vccs_gain});  // one-sided entry (inside a block)
    Csr A;
    A.n = n;
    A.rowptr.push_back(0);
    for (int i = 0; i < n; ++i) {
        if (duplicates) {
            rows[i].push_back({i, 0.5 * diag[i]});
            rows[i].push_back({i, 0.5 * diag[i]});
        } else {
            rows[i].push_back({i, diag[i]});
        }
        for (auto it = rows[i].rbegin(); it != rows[i].rend(); ++it) {
            A.col.push_back(it->first);
            A.val.push_back(it->second);
        }
        A.rowptr.push_back(int64_t(A.col.size()));
    }
    return A;
}

std::vector<int32_t> blocks(int ny, int nx, int by, int bx) {
    std::vector<int32_t> part(ny * nx);
    const int nbx = (nx + bx - 1) / bx;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) part[y * nx + x] = (y / by) * nbx + x / bx;
    return part;
}

void plan_checks() {
    const Csr A = grid(24, 20, 1, true);
    const vtm_csr a = A.view();
    const auto part = blocks(24, 20, 8, 5);
    const double Z = 0.8;
    int64_t S = 0, nw = 0;
    check(vtm_plan(&a, part.data(), &Z, 1, &S, &nw, nullptr, nullptr) == VTM_OK, "plan counts");
    check(S == 12, "sub-circuit count");
    check(nw == 3 * 24 + 2 * 20, "cut wire count");  // 3 block-column boundaries of 24 rows, 2 block-row boundaries of 20 columns
    std::vector<int32_t> wires(2 * nw);
    std::vector<double> coef(4 * nw);
    check(vtm_plan(&a, part.data(), &Z, 1, nullptr, nullptr, wires.data(), coef.data()) == VTM_OK, "plan fill");
    for (int64_t e = 0; e < nw; ++e) {
        check(wires[2 * e] < wires[2 * e + 1], "canonical wire");
        const double G = coef[4 * e], c = coef[4 * e + 1], beta = coef[4 * e + 2], gamma = coef[4 * e + 3];
        check(std::fabs(beta - 2.0 * c / Z) <= 1e-14 * beta && std::fabs(gamma - (1.0 - 2.0 * c)) <= 1e-14,
              "beta = 2 W c, gamma = 1 - 2 c");
        check(G > 0.0 && c > 0.0 && c < 1.0, "port coefficients in range");
    }
    // per-wire impedances, and every malformed input the planner rejects
    std::vector<double> Zw(nw, 0.5);
    check(vtm_plan(&a, part.data(), Zw.data(), nw, nullptr, nullptr, nullptr, nullptr) == VTM_OK, "per-wire Z");
    check(vtm_plan(&a, part.data(), Zw.data(), nw - 1, nullptr, nullptr, nullptr, nullptr) == VTM_E_ARG, "nZ");
    const double bad_z = -1.0;
    check(vtm_plan(&a, part.data(), &bad_z, 1, nullptr, nullptr, nullptr, nullptr) == VTM_E_ARG, "Z <= 0");
    check(vtm_plan(nullptr, part.data(), &Z, 1, nullptr, nullptr, nullptr, nullptr) == VTM_E_ARG, "null A");
    Csr B = A;
    B.col[3] = int32_t(B.n);
    vtm_csr b = B.view();
    check(vtm_plan(&b, part.data(), &Z, 1, nullptr, nullptr, nullptr, nullptr) == VTM_E_ARG, "column range");
    B = A;
    B.val[5] = NAN;
    b = B.view();
    check(vtm_plan(&b, part.data(), &Z, 1, nullptr, nullptr, nullptr, nullptr) == VTM_E_ARG, "non-finite");
    B = A;
    B.rowptr[7] = B.rowptr[8] + 1;
    b = B.view();
    check(vtm_plan(&b, part.data(), &Z, 1, nullptr, nullptr, nullptr, nullptr) == VTM_E_ARG, "rowptr order");
    auto p2 = part;
    for (auto& v : p2)
        if (v == 11) v = 12;  // label 11 unused
    check(vtm_plan(&a, p2.data(), &Z, 1, nullptr, nullptr, nullptr, nullptr) == VTM_E_ARG, "unused label");
    // a one-sided coupling across the cut: untearable
    const Csr C = grid(24, 20, 2, false);
    Csr D = C;
    for (int64_t q = D.rowptr[4]; q < D.rowptr[5]; ++q)
        if (D.col[q] == 5) D.val[q] *= 1.5;  // nodes 4 and 5 lie in different blocks (bx = 5)
    vtm_csr d = D.view();
    check(vtm_plan(&d, part.data(), &Z, 1, nullptr, nullptr, nullptr, nullptr) == VTM_E_UNTEARABLE, "untearable");
    // line admittance rules
    std::vector<double> W(nw);
    for (int kind = VTM_W_SCALED_MEAN; kind <= VTM_W_DIAG; ++kind)
        check(vtm_line_admittance(&a, part.data(), kind, 0.5, W.data(), nw) == VTM_OK, "line admittance rule");
    check(vtm_line_admittance(&a, part.data(), 7, 0.5, W.data(), nw) == VTM_E_ARG, "bad rule");
    check(vtm_line_admittance(&a, part.data(), VTM_W_OB, 1.0, W.data(), nw + 1) == VTM_E_ARG, "wire count");
}

// The numbering the sweeps' port-row forms rely on: in every sub-circuit the
// port nodes are its first local nodes (0 .. k-1, every one carrying a port),
// and the renumbering is a permutation that keeps each node in its sub-circuit.
bool port_nodes_first(const vtm::Plan& P, const int32_t* part) {
    for (int64_t r = 0; r < P.n; ++r)
        if (P.iperm[P.perm[r]] != r) return false;
    for (int64_t s = 0; s < P.S; ++s) {
        for (int32_t r = P.sub_off[s]; r < P.sub_off[s + 1]; ++r)
            if (part && part[P.perm[r]] != s) return false;
        const int32_t p0 = P.port_off[s], p1 = P.port_off[s + 1];
        int32_t k = 0;  // distinct port nodes, in order
        for (int32_t p = p0; p < p1; ++p) {
            if (p > p0 && P.port_node[p] == P.port_node[p - 1]) continue;
            if (P.port_node[p] != k) return false;
            ++k;
        }
    }
    return true;
}

void refresh_checks() {
    // refresh of a plan against a fresh plan of the new values, bit for bit
    const auto part = blocks(24, 20, 8, 5);
    for (double gain : {0.0, 0.3}) {
        const Csr A = grid(24, 20, 3, true, gain), A2 = grid(24, 20, 4, true, gain);
        const vtm_csr a = A.view(), a2 = A2.view();
        const double Z = 0.8, Z2 = 1.3;
        vtm::Plan P, Q;
        std::string err;
        check(vtm::build_plan(&a, part.data(), &Z, 1, P, err) == VTM_OK, "build plan");
        check(vtm::build_plan(&a2, part.data(), &Z2, 1, Q, err) == VTM_OK, "build plan of the new values");
        check(vtm::refresh_plan(P, A2.val.data(), int64_t(A2.val.size()), &Z2, 1, err) == VTM_OK, "refresh");
        check(P.val == Q.val && P.dmod == Q.dmod && P.pc == Q.pc && P.pbeta == Q.pbeta && P.pgamma == Q.pgamma &&
                  P.pg == Q.pg && P.pgd == Q.pgd && P.wg == Q.wg && P.wW == Q.wW,
              "refreshed plan equals a fresh plan");
        // refused changes leave the plan as it was
        const auto before = P.val;
        std::vector<double> v = A2.val;
        int64_t off = -1;  // an off-diagonal entry inside a block
        for (int64_t q = A2.rowptr[0]; q < A2.rowptr[1]; ++q)
            if (A2.col[q] == 1) off = q;
        v[off] = 0.0;
        check(vtm::refresh_plan(P, v.data(), int64_t(v.size()), nullptr, 0, err) == VTM_E_ARG, "pattern change");
        v = A2.val;
        v[off] *= 1.25;
        check(vtm::refresh_plan(P, v.data(), int64_t(v.size()), nullptr, 0, err) ==
                  (gain == 0.0 ? VTM_E_UNSUPPORTED : VTM_OK),
              "symmetry change (the circuit with a controlled source stays unsymmetric)");
        if (gain == 0.0) check(P.val == before, "plan unchanged after a refused refresh");
        check(vtm::refresh_plan(P, v.data(), int64_t(v.size()) - 1, nullptr, 0, err) == VTM_E_ARG, "entry count");
    }
}

void vertex_checks() {
    // a 12 x 13 grid torn at its middle column into two strips
    const int ny = 12, nx = 13;
    const Csr A = grid(ny, nx, 5, false);
    const vtm_csr a = A.view();
    std::vector<int32_t> label(ny * nx), iface, sides;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) label[y * nx + x] = x < 6 ? 0 : 1;
    for (int y = 0; y < ny; ++y) {
        iface.push_back(y * nx + 6);
        sides.push_back(0);
        sides.push_back(1);
    }
    const int64_t L = int64_t(iface.size());
    int64_t nt = 0, nnz = 0;
    check(vtm_split_vertex(&a, label.data(), iface.data(), sides.data(), L, &nt, &nnz, nullptr, nullptr, nullptr,
                           nullptr) == VTM_OK,
          "split sizes");
    check(nt == A.n + L, "torn node count");
    std::vector<int64_t> rp(nt + 1);
    std::vector<int32_t> col(nnz), part(nt);
    std::vector<double> val(nnz);
    check(vtm_split_vertex(&a, label.data(), iface.data(), sides.data(), L, nullptr, nullptr, rp.data(), col.data(),
                           val.data(), part.data()) == VTM_OK,
          "split fill");
    double sum_torn = 0.0, sum_orig = 0.0;  // the split conserves the sum of all entries
    for (double v : val) sum_torn += v;
    for (double v : A.val) sum_orig += v;
    check(std::fabs(sum_torn - sum_orig) <= 1e-12 * std::fabs(sum_orig), "split conserves entries");
    for (int kind = VTM_W_SCALED_MEAN; kind <= VTM_W_DIAG; ++kind)
        for (int side = 0; side < 2; ++side) {
            int64_t wn = 0;
            check(vtm_vertex_admittance(&a, label.data(), iface.data(), sides.data(), L, kind, 0.3, side, &wn,
                                        nullptr, nullptr, nullptr) == VTM_OK,
                  "vertex admittance size");
            std::vector<int64_t> wr(L + 1);
            std::vector<int32_t> wc(wn);
            std::vector<double> wv(wn);
            check(vtm_vertex_admittance(&a, label.data(), iface.data(), sides.data(), L, kind, 0.3, side, nullptr,
                                        wr.data(), wc.data(), wv.data()) == VTM_OK,
                  "vertex admittance fill");
            check(wr[L] == wn, "vertex admittance row pointer");
        }
    for (int depth : {0, 1, 3, -1})
        for (double drop : {0.0, 0.05}) {
            int64_t wn = 0;
            check(vtm_vertex_sca(&a, label.data(), iface.data(), sides.data(), L, 0, depth, drop, &wn, nullptr,
                                 nullptr, nullptr) == VTM_OK,
                  "SCA size");
            std::vector<int64_t> wr(L + 1);
            std::vector<int32_t> wc(wn);
            std::vector<double> wv(wn);
            check(vtm_vertex_sca(&a, label.data(), iface.data(), sides.data(), L, 0, depth, drop, nullptr, wr.data(),
                                 wc.data(), wv.data()) == VTM_OK,
                  "SCA fill");
            for (int64_t l = 0; l < L; ++l)
                for (int64_t q = wr[l]; q < wr[l + 1]; ++q)
                    if (wc[q] == l) check(wv[q] > 0.0, "SCA diagonal positive");
        }
    check(vtm_vertex_sca(&a, label.data(), iface.data(), sides.data(), L, 2, 1, 0.0, nullptr, nullptr, nullptr,
                         nullptr) == VTM_E_ARG,
          "SCA side");
    auto bad_sides = sides;
    bad_sides[1] = 0;  // both twins in one sub-circuit
    check(vtm_split_vertex(&a, label.data(), iface.data(), bad_sides.data(), L, &nt, &nnz, nullptr, nullptr, nullptr,
                           nullptr) == VTM_E_ARG,
          "sides must differ");
    auto dup = iface;
    dup[1] = dup[0];
    check(vtm_split_vertex(&a, label.data(), dup.data(), sides.data(), L, &nt, &nnz, nullptr, nullptr, nullptr,
                           nullptr) == VTM_E_ARG,
          "distinct interfacial nodes");

    // coupled lines: a dense symmetric W over the column's lines, given with its
    // rows in reverse order and every entry split in two (duplicates summed)
    std::vector<int64_t> wr(L + 1, 0);
    std::vector<int32_t> wcol;
    std::vector<double> wval;
    auto w_of = [](int64_t l, int64_t m) { return l == m ? 4.0 : 1.0 / double(1 + (l > m ? l - m : m - l)); };
    for (int64_t l = 0; l < L; ++l) {
        for (int64_t m = L - 1; m >= 0; --m)
            for (int half = 0; half < 2; ++half) {
                wcol.push_back(int32_t(m));
                wval.push_back(0.5 * w_of(l, m));
            }
        wr[l + 1] = int64_t(wcol.size());
    }
    auto plan_coupled = [&](const std::vector<double>& v, vtm::Plan& P) {
        const vtm_csr Wc{L, int64_t(wcol.size()), wr.data(), wcol.data(), v.data()};
        std::string err;
        return vtm::build_plan_vertex(&a, label.data(), iface.data(), sides.data(), L, nullptr, 0, P, err, &Wc);
    };
    vtm::Plan P;
    check(plan_coupled(wval, P) == VTM_OK && P.coupled, "coupled plan");
    check(port_nodes_first(P, nullptr), "coupled plan: port nodes (twins) numbered first in each sub-circuit");
    bool ok = int64_t(P.brow.size()) == P.nports + 1;
    for (int64_t p = 0; ok && p < P.nports; ++p) {  // B = 2 W: a full row of L entries per port
        ok = P.brow[p + 1] - P.brow[p] == L;
        for (int32_t k = P.brow[p]; ok && k < P.brow[p + 1]; ++k) ok = P.bval[k] > 0.0;
    }
    check(ok, "coupled plan: B = 2 W over the ports");
    auto asym = wval;
    asym[2] *= 1.5;  // row 0, one half of an off-diagonal entry
    check(plan_coupled(asym, P) == VTM_E_ARG, "coupled W must be symmetric");
    auto nodiag = wval;
    for (int64_t q = wr[3]; q < wr[4]; ++q)
        if (wcol[q] == 3) nodiag[q] = -2.0;
    check(plan_coupled(nodiag, P) == VTM_E_ARG, "coupled W needs a positive diagonal");
    auto nan = wval;
    nan[5] = NAN;
    check(plan_coupled(nan, P) == VTM_E_ARG, "coupled W entries finite");
}

void misc_checks() {
    vtm_options o;
    vtm_default_options(&o);
    check(o.precision == VTM_FP64 && o.check_every == 8 && o.local_form == 1, "default options");
    vtm_default_options(nullptr);
    for (int s = 0; s <= 9; ++s) check(vtm_status_str(vtm_status(s)) != nullptr, "status string");
}

// A grid large enough that the planner splits its passes over several host
// threads (1.1 M entries): the renumbered matrix must be the caller's merged and
// permuted, the recorded merge order must rebuild its values bitwise, and the
// port tables must be consistent.
void threaded_plan_checks() {
    const int ny = 300, nx = 420;
    const Csr A = grid(ny, nx, 9, true);
    const vtm_csr a = A.view();
    const auto part = blocks(ny, nx, 12, 12);
    const double Z = 1.0;
    vtm::Plan P;
    std::string err;
    check(vtm::build_plan(&a, part.data(), &Z, 1, P, err) == VTM_OK, "threaded plan: " + err);
    check(P.nwires == int64_t(34 * ny + 24 * nx), "threaded plan: cut wire count");
    check(port_nodes_first(P, part.data()), "threaded plan: port nodes numbered first in each sub-circuit");
    check(P.symmetric, "threaded plan: symmetric");
    bool ok = true;
    for (int64_t r = 0; r < P.n && ok; ++r) {
        const int32_t i = P.perm[r];
        ok = P.iperm[i] == r;
        std::map<int32_t, double> want;  // the caller's row i merged (duplicate halves sum exactly)
        for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) want[P.iperm[A.col[k]]] += A.val[k];
        ok = ok && int64_t(want.size()) == P.rowptr[r + 1] - P.rowptr[r];
        auto it = want.begin();
        for (int32_t k = P.rowptr[r]; ok && k < P.rowptr[r + 1]; ++k, ++it)
            ok = it->first == P.col[k] && it->second == P.val[k];
    }
    check(ok, "threaded plan: renumbered matrix");
    std::vector<double> rebuilt(P.val.size(), 0.0);
    for (size_t q = 0; q < P.src_ent.size(); ++q) {
        const int32_t d = P.src_dst[q];
        if (d < 0) continue;
        const double v = A.val[P.src_ent[q]];
        rebuilt[d] = (P.src_flag[q] & 1) ? v : rebuilt[d] + v;
    }
    check(std::equal(rebuilt.begin(), rebuilt.end(), P.val.begin(), P.val.end()), "threaded plan: recorded merge order");
    ok = true;
    for (int64_t q = 0; q < P.nports && ok; ++q) {
        const int32_t p = P.abi2port[q];
        ok = P.port_twin[p] == P.abi2port[q ^ 1] && P.port_twin[P.port_twin[p]] == p;
    }
    for (int64_t s = 0; s < P.S && ok; ++s)
        for (int32_t p = P.port_off[s] + 1; p < P.port_off[s + 1] && ok; ++p)
            ok = P.port_node[p - 1] < P.port_node[p] ||
                 (P.port_node[p - 1] == P.port_node[p] && P.port_slot[p] == P.port_slot[p - 1] + 1);
    check(ok, "threaded plan: port tables");
    // the transpose (split over threads) against a single pass over the rows
    std::vector<int32_t> rT, cT, rS(P.n + 1, 0), cS(P.col.size());
    std::vector<double> vT, vS(P.col.size());
    vtm::transpose_csr(P, rT, cT, vT);
    for (int32_t c : P.col) rS[c + 1]++;
    for (int64_t i = 0; i < P.n; ++i) rS[i + 1] += rS[i];
    std::vector<int32_t> fill(rS.begin(), rS.end() - 1);
    for (int64_t r = 0; r < P.n; ++r)
        for (int32_t k = P.rowptr[r]; k < P.rowptr[r + 1]; ++k) {
            const int32_t w = fill[P.col[k]]++;
            cS[w] = int32_t(r);
            vS[w] = P.val[k];
        }
    check(rT == rS && cT == cS && vT == vS, "threaded plan: transpose");
    vtm::Plan R = P;
    check(vtm::refresh_plan(R, A.val.data(), int64_t(A.val.size()), &Z, 1, err) == VTM_OK &&
              R.val == P.val && R.dmod == P.dmod && R.pbeta == P.pbeta,
          "threaded plan: refresh with the same values");
    // the refresh (its passes split over threads) against a fresh plan of new values
    const Csr A2 = grid(ny, nx, 10, true);
    const vtm_csr a2 = A2.view();
    const double Z2 = 0.7;
    vtm::Plan Q;
    check(vtm::build_plan(&a2, part.data(), &Z2, 1, Q, err) == VTM_OK, "threaded plan of new values");
    check(vtm::refresh_plan(R, A2.val.data(), int64_t(A2.val.size()), &Z2, 1, err) == VTM_OK, "threaded refresh");
    check(R.val == Q.val && R.dmod == Q.dmod && R.pc == Q.pc && R.pbeta == Q.pbeta && R.pgamma == Q.pgamma &&
              R.pg == Q.pg && R.pgd == Q.pgd && R.wg == Q.wg && R.wW == Q.wW,
          "threaded refresh equals a fresh plan");
    // with two faults the one a single pass over the recorded order meets first is
    // reported, wherever the threads' chunks fall: a merged off-diagonal entry made
    // zero (all its sources) and a non-finite value
    const int64_t nq = int64_t(P.src_ent.size());
    auto group_at = [&](int64_t q) {  // first off-diagonal merged entry starting at or after q
        while (q < nq && !((P.src_flag[q] & 1) && !(P.src_flag[q] & 2) && P.src_dst[q] >= 0)) ++q;
        int64_t e = q + 1;
        while (e < nq && !(P.src_flag[e] & 1)) ++e;
        return std::make_pair(q, e);
    };
    auto two_faults = [&](int64_t zero_from, int64_t nan_at) {
        std::vector<double> v = A2.val;
        const auto g = group_at(zero_from);
        for (int64_t q = g.first; q < g.second; ++q) v[P.src_ent[q]] = 0.0;
        const int64_t qn = nan_at < 0 ? g.second : nan_at;
        v[P.src_ent[qn]] = NAN;
        vtm::Plan T = R;
        const vtm_status st = vtm::refresh_plan(T, v.data(), int64_t(v.size()), nullptr, 0, err);
        check(T.val == R.val && T.dmod == R.dmod, "threaded refresh: a refused refresh changes nothing");
        const std::string msg = st == VTM_E_ARG ? err : std::string("status ") + std::to_string(int(st));
        // the refused refresh left partial values in the plan's spare buffer: the next
        // refresh still forms every value
        check(vtm::refresh_plan(T, A.val.data(), int64_t(A.val.size()), &Z, 1, err) == VTM_OK && T.val == P.val &&
                  T.dmod == P.dmod && T.pc == P.pc,
              "threaded refresh after a refused one equals a fresh plan");
        return msg;
    };
    const std::string pattern = "the new values change which off-diagonal entries are zero (the sparsity pattern)";
    check(two_faults(nq / 10, 9 * nq / 10) == pattern, "threaded refresh: an earlier pattern change first");
    check(two_faults(9 * nq / 10, nq / 10) == "non-finite matrix entry",
          "threaded refresh: an earlier non-finite value first");
    check(two_faults(nq / 2, -1) == "non-finite matrix entry",
          "threaded refresh: a non-finite value where the zeroed entry's successor starts comes first");
}

}  // namespace

int main() {
    plan_checks();
    threaded_plan_checks();
    refresh_checks();
    vertex_checks();
    misc_checks();
    if (g_failures) {
        std::fprintf(stderr, "%d checks failed\n", g_failures);
        return 1;
    }
    std::printf("host ABI checks passed\n");
    return 0;
}
