// Host tearing planner (Section V, Steps 1-4, in the edge-cut reading).
//
// A branch i --g-- j whose nodes lie in different sub-circuits is cut at its
// middle: i --2g-- m --2g-- j.  The middle node m is split into two twins, one
// per side, joined by a lossless line of admittance W.  Eliminating a twin from
// its sub-circuit (twin equation 2g(v - u_i) + W v = a) leaves, at node i:
//   - the cut branch g replaced by a port conductance G = 2gW / (2g + W)
//     on the diagonal (the "C + W" block of eq. 11 after elimination),
//   - the incident wave a entering the right-hand side as c * a, c = 2g/(2g+W),
//   - the outgoing wave W v - i = 2 W v - a = beta * u_i + gamma * a with
//     beta = 4gW/(2g+W), gamma = (W - 2g)/(2g+W) (eq. 11, second line).
#include "plan.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <exception>
#include <limits>
#include <map>
#include <numeric>
#include <thread>
#include <utility>

namespace vtm {

PortCoef port_coef(double g, double W) {
    const double s = 2.0 * g + W;
    return PortCoef{2.0 * g * W / s, 2.0 * g / s, 4.0 * g * W / s, (W - 2.0 * g) / s};
}

namespace {

struct Entry {
    int32_t c;
    double v;
};

// an entry of the caller's CSR while its row is merged: column, value, index
struct SrcEntry {
    int32_t c;
    double v;
    int32_t k;
};

// Host threads for a pass over `work` items: up to 16, none below 64k items each.
int plan_threads(int64_t work) {
    const int64_t hw = std::max(1u, std::thread::hardware_concurrency());
    return int(std::max<int64_t>(1, std::min<int64_t>({hw, 16, work / 65536})));
}

// f(t, lo, hi) over the T contiguous chunks [n t / T, n (t + 1) / T) of [0, n),
// chunk 0 on the calling thread; a chunk whose thread cannot start runs here.
// The first exception of a chunk (in chunk order) is rethrown after all joined.
// The same (n, T) always gives the same chunks.
template <typename F>
void for_chunks(int64_t n, int T, F&& f) {
    std::vector<std::exception_ptr> errs(T);
    auto run = [&](int t) {
        try {
            f(t, n * t / T, n * (t + 1) / T);
        } catch (...) {
            errs[t] = std::current_exception();
        }
    };
    std::vector<std::thread> th;
    th.reserve(T);
    for (int t = 1; t < T; ++t) {
        try {
            th.emplace_back(run, t);
        } catch (...) {
            run(t);
        }
    }
    run(0);
    for (auto& x : th) x.join();
    for (auto& e : errs)
        if (e) std::rethrow_exception(e);
}

}  // namespace

vtm_status build_plan(const vtm_csr* A, const int32_t* part, const double* Z, int64_t nZ,
                      Plan& P, std::string& err, const int32_t* line_a, const int32_t* line_b, int64_t n_lines) {
    const bool explicit_lines = line_a != nullptr;
    if (!A || !part || !Z || !A->rowptr || (!A->col && A->nnz) || (!A->val && A->nnz)) {
        err = "null argument";
        return VTM_E_ARG;
    }
    const int64_t n = A->n, nnz = A->nnz;
    if (n <= 0 || nnz < 0) {
        err = "n must be positive and nnz non-negative";
        return VTM_E_ARG;
    }
    if (n > std::numeric_limits<int32_t>::max() || nnz > std::numeric_limits<int32_t>::max()) {
        err = "n and nnz must fit int32";
        return VTM_E_UNSUPPORTED;
    }
    if (A->rowptr[0] != 0 || A->rowptr[n] != nnz) {
        err = "rowptr must start at 0 and end at nnz";
        return VTM_E_ARG;
    }
    for (int64_t i = 0; i < n; ++i)
        if (A->rowptr[i + 1] < A->rowptr[i]) {
            err = "rowptr must be non-decreasing";
            return VTM_E_ARG;
        }
    {
        // entries checked on threads; the first bad entry in order decides the message
        const int TV = plan_threads(nnz);
        std::vector<int64_t> first_bad(TV, INT64_MAX);
        for_chunks(nnz, TV, [&](int t, int64_t k0, int64_t k1) {
            for (int64_t k = k0; k < k1; ++k)
                if (A->col[k] < 0 || A->col[k] >= n || !std::isfinite(A->val[k])) {
                    first_bad[t] = k;
                    return;
                }
        });
        const int64_t k = *std::min_element(first_bad.begin(), first_bad.end());
        if (k != INT64_MAX) {
            err = (A->col[k] < 0 || A->col[k] >= n) ? "column index out of range" : "non-finite matrix entry";
            return VTM_E_ARG;
        }
    }

    // ---- labels -------------------------------------------------------------
    int64_t S = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (part[i] < 0) {
            err = "negative sub-circuit label";
            return VTM_E_ARG;
        }
        S = std::max<int64_t>(S, int64_t(part[i]) + 1);
    }
    std::vector<int32_t> count(S, 0);
    for (int64_t i = 0; i < n; ++i) count[part[i]]++;
    for (int64_t s = 0; s < S; ++s)
        if (count[s] == 0) {
            err = "sub-circuit label " + std::to_string(s) + " is unused";
            return VTM_E_ARG;
        }
    P.n = n;
    P.S = S;
    P.sub_off.assign(S + 1, 0);
    for (int64_t s = 0; s < S; ++s) P.sub_off[s + 1] = P.sub_off[s] + count[s];
    P.max_ns = *std::max_element(count.begin(), count.end());
    if (P.max_ns > kMaxSubCircuit) {
        err = "a sub-circuit has more than " + std::to_string(kMaxSubCircuit) + " nodes";
        return VTM_E_UNSUPPORTED;
    }
    // inverse blocks start 16-byte aligned (multiples of 4 elements), as the sweep's loads need
    P.kofs.assign(S + 1, 0);
    for (int64_t s = 0; s < S; ++s) P.kofs[s + 1] = P.kofs[s] + ((int64_t(count[s]) * count[s] + 3) & ~int64_t(3));
    // MFMA tile blocks: each sub-circuit padded to a multiple of 32 rows and columns
    P.mofs.assign(S + 1, 0);
    for (int64_t s = 0; s < S; ++s) {
        const int64_t np = (int64_t(count[s]) + 31) & ~int64_t(31);
        P.mofs[s + 1] = P.mofs[s] + np * np;
    }

    // ---- rows with merged duplicates and sorted columns (old numbering) -------
    // The order in which the caller's entries are summed is recorded (src_*) so
    // that vtm_refresh can merge new values the same way without sorting again.
    scratch_vec<int64_t> mrow(n + 1);  // every entry written below
    mrow[0] = 0;
    scratch_vec<Entry> ment;
    const bool record = !explicit_lines;
    scratch_vec<int32_t> src_merged;  // per summed position: merged entry (before renumbering), -1 if dropped
    if (record) {
        P.src_ent.resize(nnz);
        P.src_flag.resize(nnz);
        src_merged.resize(nnz);
    }
    // rows are merged on host threads in two passes: the merged length of every row,
    // then, with the row offsets known, the merged entries written in place
    const int TR = plan_threads(nnz);
    {
        // row i merged into tmp (columns sorted, duplicates summed, zeros off the
        // diagonal dropped); with record, the summation order goes to src_ent and
        // src_flag and each position's entry index within tmp (-1: dropped) to pos_of
        auto merge_row = [&](int64_t i, std::vector<SrcEntry>& row, std::vector<Entry>& tmp,
                             std::vector<int32_t>& run_of, int32_t* pos_of) {
            row.clear();
            bool sorted = true;
            for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
                if (!row.empty() && A->col[k] <= row.back().c) sorted = false;
                row.push_back({A->col[k], A->val[k], int32_t(k)});
            }
            if (!sorted)
                std::sort(row.begin(), row.end(), [](const SrcEntry& a, const SrcEntry& b) { return a.c < b.c; });
            tmp.clear();
            int64_t pos = A->rowptr[i];
            for (const SrcEntry& e : row) {
                const bool first = !(!tmp.empty() && tmp.back().c == e.c);
                if (!first)
                    tmp.back().v += e.v;
                else
                    tmp.push_back({e.c, e.v});
                if (pos_of) {
                    P.src_ent[pos] = e.k;
                    P.src_flag[pos] = uint8_t((first ? 1 : 0) | (e.c == i ? 2 : 0));
                    pos_of[pos - A->rowptr[i]] = int32_t(tmp.size() - 1);  // run index for now
                }
                ++pos;
            }
            // explicit zeros off the diagonal couple nothing
            size_t w = 0;
            run_of.assign(tmp.size(), -1);
            for (size_t k = 0; k < tmp.size(); ++k)
                if (tmp[k].v != 0.0 || tmp[k].c == i) {
                    run_of[k] = int32_t(w);
                    tmp[w++] = tmp[k];
                }
            tmp.resize(w);
            if (pos_of)
                for (int64_t q = 0; q < pos - A->rowptr[i]; ++q) pos_of[q] = run_of[pos_of[q]];
        };
        for_chunks(n, TR, [&](int, int64_t i0, int64_t i1) {
            std::vector<SrcEntry> row;
            std::vector<Entry> tmp;
            std::vector<int32_t> run_of;
            for (int64_t i = i0; i < i1; ++i) {
                // a row with strictly increasing columns has no duplicates to sum
                bool inc = true;
                int64_t cnt = 0;
                for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
                    if (k > A->rowptr[i] && A->col[k] <= A->col[k - 1]) inc = false;
                    if (A->val[k] != 0.0 || A->col[k] == i) ++cnt;
                }
                if (!inc) {
                    merge_row(i, row, tmp, run_of, nullptr);
                    cnt = int64_t(tmp.size());
                }
                mrow[i + 1] = cnt;
            }
        });
        for (int64_t i = 0; i < n; ++i) mrow[i + 1] += mrow[i];
        ment.resize(size_t(mrow[n]));
        for_chunks(n, TR, [&](int, int64_t i0, int64_t i1) {
            std::vector<SrcEntry> row;
            std::vector<Entry> tmp;
            std::vector<int32_t> run_of;
            for (int64_t i = i0; i < i1; ++i) {
                int32_t* pos_of = record ? src_merged.data() + A->rowptr[i] : nullptr;
                merge_row(i, row, tmp, run_of, pos_of);
                std::copy(tmp.begin(), tmp.end(), ment.begin() + mrow[i]);
                if (record)
                    for (int64_t q = 0; q < A->rowptr[i + 1] - A->rowptr[i]; ++q)
                        if (pos_of[q] >= 0) pos_of[q] += int32_t(mrow[i]);
            }
        });
    }

    // ---- exact symmetry (lets the adjoint share the forward path) -------------
    auto find = [&](int64_t r, int32_t c, double& v) -> bool {
        auto lo = ment.begin() + mrow[r], hi = ment.begin() + mrow[r + 1];
        auto it = std::lower_bound(lo, hi, c, [](const Entry& e, int32_t cc) { return e.c < cc; });
        if (it == hi || it->c != c) return false;
        v = it->v;
        return true;
    };
    {
        std::atomic<bool> sym{true};
        for_chunks(n, TR, [&](int, int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1 && sym.load(std::memory_order_relaxed); ++i)
                for (int64_t k = mrow[i]; k < mrow[i + 1]; ++k) {
                    double v;
                    if (!find(ment[k].c, int32_t(i), v) || v != ment[k].v) {
                        sym.store(false, std::memory_order_relaxed);
                        break;
                    }
                }
        });
        P.symmetric = sym.load();
    }

    // ---- cut wires (canonical order falls out of the row scan) ----------------
    P.wi.clear();
    P.wj.clear();
    P.wg.clear();
    {
        // per chunk of rows: its wires in row order, or its first error
        struct Cut {
            std::vector<int32_t> wi, wj;
            std::vector<double> wg;
            vtm_status st = VTM_OK;
            std::string err;
        };
        std::vector<Cut> cuts(TR);
        for_chunks(n, TR, [&](int t, int64_t i0, int64_t i1) {
            Cut& C = cuts[t];
            for (int64_t i = i0; i < i1 && C.st == VTM_OK; ++i)
                for (int64_t k = mrow[i]; k < mrow[i + 1]; ++k) {
                    const int32_t j = ment[k].c;
                    if (part[i] == part[j]) continue;
                    auto pair = [&] { return "nodes " + std::to_string(i) + " and " + std::to_string(j); };
                    if (explicit_lines) {
                        C.err = pair() + " in different sub-circuits are coupled directly, not through an interfacial node";
                        C.st = VTM_E_UNTEARABLE;
                        break;
                    }
                    double vt;
                    if (!find(j, int32_t(i), vt) || vt != ment[k].v) {
                        C.err = "coupling between " + pair() + " in different sub-circuits is not symmetric";
                        C.st = VTM_E_UNTEARABLE;
                        break;
                    }
                    if (!(ment[k].v < 0.0)) {
                        C.err = "coupling between " + pair() + " in different sub-circuits is not a positive conductance";
                        C.st = VTM_E_UNTEARABLE;
                        break;
                    }
                    if (j > i) {
                        C.wi.push_back(int32_t(i));
                        C.wj.push_back(j);
                        C.wg.push_back(-ment[k].v);
                    }
                }
        });
        for (Cut& C : cuts) {
            if (C.st != VTM_OK) {
                err = C.err;
                return C.st;
            }
            P.wi.insert(P.wi.end(), C.wi.begin(), C.wi.end());
            P.wj.insert(P.wj.end(), C.wj.begin(), C.wj.end());
            P.wg.insert(P.wg.end(), C.wg.begin(), C.wg.end());
        }
    }
    if (explicit_lines) {
        if (!line_b || n_lines < 0) {
            err = "bad line list";
            return VTM_E_ARG;
        }
        for (int64_t e = 0; e < n_lines; ++e) {
            const int32_t a = line_a[e], b = line_b[e];
            if (a < 0 || a >= n || b < 0 || b >= n || part[a] == part[b]) {
                err = "a line must join two nodes of different sub-circuits";
                return VTM_E_ARG;
            }
            P.wi.push_back(a);
            P.wj.push_back(b);
            P.wg.push_back(0.0);
        }
        P.vertex = true;
    }
    const int64_t nw = int64_t(P.wi.size());
    P.nwires = nw;
    P.nports = 2 * nw;
    if (nZ != 1 && nZ != nw) {
        err = "nZ must be 1 or the number of cut wires (" + std::to_string(nw) + ")";
        return VTM_E_ARG;
    }
    P.wW.resize(nw);
    for (int64_t e = 0; e < nw; ++e) {
        const double z = Z[nZ == 1 ? 0 : e];
        if (!(z > 0.0) || !std::isfinite(z)) {
            err = "line impedance must be positive and finite";
            return VTM_E_ARG;
        }
        P.wW[e] = 1.0 / z;
    }

    // ---- renumbering: sub-circuit by sub-circuit, each one's port nodes (the ends of
    // its lines) first, then its other nodes, ascending node id in each group; the
    // rows a sweep needs for the waves alone are then a sub-circuit's first rows
    P.perm.resize(n);
    P.iperm.resize(n);
    {
        std::vector<uint8_t> is_port(n, 0);
        for (int64_t e = 0; e < nw; ++e) is_port[P.wi[e]] = is_port[P.wj[e]] = 1;
        std::vector<int32_t> fill_p(P.sub_off.begin(), P.sub_off.end() - 1), fill_o(S);
        for (int64_t i = 0; i < n; ++i)
            if (is_port[i]) fill_o[part[i]]++;
        for (int64_t s = 0; s < S; ++s) fill_o[s] += P.sub_off[s];
        for (int64_t i = 0; i < n; ++i) {
            const int32_t r = is_port[i] ? fill_p[part[i]]++ : fill_o[part[i]]++;
            P.perm[r] = int32_t(i);
            P.iperm[i] = r;
        }
    }

    // ---- ports -----------------------------------------------------------------
    // key per ABI port q (2e lower node, 2e+1 upper): (sub, local node, wire)
    const int64_t np = P.nports;
    const int TP = plan_threads(np);
    std::vector<int32_t> q_sub(np), q_loc(np);
    for_chunks(nw, TP, [&](int, int64_t e0, int64_t e1) {
        for (int64_t e = e0; e < e1; ++e)
            for (int side = 0; side < 2; ++side) {
                const int32_t node = side ? P.wj[e] : P.wi[e];
                const int64_t q = 2 * e + side;
                q_sub[q] = part[node];
                q_loc[q] = P.iperm[node] - P.sub_off[part[node]];
            }
    });
    // ports in (sub-circuit, local node, ABI port) order: a counting sort by
    // sub-circuit (ABI order inside each), then each sub-circuit's run sorted by
    // local node, stably; beg[s] is the first port of sub-circuit s
    std::vector<int64_t> order(np), beg(S + 1, 0);
    {
        for (int64_t q = 0; q < np; ++q) beg[q_sub[q] + 1]++;
        for (int64_t s = 0; s < S; ++s) beg[s + 1] += beg[s];
        std::vector<int64_t> fill(beg.begin(), beg.end() - 1);
        for (int64_t q = 0; q < np; ++q) order[fill[q_sub[q]]++] = q;
        for_chunks(S, TP, [&](int, int64_t s0, int64_t s1) {
            for (int64_t s = s0; s < s1; ++s)
                std::stable_sort(order.begin() + beg[s], order.begin() + beg[s + 1],
                                 [&](int64_t a, int64_t b) { return q_loc[a] < q_loc[b]; });
        });
    }
    P.port_off.assign(S + 1, 0);
    for (int64_t s = 0; s < S; ++s) P.port_off[s + 1] = int32_t(beg[s + 1] - beg[s]);  // counts for now
    P.port_node.resize(np);
    P.port_slot.resize(np);
    P.port_twin.resize(np);
    P.abi2port.resize(np);
    P.pc.resize(np);
    P.pbeta.resize(np);
    P.pgamma.resize(np);
    P.pg.resize(np);
    P.pgd.resize(np);
    P.dmod.assign(n, 0.0);
    P.max_slot = 0;
    for_chunks(np, TP, [&](int, int64_t p0, int64_t p1) {
        for (int64_t p = p0; p < p1; ++p) {
            const int64_t q = order[p];
            P.abi2port[q] = int32_t(p);
            P.port_node[p] = q_loc[q];
            const int64_t e = q / 2;
            // a line between twins has no branch: its port adds W to the twin's row, the
            // wave enters whole (c = 1) and leaves as 2 W u - a (beta = 2 W, gamma = -1),
            // the limit of a cut branch whose g grows without bound
            const PortCoef k = P.vertex ? PortCoef{P.coupled ? 0.0 : P.wW[e], 1.0, 2.0 * P.wW[e], -1.0}
                                        : port_coef(P.wg[e], P.wW[e]);
            P.pc[p] = k.c;
            P.pbeta[p] = k.beta;
            P.pgamma[p] = k.gamma;
            P.pg[p] = P.wg[e];
            P.pgd[p] = k.G - P.wg[e];
        }
    });
    // in port order: the slots, and the diagonal changes summed as ports come; a
    // node's ports are its sub-circuit's, so sub-circuits split over threads keep
    // every node's order
    std::vector<int32_t> tmax(TP, 0);
    for_chunks(S, TP, [&](int t, int64_t s0, int64_t s1) {
        int32_t mx = 0;
        for (int64_t p = beg[s0]; p < beg[s1]; ++p) {
            const int64_t q = order[p];
            P.port_slot[p] = (p > beg[s0] && q_sub[order[p - 1]] == q_sub[q] && q_loc[order[p - 1]] == q_loc[q])
                                 ? P.port_slot[p - 1] + 1
                                 : 0;
            mx = std::max(mx, P.port_slot[p]);
            const int32_t node = (q & 1) ? P.wj[q / 2] : P.wi[q / 2];
            P.dmod[P.iperm[node]] += P.pgd[p];
        }
        tmax[t] = mx;
    });
    for (int32_t v : tmax) P.max_slot = std::max(P.max_slot, v);
    P.pofs.assign(S + 1, 0);
    P.qmofs.assign(S + 1, 0);
    for (int64_t s = 0; s < S; ++s) {
        const int64_t q = P.port_off[s + 1];
        P.max_ports = std::max<int32_t>(P.max_ports, int32_t(q));
        P.pofs[s + 1] = P.pofs[s] + ((q * q + 3) & ~int64_t(3));
        P.sq_entries += q * q;
        const int64_t qp = (q + 31) & ~int64_t(31);
        P.qmofs[s + 1] = P.qmofs[s] + qp * qp;
        P.port_off[s + 1] += P.port_off[s];
    }
    for_chunks(np, TP, [&](int, int64_t q0, int64_t q1) {
        for (int64_t q = q0; q < q1; ++q) P.port_twin[P.abi2port[q]] = P.abi2port[q ^ 1];
    });
    for (int64_t e = 1; e < nw; ++e)
        if (P.wW[e] != P.wW[0]) P.uniform_W = false;

    // port nodes (runs of equal local node inside each sub-circuit's port range)
    P.pn_off.assign(S + 1, 0);
    P.pn_node.clear();
    P.pn_pfirst.clear();
    P.sofs.assign(S + 1, 0);
    P.nofs.assign(S + 1, 0);
    P.max_npn = 0;
    for (int64_t s = 0; s < S; ++s) {
        for (int32_t p = P.port_off[s]; p < P.port_off[s + 1]; ++p)
            if (p == P.port_off[s] || P.port_node[p] != P.port_node[p - 1]) {
                P.pn_node.push_back(P.port_node[p]);
                P.pn_pfirst.push_back(p);
            }
        P.pn_off[s + 1] = int32_t(P.pn_node.size());
        const int64_t k = P.pn_off[s + 1] - P.pn_off[s];
        P.max_npn = std::max<int32_t>(P.max_npn, int32_t(k));
        // upper triangle stored as pairs of diagonals, row-interleaved (the last row of a
        // pair pads its second entry): k (k + 2) / 2 entries for even k, (k + 1)^2 / 2 for odd
        const int64_t pairs = (k % 2 == 0) ? k * (k + 2) / 2 : (k + 1) * (k + 1) / 2;
        P.tri_entries += k * (k + 1) / 2;
        P.sqn_entries += k * k;
        P.nofs[s + 1] = P.nofs[s] + ((k * k + 3) & ~int64_t(3));
        P.sofs[s + 1] = P.sofs[s] + ((pairs + 3) & ~int64_t(3));
    }
    P.pn_pfirst.push_back(int32_t(np));

    // ---- renumbered untorn matrix ------------------------------------------------
    P.rowptr.assign(n + 1, 0);
    P.col.resize(ment.size());
    P.val.resize(ment.size());
    scratch_vec<int32_t> m2r(record ? ment.size() : 0);  // merged entry -> renumbered entry (each written once)
    for (int64_t r = 0; r < n; ++r) {
        const int32_t i = P.perm[r];
        P.rowptr[r + 1] = P.rowptr[r] + int32_t(mrow[i + 1] - mrow[i]);
    }
    for_chunks(n, TR, [&](int, int64_t r0, int64_t r1) {
        std::vector<SrcEntry> row;  // k: the merged entry
        for (int64_t r = r0; r < r1; ++r) {
            const int32_t i = P.perm[r];
            row.clear();
            for (int64_t k = mrow[i]; k < mrow[i + 1]; ++k)
                row.push_back({P.iperm[ment[k].c], ment[k].v, int32_t(k)});
            std::sort(row.begin(), row.end(), [](const SrcEntry& a, const SrcEntry& b) { return a.c < b.c; });
            int64_t w = P.rowptr[r];
            for (const SrcEntry& e : row) {
                P.col[w] = e.c;
                P.val[w] = e.v;
                if (record) m2r[e.k] = int32_t(w);
                ++w;
            }
        }
    });
    if (record) {
        P.src_dst.resize(nnz);
        for_chunks(nnz, TR, [&](int, int64_t q0, int64_t q1) {
            for (int64_t q = q0; q < q1; ++q) P.src_dst[q] = src_merged[q] < 0 ? -1 : m2r[src_merged[q]];
        });
        // transpose and wire positions, so that a refresh compares values without searching
        auto at = [&](int32_t r, int32_t c) -> int32_t {
            auto lo = P.col.begin() + P.rowptr[r], hi = P.col.begin() + P.rowptr[r + 1];
            auto it = std::lower_bound(lo, hi, c);
            return (it == hi || *it != c) ? -1 : int32_t(it - P.col.begin());
        };
        P.tpos.resize(P.col.size());
        for_chunks(n, TR, [&](int, int64_t r0, int64_t r1) {
            for (int64_t r = r0; r < r1; ++r)
                for (int32_t k = P.rowptr[r]; k < P.rowptr[r + 1]; ++k) P.tpos[k] = at(P.col[k], int32_t(r));
        });
        P.wpos.resize(2 * nw);
        for_chunks(nw, TP, [&](int, int64_t e0, int64_t e1) {
            for (int64_t e = e0; e < e1; ++e) {
                const int32_t r = P.iperm[P.wi[e]], c = P.iperm[P.wj[e]];
                P.wpos[2 * e] = at(r, c);
                P.wpos[2 * e + 1] = at(c, r);
            }
        });
    }
    return VTM_OK;
}

// New values of the caller's A on the pattern the plan was built from, merged
// in the recorded order (so bitwise as build_plan merges them), then the cut
// wires' conductances, the port coefficients and the diagonal changes as
// build_plan forms them.  The plan is changed only when every check passes.
vtm_status refresh_plan(Plan& P, const double* val, int64_t nnz, const double* Z, int64_t nZ, std::string& err) {
    if (P.vertex || int64_t(P.src_ent.size()) != nnz) {
        err = P.vertex ? "refresh applies to handles torn along a node partition (vtm_setup)"
                       : "nnz differs from the A the handle was set up with";
        return P.vertex ? VTM_E_UNSUPPORTED : VTM_E_ARG;
    }
    if (nnz > 0 && !val) {
        err = "null values";
        return VTM_E_ARG;
    }
    // The merge runs on threads, each over whole merged entries: chunk t starts at
    // the first merged entry that begins at or after nnz t / T.  A chunk stops at
    // its first failure; the failure a single pass would meet first wins, keyed by
    // the source position (a non-finite value at q before the pattern check of the
    // merged entry that ends just before q).  Every entry of nv is written when no
    // chunk fails.  It is the plan's spare value buffer, left uninitialised the
    // first time so that its pages are first touched by the threads rather than
    // zeroed on one, and swapped with the values once every check has passed.
    const int64_t m = int64_t(P.val.size());
    if (int64_t(P.val_spare.size()) != m) P.val_spare.resize(size_t(m));
    double* const nv = P.val_spare.data();
    const int T = plan_threads(nnz);
    std::vector<int64_t> lo(T + 1, nnz), fkey(T, INT64_MAX);
    lo[0] = 0;
    for (int t = 1; t < T; ++t) {
        int64_t q = nnz * t / T;
        while (q < nnz && !(P.src_flag[q] & 1)) ++q;
        lo[t] = q;
    }
    for (int t = T - 1; t >= 1; --t) lo[t] = std::min(lo[t], lo[t + 1]);
    for_chunks(T, T, [&](int t, int64_t, int64_t) {
        double cur = 0.0;
        int32_t dst = -1;
        bool diag = false;
        auto close = [&]() -> bool {  // false: the merged entry changes the pattern
            if (dst >= 0) {
                if (cur == 0.0 && !diag) return false;
                nv[dst] = cur;
            } else if (cur != 0.0) {
                return false;
            }
            return true;
        };
        const int64_t q0 = lo[t], q1 = lo[t + 1];
        for (int64_t q = q0; q < q1; ++q) {
            const double v = val[P.src_ent[q]];
            if (!std::isfinite(v)) {
                fkey[t] = 2 * q;
                return;
            }
            if (P.src_flag[q] & 1) {
                if (q > q0 && !close()) {
                    fkey[t] = 2 * q + 1;
                    return;
                }
                cur = v;
                dst = P.src_dst[q];
                diag = (P.src_flag[q] & 2) != 0;
            } else {
                cur += v;
            }
        }
        if (q1 > q0 && !close()) fkey[t] = 2 * q1 + 1;
    });
    const int64_t first = *std::min_element(fkey.begin(), fkey.end());
    if (first != INT64_MAX) {
        err = (first & 1) ? "the new values change which off-diagonal entries are zero (the sparsity pattern)"
                          : "non-finite matrix entry";
        return VTM_E_ARG;
    }
    // symmetric: every entry has its transpose in the pattern, of equal value
    std::vector<uint8_t> asym(T, 0);
    for_chunks(m, T, [&](int t, int64_t k0, int64_t k1) {
        for (int64_t k = k0; k < k1; ++k) {
            const int32_t u = P.tpos[k];
            if (u < 0 || nv[u] != nv[k]) {
                asym[t] = 1;
                return;
            }
        }
    });
    const bool sym = std::find(asym.begin(), asym.end(), 1) == asym.end();
    if (sym != P.symmetric) {
        err = "the new values change whether A is symmetric (the handle's local forms depend on it)";
        return VTM_E_UNSUPPORTED;
    }
    const int64_t nw = P.nwires;
    const int TW = plan_threads(nw);
    std::vector<double> wg(nw), wW = P.wW;
    std::vector<int64_t> bad(TW, INT64_MAX);  // each chunk's first wire that is no conductance
    for_chunks(nw, TW, [&](int t, int64_t e0, int64_t e1) {
        for (int64_t e = e0; e < e1; ++e) {
            const double v = nv[P.wpos[2 * e]], vt = nv[P.wpos[2 * e + 1]];
            if (v != vt || !(v < 0.0)) {
                bad[t] = e;
                return;
            }
            wg[e] = -v;
        }
    });
    if (const int64_t e = *std::min_element(bad.begin(), bad.end()); e != INT64_MAX) {
        err = "coupling between nodes " + std::to_string(P.wi[e]) + " and " + std::to_string(P.wj[e]) +
              " in different sub-circuits is not a symmetric positive conductance";
        return VTM_E_UNTEARABLE;
    }
    if (Z && nZ > 0) {
        if (nZ != 1 && nZ != nw) {
            err = "nZ must be 0, 1 or the number of cut wires (" + std::to_string(nw) + ")";
            return VTM_E_ARG;
        }
        for (int64_t e = 0; e < nw; ++e) {
            const double z = Z[nZ == 1 ? 0 : e];
            if (!(z > 0.0) || !std::isfinite(z)) {
                err = "line impedance must be positive and finite";
                return VTM_E_ARG;
            }
            wW[e] = 1.0 / z;
        }
    }
    // commit, then the port quantities as build_plan forms them (the diagonal
    // changes summed in port order, one pass)
    P.val.swap(P.val_spare);
    P.wg.swap(wg);
    P.wW.swap(wW);
    const int64_t np = P.nports;
    const int TP = plan_threads(np);
    std::vector<int32_t> port2abi(np);
    for_chunks(np, TP, [&](int, int64_t q0, int64_t q1) {
        for (int64_t q = q0; q < q1; ++q) port2abi[P.abi2port[q]] = int32_t(q);
    });
    for_chunks(np, TP, [&](int, int64_t p0, int64_t p1) {
        for (int64_t p = p0; p < p1; ++p) {
            const int64_t e = port2abi[p] / 2;
            const PortCoef k = port_coef(P.wg[e], P.wW[e]);
            P.pc[p] = k.c;
            P.pbeta[p] = k.beta;
            P.pgamma[p] = k.gamma;
            P.pg[p] = P.wg[e];
            P.pgd[p] = k.G - P.wg[e];
        }
    });
    // a node's ports are those of its sub-circuit, consecutive in port order: the
    // sub-circuits split over threads sum each node's changes in that order
    for_chunks(P.n, plan_threads(P.n), [&](int, int64_t r0, int64_t r1) {
        std::fill(P.dmod.begin() + r0, P.dmod.begin() + r1, 0.0);
    });
    for_chunks(P.S, TP, [&](int, int64_t s0, int64_t s1) {
        for (int64_t p = P.port_off[s0]; p < P.port_off[s1]; ++p) {
            const int64_t q = port2abi[p];
            const int32_t node = (q & 1) ? P.wj[q / 2] : P.wi[q / 2];
            P.dmod[P.iperm[node]] += P.pgd[p];
        }
    });
    P.uniform_W = true;
    for (int64_t e = 1; e < nw; ++e)
        if (P.wW[e] != P.wW[0]) P.uniform_W = false;
    return VTM_OK;
}

// ---- tearing at interfacial nodes ---------------------------------------------
// Step 1 names the interfacial nodes, Steps 2-3 split each into two twins and
// distribute what touches it, Step 4 joins the twins by a line.  The split
// (reading of Step 3 and of the op-amp example, eqs. 15-17): an entry between
// an interfacial node v and a non-interfacial node w stays whole and moves to
// the twin of v on w's side; a two-terminal branch (A_vw == A_wv < 0) also
// moves its conductance to that twin's diagonal; what remains of A_vv (the
// ground conductance and the branches between interfacial nodes), the entries
// between two interfacial nodes (split between the twins of each side) and the
// source at v are shared in equal halves.  Twin a of line l keeps v's number,
// twin b is node n + l of the expanded system.
vtm_status split_at_vertices(const vtm_csr* A, const int32_t* label, const int32_t* iface, const int32_t* sides,
                             int64_t L, VertexSplit& out, std::string& err) {
    if (!A || !label || !A->rowptr || (!A->col && A->nnz) || (!A->val && A->nnz) || L < 0 ||
        (L > 0 && (!iface || !sides))) {
        err = "null argument";
        return VTM_E_ARG;
    }
    const int64_t n = A->n;
    if (n <= 0 || A->nnz < 0 || A->rowptr[0] != 0 || A->rowptr[n] != A->nnz) {
        err = "malformed CSR";
        return VTM_E_ARG;
    }
    for (int64_t i = 0; i < n; ++i)
        if (A->rowptr[i + 1] < A->rowptr[i]) {
            err = "rowptr must be non-decreasing";
            return VTM_E_ARG;
        }
    if (n + L > std::numeric_limits<int32_t>::max()) {
        err = "n plus the interfacial nodes must fit int32";
        return VTM_E_UNSUPPORTED;
    }
    std::vector<int64_t> line_of(n, -1);
    for (int64_t l = 0; l < L; ++l) {
        const int32_t v = iface[l];
        if (v < 0 || v >= n || line_of[v] >= 0) {
            err = "interfacial nodes must be distinct node ids";
            return VTM_E_ARG;
        }
        if (sides[2 * l] < 0 || sides[2 * l + 1] < 0 || sides[2 * l] == sides[2 * l + 1]) {
            err = "each interfacial node needs two distinct sub-circuits";
            return VTM_E_ARG;
        }
        line_of[v] = l;
    }
    for (int64_t i = 0; i < n; ++i)
        if (line_of[i] < 0 && label[i] < 0) {
            err = "negative sub-circuit label";
            return VTM_E_ARG;
        }
    for (int64_t k = 0; k < A->nnz; ++k)
        if (A->col[k] < 0 || A->col[k] >= n || !std::isfinite(A->val[k])) {
            err = "column index out of range or non-finite entry";
            return VTM_E_ARG;
        }
    // the caller's A with duplicates merged and columns sorted: the split reads it,
    // and the residual of the untorn system uses it
    std::vector<int32_t> orow(n + 1, 0), ocol;
    std::vector<double> oval;
    {
        std::vector<std::pair<int32_t, double>> row;
        for (int64_t i = 0; i < n; ++i) {
            row.clear();
            for (int64_t q = A->rowptr[i]; q < A->rowptr[i + 1]; ++q) row.push_back({A->col[q], A->val[q]});
            std::sort(row.begin(), row.end());
            for (size_t k = 0; k < row.size(); ++k) {
                if (k > 0 && row[k].first == row[k - 1].first) {
                    oval.back() += row[k].second;
                } else {
                    ocol.push_back(row[k].first);
                    oval.push_back(row[k].second);
                }
            }
            orow[i + 1] = int32_t(ocol.size());
        }
    }
    auto entry = [&](int64_t r, int64_t c, double& v) -> bool {  // A[r, c]
        auto lo = ocol.begin() + orow[r], hi = ocol.begin() + orow[r + 1];
        auto it = std::lower_bound(lo, hi, int32_t(c));
        if (it == hi || *it != c) return false;
        v = oval[it - ocol.begin()];
        return true;
    };
    // the twin of interfacial node v (line l) in sub-circuit s, or -1
    auto twin_in = [&](int64_t l, int32_t s) -> int64_t {
        if (sides[2 * l] == s) return iface[l];
        if (sides[2 * l + 1] == s) return n + l;
        return -1;
    };
    const int64_t N = n + L;
    std::vector<std::vector<std::pair<int32_t, double>>> rows(N);
    std::vector<double> remainder(L, 0.0);  // what of A_vv is split in halves
    for (int64_t i = 0; i < n; ++i) {
        const int64_t li = line_of[i];
        for (int64_t q = orow[i]; q < orow[i + 1]; ++q) {
            const int64_t j = ocol[q];
            const int64_t lj = line_of[j];
            const double v = oval[q];
            if (v == 0.0 && i != j) continue;
            if (li < 0 && lj < 0) {
                if (label[i] != label[j]) {
                    err = "nodes " + std::to_string(i) + " and " + std::to_string(j) +
                          " of different sub-circuits are coupled directly, not through an interfacial node";
                    return VTM_E_UNTEARABLE;
                }
                rows[i].push_back({int32_t(j), v});
            } else if (li < 0) {  // row i inner, column j interfacial
                const int64_t t = twin_in(lj, label[i]);
                if (t < 0) {
                    err = "node " + std::to_string(i) + " is coupled to interfacial node " + std::to_string(j) +
                          " of sub-circuits it does not belong to";
                    return VTM_E_UNTEARABLE;
                }
                rows[i].push_back({int32_t(t), v});
            } else if (lj < 0) {  // row i interfacial, column j inner
                const int64_t t = twin_in(li, label[j]);
                if (t < 0) {
                    err = "interfacial node " + std::to_string(i) + " is coupled to node " + std::to_string(j) +
                          " of a sub-circuit it does not border";
                    return VTM_E_UNTEARABLE;
                }
                rows[t].push_back({int32_t(j), v});
                double vt;
                if (v < 0.0 && entry(j, i, vt) && vt == v) rows[t].push_back({int32_t(t), -v});  // branch g
            } else if (i == j) {
                remainder[li] += v;
            } else {  // two interfacial nodes: the same two sub-circuits, half on each side
                const int32_t s0 = sides[2 * li], s1 = sides[2 * li + 1];
                const int64_t a0 = twin_in(lj, s0), a1 = twin_in(lj, s1);
                if (a0 < 0 || a1 < 0) {
                    err = "interfacial nodes " + std::to_string(i) + " and " + std::to_string(j) +
                          " border different sub-circuits";
                    return VTM_E_UNTEARABLE;
                }
                rows[iface[li]].push_back({int32_t(a0), 0.5 * v});
                rows[n + li].push_back({int32_t(a1), 0.5 * v});
            }
        }
    }
    // the interfacial node's diagonal less the branch conductances moved to its twins
    for (int64_t l = 0; l < L; ++l) {
        const int64_t v = iface[l];
        double moved = 0.0;
        for (int64_t q = orow[v]; q < orow[v + 1]; ++q) {
            const int64_t j = ocol[q];
            double vt;
            if (line_of[j] < 0 && oval[q] < 0.0 && entry(j, v, vt) && vt == oval[q]) moved += -oval[q];
        }
        const double half = 0.5 * (remainder[l] - moved);
        rows[v].push_back({int32_t(v), half});
        rows[n + l].push_back({int32_t(n + l), half});
    }
    // expanded CSR and partition
    out.n = n;
    out.L = L;
    out.rowptr.assign(N + 1, 0);
    out.col.clear();
    out.val.clear();
    for (int64_t r = 0; r < N; ++r) {
        for (const auto& e : rows[r]) {
            out.col.push_back(e.first);
            out.val.push_back(e.second);
        }
        out.rowptr[r + 1] = int64_t(out.col.size());
    }
    out.part.resize(N);
    for (int64_t i = 0; i < n; ++i) out.part[i] = line_of[i] < 0 ? label[i] : sides[2 * line_of[i]];
    for (int64_t l = 0; l < L; ++l) out.part[n + l] = sides[2 * l + 1];
    out.orow = std::move(orow);
    out.ocol = std::move(ocol);
    out.oval = std::move(oval);
    return VTM_OK;
}

vtm_status partial_schur_vertex(const VertexSplit& X, const int32_t* iface, const int32_t* sides, int side,
                                int depth, double drop, std::vector<std::vector<std::pair<int32_t, double>>>& W,
                                std::string& err) {
    const int64_t n = X.n, L = X.L, N = n + L;
    std::vector<char> is_twin(N, 0);
    for (int64_t l = 0; l < L; ++l) {
        is_twin[iface[l]] = 1;
        is_twin[n + l] = 1;
    }
    // graph of the torn matrix, both directions
    std::vector<std::vector<int32_t>> adj(N);
    for (int64_t r = 0; r < N; ++r)
        for (int64_t q = X.rowptr[r]; q < X.rowptr[r + 1]; ++q) {
            const int32_t c = X.col[q];
            if (c == r) continue;
            adj[r].push_back(c);
            adj[c].push_back(int32_t(r));
        }
    // groups of lines with the same two sub-circuits, in (first, second) order
    std::map<std::pair<int32_t, int32_t>, std::vector<int32_t>> by_pair;
    for (int64_t l = 0; l < L; ++l) by_pair[{sides[2 * l], sides[2 * l + 1]}].push_back(int32_t(l));
    const std::vector<std::pair<std::pair<int32_t, int32_t>, std::vector<int32_t>>> groups(by_pair.begin(),
                                                                                         by_pair.end());
    const int64_t G = int64_t(groups.size());
    W.assign(L, {});
    // the groups are independent (each writes the rows of its own lines): they run
    // on host threads, each thread with its own node-index scratch
    std::vector<char> singular(G, 0);
    const int64_t hw = std::max(1u, std::thread::hardware_concurrency());
    const int T = int(std::max<int64_t>(1, std::min<int64_t>({hw, 16, G})));
    for_chunks(G, T, [&](int, int64_t g0, int64_t g1) {
        std::vector<int32_t> loc(N, -1);  // index among the group's twins (< k) or chosen inner nodes (>= k)
        for (int64_t g = g0; g < g1; ++g) {
            auto one_group = [&]() {
                const std::vector<int32_t>& lines = groups[g].second;
                const int32_t blk = side ? groups[g].first.second : groups[g].first.first;
                const int k = int(lines.size());
                std::vector<int32_t> nodes(k);
                for (int a = 0; a < k; ++a) {
                    nodes[a] = side ? int32_t(n + lines[a]) : iface[lines[a]];
                    loc[nodes[a]] = a;
                }
                // inner nodes of the sub-circuit within depth hops of the twins, breadth first
                std::vector<int32_t> frontier(nodes), next;
                for (int hop = 0; !frontier.empty() && (depth < 0 || hop < depth); ++hop) {
                    next.clear();
                    for (int32_t u : frontier)
                        for (int32_t v : adj[u])
                            if (!is_twin[v] && X.part[v] == blk && loc[v] < 0) {
                                loc[v] = int32_t(nodes.size());
                                nodes.push_back(v);
                                next.push_back(v);
                            }
                    frontier.swap(next);
                }
                const int m = int(nodes.size()) - k;
                // dense blocks: C (k x k), E (k x m), F (m x k), D (m x m), from the torn rows
                std::vector<double> C(size_t(k) * k, 0.0), E(size_t(k) * m, 0.0), F(size_t(m) * k, 0.0),
                    D(size_t(m) * m, 0.0);
                for (int a = 0; a < int(nodes.size()); ++a) {
                    const int32_t r = nodes[a];
                    for (int64_t q = X.rowptr[r]; q < X.rowptr[r + 1]; ++q) {
                        const int b = loc[X.col[q]];
                        if (b < 0) continue;
                        const double v = X.val[q];
                        if (a < k && b < k) C[size_t(a) * k + b] += v;
                        else if (a < k) E[size_t(a) * m + (b - k)] += v;
                        else if (b < k) F[size_t(a - k) * k + b] += v;
                        else D[size_t(a - k) * m + (b - k)] += v;
                    }
                }
                // F <- D^-1 F by Gaussian elimination with partial pivoting
                for (int c = 0; c < m; ++c) {
                    int p = c;
                    for (int r = c + 1; r < m; ++r)
                        if (std::fabs(D[size_t(r) * m + c]) > std::fabs(D[size_t(p) * m + c])) p = r;
                    const double piv = D[size_t(p) * m + c];
                    if (piv == 0.0 || !std::isfinite(piv)) {
                        singular[g] = 1;
                        for (int32_t v : nodes) loc[v] = -1;
                        return;
                    }
                    if (p != c) {
                        for (int j = 0; j < m; ++j) std::swap(D[size_t(p) * m + j], D[size_t(c) * m + j]);
                        for (int j = 0; j < k; ++j) std::swap(F[size_t(p) * k + j], F[size_t(c) * k + j]);
                    }
                    for (int r = c + 1; r < m; ++r) {
                        const double f = D[size_t(r) * m + c] / piv;
                        if (f == 0.0) continue;
                        for (int j = c; j < m; ++j) D[size_t(r) * m + j] -= f * D[size_t(c) * m + j];
                        for (int j = 0; j < k; ++j) F[size_t(r) * k + j] -= f * F[size_t(c) * k + j];
                    }
                }
                // back substitution as row operations: each entry of row c takes the
                // products of rows t = c + 1, ... in that order, then the division
                for (int c = m - 1; c >= 0; --c) {
                    const double piv = D[size_t(c) * m + c];
                    double* Fc = &F[size_t(c) * k];
                    for (int t = c + 1; t < m; ++t) {
                        const double d = D[size_t(c) * m + t];
                        const double* Ft = &F[size_t(t) * k];
                        for (int j = 0; j < k; ++j) Fc[j] -= d * Ft[j];
                    }
                    for (int j = 0; j < k; ++j) Fc[j] /= piv;
                }
                // S = C - E (D^-1 F), symmetrized, small entries dropped
                for (int a = 0; a < k; ++a)
                    for (int t = 0; t < m; ++t) {
                        const double e = E[size_t(a) * m + t];
                        if (e == 0.0) continue;
                        for (int j = 0; j < k; ++j) C[size_t(a) * k + j] -= e * F[size_t(t) * k + j];
                    }
                for (int a = 0; a < k; ++a)
                    for (int j = 0; j < k; ++j) {
                        const double v = 0.5 * (C[size_t(a) * k + j] + C[size_t(j) * k + a]);
                        if (a != j && (v == 0.0 || std::fabs(v) < drop * std::sqrt(std::fabs(C[size_t(a) * k + a] *
                                                                                              C[size_t(j) * k + j]))))
                            continue;
                        W[lines[a]].push_back({lines[j], v});
                    }
                for (int32_t v : nodes) loc[v] = -1;
            };
            one_group();
        }
    });
    for (int64_t g = 0; g < G; ++g)
        if (singular[g]) {
            err = "the inner block of the Schur complement approximation is singular";
            return VTM_E_SINGULAR;
        }
    return VTM_OK;
}

vtm_status build_plan_vertex(const vtm_csr* A, const int32_t* label, const int32_t* iface, const int32_t* sides,
                             int64_t L, const double* W, int64_t nW, Plan& P, std::string& err, const vtm_csr* Wc) {
    if (!Wc && (!W || (nW != 1 && nW != L))) {
        err = "nW must be 1 or the number of interfacial nodes";
        return VTM_E_ARG;
    }
    VertexSplit X;
    vtm_status st = split_at_vertices(A, label, iface, sides, L, X, err);
    if (st != VTM_OK) return st;
    const int64_t n = X.n, N = n + L;
    std::vector<int32_t> la(L), lb(L);
    for (int64_t l = 0; l < L; ++l) {
        la[l] = iface[l];
        lb[l] = int32_t(n + l);
    }
    std::vector<double> Z(Wc ? L : nW);
    std::vector<int32_t> wr, wc;  // coupled W, merged and sorted (rows over lines)
    std::vector<double> wv;
    if (Wc) {
        if (Wc->n != L || !Wc->rowptr || (Wc->nnz && (!Wc->col || !Wc->val)) || Wc->rowptr[0] != 0 ||
            Wc->rowptr[L] != Wc->nnz) {
            err = "W must be an n_iface x n_iface CSR";
            return VTM_E_ARG;
        }
        // rows of W with duplicates summed in the caller's order and columns sorted
        wr.assign(L + 1, 0);
        {
            std::vector<std::pair<int32_t, double>> row;
            for (int64_t l = 0; l < L; ++l) {
                if (Wc->rowptr[l + 1] < Wc->rowptr[l]) {
                    err = "W: rowptr must be non-decreasing";
                    return VTM_E_ARG;
                }
                row.clear();
                for (int64_t q = Wc->rowptr[l]; q < Wc->rowptr[l + 1]; ++q) {
                    const int32_t m = Wc->col[q];
                    if (m < 0 || m >= L || !std::isfinite(Wc->val[q])) {
                        err = "W: column out of range or non-finite entry";
                        return VTM_E_ARG;
                    }
                    if (sides[2 * l] != sides[2 * m] || sides[2 * l + 1] != sides[2 * m + 1]) {
                        err = "W couples interfacial nodes " + std::to_string(iface[l]) + " and " +
                              std::to_string(iface[m]) +
                              ", which do not border the same two sub-circuits in the same order";
                        return VTM_E_ARG;
                    }
                    row.push_back({m, Wc->val[q]});
                }
                std::stable_sort(row.begin(), row.end(),
                                 [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
                                     return x.first < y.first;
                                 });
                const size_t start = wc.size();
                for (const auto& e : row) {
                    if (wc.size() > start && wc.back() == e.first)
                        wv.back() += e.second;
                    else {
                        wc.push_back(e.first);
                        wv.push_back(e.second);
                    }
                }
                wr[l + 1] = int32_t(wc.size());
            }
        }
        auto wfind = [&](int32_t r, int32_t c, double& v) -> bool {
            auto lo = wc.begin() + wr[r], hi = wc.begin() + wr[r + 1];
            auto it = std::lower_bound(lo, hi, c);
            if (it == hi || *it != c) return false;
            v = wv[size_t(it - wc.begin())];
            return true;
        };
        for (int64_t l = 0; l < L; ++l)
            for (int32_t q = wr[l]; q < wr[l + 1]; ++q) {
                double v;
                if (!wfind(wc[q], int32_t(l), v) || v != wv[q]) {
                    err = "W must be symmetric";
                    return VTM_E_ARG;
                }
            }
        for (int64_t l = 0; l < L; ++l) {
            double v;
            if (!wfind(int32_t(l), int32_t(l), v) || !(v > 0.0)) {
                err = "W needs a positive diagonal";
                return VTM_E_ARG;
            }
            Z[l] = 1.0 / v;
        }
        // W between the twins on each side: rows of the torn matrix
        std::vector<std::vector<std::pair<int32_t, double>>> rows(N);
        for (int64_t r = 0; r < N; ++r)
            for (int64_t q = X.rowptr[r]; q < X.rowptr[r + 1]; ++q) rows[r].push_back({X.col[q], X.val[q]});
        for (int64_t l = 0; l < L; ++l)
            for (int32_t q = wr[l]; q < wr[l + 1]; ++q) {
                rows[la[l]].push_back({la[wc[q]], wv[q]});
                rows[lb[l]].push_back({lb[wc[q]], wv[q]});
            }
        X.col.clear();
        X.val.clear();
        for (int64_t r = 0; r < N; ++r) {
            for (const auto& e : rows[r]) {
                X.col.push_back(e.first);
                X.val.push_back(e.second);
            }
            X.rowptr[r + 1] = int64_t(X.col.size());
        }
        P.coupled = true;
    } else {
        for (int64_t l = 0; l < nW; ++l) {
            if (!(W[l] > 0.0) || !std::isfinite(W[l])) {
                err = "line admittance must be positive and finite";
                return VTM_E_ARG;
            }
            Z[l] = 1.0 / W[l];
        }
    }
    vtm_csr XA{N, int64_t(X.col.size()), X.rowptr.data(), X.col.data(), X.val.data()};
    st = build_plan(&XA, X.part.data(), Z.data(), int64_t(Z.size()), P, err, la.data(), lb.data(), L);
    if (st != VTM_OK) return st;
    if (P.coupled) {
        // B = 2 W over plan ports: port 2l + s (ABI) couples to 2m + s
        const int64_t np = P.nports;
        std::vector<int32_t> abi_of(np);
        for (int64_t q = 0; q < np; ++q) abi_of[P.abi2port[q]] = int32_t(q);
        P.brow.assign(np + 1, 0);
        P.bcol.clear();
        P.bval.clear();
        for (int64_t p = 0; p < np; ++p) {
            const int32_t q = abi_of[p], l = q >> 1, side = q & 1;
            for (int32_t k = wr[l]; k < wr[l + 1]; ++k) {
                P.bcol.push_back(P.abi2port[2 * wc[k] + side]);
                P.bval.push_back(2.0 * wv[k]);
            }
            P.brow[p + 1] = int32_t(P.bcol.size());
        }
        P.port_row.resize(np);
        for (int64_t s = 0; s < P.S; ++s)
            for (int32_t p = P.port_off[s]; p < P.port_off[s + 1]; ++p) P.port_row[p] = P.sub_off[s] + P.port_node[p];
    }
    // maps between the plan rows and the caller's nodes
    P.n_orig = n;
    std::vector<char> is_if(n, 0);
    for (int64_t l = 0; l < L; ++l) is_if[iface[l]] = 1;
    P.vx_src.resize(N);
    P.vx_w.resize(N);
    for (int64_t r = 0; r < N; ++r) {
        const int64_t e = P.perm[r];  // expanded node
        const bool twin = e >= n || is_if[e];
        P.vx_src[r] = int32_t(e >= n ? iface[e - n] : e);
        P.vx_w[r] = twin ? 0.5 : 1.0;
    }
    P.vr0.resize(n);
    P.vr1.assign(n, -1);
    for (int64_t i = 0; i < n; ++i) P.vr0[i] = P.iperm[i];
    for (int64_t l = 0; l < L; ++l) P.vr1[iface[l]] = P.iperm[n + l];
    P.orow = std::move(X.orow);
    P.ocol = std::move(X.ocol);
    P.oval = std::move(X.oval);
    // the caller's A^T, sorted like A (rows ascending give sorted columns)
    P.orowT.assign(n + 1, 0);
    for (int32_t c : P.ocol) P.orowT[c + 1]++;
    for (int64_t i = 0; i < n; ++i) P.orowT[i + 1] += P.orowT[i];
    P.ocolT.resize(P.ocol.size());
    P.ovalT.resize(P.oval.size());
    std::vector<int32_t> fill(P.orowT.begin(), P.orowT.end() - 1);
    for (int64_t r = 0; r < n; ++r)
        for (int32_t k = P.orow[r]; k < P.orow[r + 1]; ++k) {
            const int32_t w = fill[P.ocol[k]]++;
            P.ocolT[w] = int32_t(r);
            P.ovalT[w] = P.oval[k];
        }
    P.osymmetric = P.orowT == P.orow && P.ocolT == P.ocol && P.ovalT == P.oval;
    if (P.osymmetric) {
        P.orowT.clear();
        P.ocolT.clear();
        P.ovalT.clear();
    }
    return VTM_OK;
}

void transpose_csr(const Plan& P, std::vector<int32_t>& rowptr, std::vector<int32_t>& col,
                   std::vector<double>& val) {
    const int64_t n = P.n, nnz = int64_t(P.col.size());
    // contiguous ranges of rows on host threads; a thread's entries of column c go
    // after those of the threads before it, so every column of A^T lists its rows
    // in ascending order (as a single pass over the rows would)
    const int T = plan_threads(nnz);
    std::vector<std::vector<int32_t>> cnt(T, std::vector<int32_t>(n, 0));
    for_chunks(n, T, [&](int t, int64_t r0, int64_t r1) {
        for (int64_t k = P.rowptr[r0]; k < P.rowptr[r1]; ++k) cnt[t][P.col[k]]++;
    });
    rowptr.assign(n + 1, 0);
    for_chunks(n, T, [&](int, int64_t c0, int64_t c1) {  // per column: its length, each thread's start in it
        for (int64_t c = c0; c < c1; ++c) {
            int32_t run = 0;
            for (int t = 0; t < T; ++t) {
                const int32_t k = cnt[t][c];
                cnt[t][c] = run;
                run += k;
            }
            rowptr[c + 1] = run;
        }
    });
    for (int64_t i = 0; i < n; ++i) rowptr[i + 1] += rowptr[i];
    col.resize(nnz);
    val.resize(nnz);
    for_chunks(n, T, [&](int t, int64_t r0, int64_t r1) {
        std::vector<int32_t>& fill = cnt[t];
        for (int64_t r = r0; r < r1; ++r)
            for (int32_t k = P.rowptr[r]; k < P.rowptr[r + 1]; ++k) {
                const int32_t c = P.col[k];
                const int32_t w = rowptr[c] + fill[c]++;
                col[w] = int32_t(r);
                val[w] = P.val[k];
            }
    });
}

}  // namespace vtm
