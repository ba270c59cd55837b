"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's own
formulas: they check closed forms (Section VIII, Appendix), the paper's printed
worked example (Section IX), exact circuit identities, direct sparse solves and
finite differences.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import workloads


def small_grid(ny=8, nx=8, by=4, bx=4, seed=0, law="uniform"):
    rng = np.random.default_rng(seed)
    e = workloads.grid2d_edges(ny, nx)
    g = rng.uniform(0.5, 2.0, e.shape[0]) if law == "uniform" else 10 ** rng.uniform(-1, 1, e.shape[0])
    n = ny * nx
    A = workloads.nodal_matrix(n, e, g, np.full(n, 0.01))
    part = workloads.block_partition_2d(ny, nx, by, bx)
    b = rng.standard_normal((1, n))
    return A, part, b, e, g


def checkerboard(ny, nx, by, bx):
    nby, nbx = -(-ny // by), -(-nx // bx)
    return np.array([(k // nbx + k % nbx) % 2 for k in range(nby * nbx)])


# ----------------------------------------------------------------------------- O1
def test_midpoint_split_is_exact():
    """Edge-cut reading: i--g--j equals i--2g--m--2g--j; eliminating every middle
    node m (Schur complement) gives back the untorn matrix exactly."""
    A, part, _, _, _ = small_grid()
    wires = oracle.cut_wires(A, part)
    Ae = oracle.expand_midpoints(A, wires).toarray()
    n = A.shape[0]
    S = Ae[:n, :n] - Ae[:n, n:] @ np.linalg.solve(Ae[n:, n:], Ae[n:, :n])
    assert np.allclose(S, A.toarray(), atol=1e-13, rtol=0)


def test_twin_split_identities():
    """Section V, Example 1: C_1 + C_2 = C and f_1 + f_2 = f at the interfacial
    nodes; the torn sub-circuit systems (7)-(8) put together with u_1 = u_2 and
    i_1 = -i_2 give back (6)."""
    A, part, b, _, _ = small_grid()
    torn = oracle.tear_wires(A, part, 1.0)
    wires = oracle.cut_wires(A, part)
    Ae = oracle.expand_midpoints(A, wires)
    n = A.shape[0]
    T = torn.T.tocsr()
    Ca = T[torn.pa, torn.pa].A1
    Cb = T[torn.pb, torn.pb].A1
    assert np.allclose(Ca + Cb, Ae.diagonal()[n:], rtol=0, atol=1e-14)
    # gluing the twins back (sum their rows and columns) reproduces the expanded system
    N = T.shape[0]
    glue = np.zeros((N, Ae.shape[0]))
    for node in range(n):
        glue[torn.out[node].indices[0], node] = 1.0
    glue[torn.pa, n + np.arange(torn.n_lines)] = 1.0
    glue[torn.pb, n + np.arange(torn.n_lines)] = 1.0
    assert np.allclose(glue.T @ T.toarray() @ glue, Ae.toarray(), atol=1e-13, rtol=0)
    f = torn.src @ b.T
    assert np.allclose(glue.T @ f, np.concatenate([b.ravel(), np.zeros(torn.n_lines)])[:, None])


# ----------------------------------------------------------------------------- P1
@pytest.mark.parametrize("cfg,dims,kw", [
    (1, (32, 32), dict()),
    (2, (64, 64), dict()),
    (3, (16, 16, 16), dict()),
    (4, (64, 64), dict(nrhs=3)),
])
def test_fixed_point_is_direct_solution(cfg, dims, kw):
    """Appendix: the limit of the iteration is S^-1 r, i.e. the solution of the
    untorn system; converged VTM equals a sparse LU solve of A x = b."""
    w = workloads.make(cfg, dims=dims, **kw)
    torn = oracle.tear_wires(w.A, w.part, w.Z)
    r = oracle.vtm_solve(torn, w.A, w.b, 1e-13)
    assert r.status == "ok"
    xs = spla.splu(sp.csc_matrix(w.A)).solve(w.b.T).T
    assert np.abs(r.x - xs).max() <= 1e-9 * np.abs(xs).max()


# ----------------------------------------------------------------------------- P2
@pytest.mark.parametrize("law,wmode", [("uniform", "scalar"), ("loguniform", "perwire"),
                                       ("uniform", "coupled")])
def test_sweep_operator_is_reflection(law, wmode):
    """Section VIII / Appendix eqs. (25)-(30): on a 2-coloured tear, one sweep maps
    the waves entering side a to those entering side b by T_a = (W - S_a)(W + S_a)^-1
    (and b to a by T_b), so the sweep operator is [[0, T_b], [T_a, 0]] and its
    spectral radius is sqrt(rho(T_a T_b)) < 1 (Theorem 1, Lemma 3)."""
    A, part, _, _, g = small_grid(8, 8, 4, 4, seed=3, law=law)
    col = checkerboard(8, 8, 4, 4)
    L = oracle.cut_wires(A, part)[0].size
    rng = np.random.default_rng(7)
    if wmode == "scalar":
        W = np.full(L, 1.0 / np.mean(g))
    elif wmode == "perwire":
        W = rng.uniform(0.2, 3.0, L)
    else:
        B = rng.standard_normal((L, L))
        W = B @ B.T / L + 0.5 * np.eye(L)
    if W.ndim == 1:
        torn = oracle.tear_wires(A, part, 1.0 / W, color=col)
    else:
        torn = oracle.tear_wires(A, part, 1.0, color=col)
        torn.W = W
    M = oracle.sweep_operator(torn)
    Sa = oracle.interface_schur(torn, 0)
    Sb = oracle.interface_schur(torn, 1)
    Ta, Tb = oracle.reflection(Sa, torn.W), oracle.reflection(Sb, torn.W)
    assert np.allclose(M[:L, :L], 0, atol=1e-14) and np.allclose(M[L:, L:], 0, atol=1e-14)
    assert np.allclose(M[L:, :L], Ta, atol=1e-12)
    assert np.allclose(M[:L, L:], Tb, atol=1e-12)
    rho = oracle.spectral_radius(M)
    cf = np.sqrt(oracle.spectral_radius(Ta @ Tb))
    assert abs(rho - cf) < 1e-10
    assert rho < 1.0
    assert oracle.spectral_radius(Ta @ Tb) <= oracle.spectral_radius(Ta) * oracle.spectral_radius(Tb) + 1e-12
    assert oracle.spectral_radius(Ta) < 1 and oracle.spectral_radius(Tb) < 1


def test_asymptotic_rate_matches_convergence_factor():
    """The residual of the iteration falls per sweep by the convergence factor
    sqrt(rho(T_1 T_2)) asymptotically (Section VIII)."""
    A, part, b, _, g = small_grid(16, 16, 8, 8, seed=0)
    col = checkerboard(16, 16, 8, 8)
    torn = oracle.tear_wires(A, part, 1.0 / np.mean(g), color=col)
    cf = np.sqrt(oracle.spectral_radius(oracle.reflection(oracle.interface_schur(torn, 0), torn.W)
                                        @ oracle.reflection(oracle.interface_schur(torn, 1), torn.W)))
    r = oracle.vtm_solve(torn, A, b, 1e-13)
    h = np.array(r.history)
    k = len(h) - 60
    ratio = (h[k + 40] / h[k]) ** (1 / 40)
    assert abs(ratio - cf) < 5e-3


# ----------------------------------------------------------------------------- P3
@pytest.mark.parametrize("side", [0, 1])
def test_matched_line_converges_in_one_round_trip(side):
    """Section VIII: with W equal to one side's input admittance that side
    reflects nothing (rho(T_1 T_2) = 0) and the iteration is exact after the
    wave has crossed once each way."""
    A, part, b, _, _ = small_grid(8, 8, 4, 4, seed=5)
    col = checkerboard(8, 8, 4, 4)
    torn = oracle.tear_wires(A, part, 1.0, color=col)
    torn.W = oracle.interface_schur(torn, side)
    torn.W = 0.5 * (torn.W + torn.W.T)
    r = oracle.vtm_solve(torn, A, b, 1e-12, max_sweeps=50)
    assert r.status == "ok" and r.sweeps <= 3
    M = oracle.sweep_operator(torn)
    assert np.abs(M @ M).max() < 1e-10


# ----------------------------------------------------------------------------- P4
@pytest.fixture(scope="module")
def opamp(golden_dir):
    with open(os.path.join(golden_dir, "opamp_example.json")) as fh:
        return json.load(fh)


def opamp_torn(ex, W2, W3):
    A = sp.csr_matrix(np.array(ex["A_eq15"]))
    # 0-based: nodes 1..4 -> 0..3; interfacial nodes 2 and 3; side a holds node 1, side b node 4
    label = np.array([0, -1, -1, 1])
    return A, oracle.tear_at_vertices(A, label, [1, 2], [[0, 1], [0, 1]], np.array([W2, W3]))


def test_opamp_matrix_and_loop_gain(opamp):
    """Section IX, eq. (15): the printed matrix from the printed conductances, and
    the printed loop gain -10^4."""
    c = opamp["conductances"]
    A = np.array([[c["g1"], c["g21"], 0, 0], [0, c["g2"], 0, c["g42"]],
                  [c["g13"], 0, c["g3"], 0], [0, 0, c["g34"], c["g4"]]])
    assert np.array_equal(A, np.array(opamp["A_eq15"]))
    gain = c["g13"] * c["g34"] * c["g42"] * c["g21"] / (c["g1"] * c["g2"] * c["g3"] * c["g4"])
    assert gain == opamp["loop_gain"]


def test_opamp_tear_reproduces_eqs_16_17(opamp):
    """Section IX, eqs. (16)-(17): splitting nodes 2 and 3 with equal halves gives
    exactly the two printed sub-circuit systems; eliminating the inner node of
    each gives the right-hand sides printed in eqs. (20)-(21)."""
    A, torn = opamp_torn(opamp, 1.0, 1.0)
    T = torn.T.toarray()
    blk0 = np.nonzero(torn.block_of == 0)[0]   # u1, u2a, u3a
    blk1 = np.nonzero(torn.block_of == 1)[0]   # u2b, u3b, u4
    # twins come after inner nodes inside a block: reorder block 1 to (u2b, u3b, u4)
    blk1 = np.concatenate([blk1[1:], blk1[:1]])
    assert np.allclose(T[np.ix_(blk0, blk0)], opamp["sub1_eq16"], atol=0)
    assert np.allclose(T[np.ix_(blk1, blk1)], opamp["sub2_eq17"], atol=0)
    # eqs. (20)-(21) right-hand sides for I = (I1..I4)
    I = np.array([0.3, -1.1, 0.7, 2.0])
    f = torn.src @ I
    c = opamp["conductances"]
    r1 = np.array([f[blk0[1]], f[blk0[2]]]) - T[np.ix_(blk0[1:], blk0[:1])] @ [f[blk0[0]] / c["g1"]]
    assert np.allclose(r1, [0.5 * I[1], 0.5 * I[2] - c["g13"] / c["g1"] * I[0]])
    r2 = np.array([f[blk1[0]], f[blk1[1]]]) - T[np.ix_(blk1[:2], blk1[2:])] @ [f[blk1[2]] / c["g4"]]
    assert np.allclose(r2, [0.5 * I[1] - c["g42"] / c["g4"] * I[3], 0.5 * I[2]])
    # the reduced matrices: elimination gives minus signs where the text prints plus
    S1 = oracle.interface_schur(torn, 0)
    assert np.allclose(S1, [[0.5, 0.0], [-c["g13"] * c["g21"] / c["g1"], 0.5]])
    S2 = oracle.interface_schur(torn, 1)
    assert np.allclose(S2, [[0.5, -c["g42"] * c["g34"] / c["g4"]], [0.0, 0.5]])


def test_opamp_classical_methods_diverge(opamp):
    """Section IX, Fig. 6: the classical stationary methods do not converge on
    this circuit.  Jacobi's iteration matrix has lambda^4 = loop gain, so its
    spectral radius is |gain|^(1/4) = 10; Gauss-Seidel also exceeds 1."""
    A = np.array(opamp["A_eq15"])
    assert abs(oracle.spectral_radius(oracle.jacobi_matrix(A)) - 10.0) < 1e-9
    assert oracle.spectral_radius(oracle.gauss_seidel_matrix(A)) > 1.0


def test_opamp_vtm_converges_with_papers_W(opamp):
    """Section IX: with W2 = 0.5 and W3 = 20000 VTM converges to A^-1 I."""
    A, torn = opamp_torn(opamp, opamp["W2"], opamp["W3"])
    I = np.ones((1, 4))
    r = oracle.vtm_solve(torn, A, I, 1e-12, max_sweeps=1000)
    assert r.status == "ok"
    assert np.allclose(r.x.ravel(), np.linalg.solve(A.toarray(), I.ravel()), rtol=1e-10, atol=1e-12)
    assert oracle.spectral_radius(oracle.sweep_operator(torn)) < 0.01


def test_opamp_vtm_diverges_with_poor_W(opamp):
    """Section VIII: for unsymmetric systems the choice of W decides convergence;
    with both admittances 0.5 the same tear diverges and is reported so."""
    A, torn = opamp_torn(opamp, 0.5, 0.5)
    assert oracle.spectral_radius(oracle.sweep_operator(torn)) > 1.0
    r = oracle.vtm_solve(torn, A, np.ones((1, 4)), 1e-12, max_sweeps=1000)
    assert r.status == "diverged"


# ----------------------------------------------------------------------------- P5
def test_single_subcircuit_is_one_direct_solve():
    """No cut: one sweep is one direct solve (Section VI with no lines)."""
    A, _, b, _, _ = small_grid(6, 6, 6, 6)
    part = np.zeros(36, dtype=np.int32)
    torn = oracle.tear_wires(A, part, 1.0)
    assert torn.n_lines == 0
    r = oracle.vtm_solve(torn, A, b, 1e-14)
    assert r.sweeps == 1
    assert np.allclose(r.x, np.linalg.solve(A.toarray(), b.ravel()), rtol=1e-13)


def test_two_nodes_one_wire_closed_form():
    """Two grounded nodes joined by g, torn at the branch: each side's input
    admittance at its half-wire is the series value 2g*g_k/(2g + g_k), so the
    sweep operator has spectral radius sqrt(|T_1 T_2|) with scalar
    T_k = (W - S_k)/(W + S_k)."""
    g, g1, g2, W = 0.7, 0.3, 1.9, 1.3
    A = sp.csr_matrix(np.array([[g1 + g, -g], [-g, g2 + g]]))
    torn = oracle.tear_wires(A, np.array([0, 1]), 1.0 / W)
    S1 = 2 * g * g1 / (2 * g + g1)
    S2 = 2 * g * g2 / (2 * g + g2)
    T1, T2 = (W - S1) / (W + S1), (W - S2) / (W + S2)
    M = oracle.sweep_operator(torn)
    assert np.allclose(M, [[0, T2], [T1, 0]], atol=1e-15)
    b = np.array([[1.0, -2.0]])
    r = oracle.vtm_solve(torn, A, b, 1e-14)
    assert np.allclose(r.x.ravel(), np.linalg.solve(A.toarray(), b.ravel()), rtol=1e-12)


def test_fixed_point_independent_of_partition_and_W():
    """Appendix: the limit S^-1 r depends on neither the tear nor W."""
    A, part, b, _, g = small_grid(12, 12, 4, 4, seed=2)
    xs = np.linalg.solve(A.toarray(), b.ravel())
    for p, Z in [(part, 1 / np.mean(g)), (workloads.block_partition_2d(12, 12, 6, 3), 0.2),
                 (workloads.block_partition_2d(12, 12, [5, 7], [2, 10]), 3.0)]:
        r = oracle.vtm_solve(oracle.tear_wires(A, p, Z), A, b, 1e-13)
        assert np.abs(r.x.ravel() - xs).max() < 1e-10 * np.abs(xs).max()


def test_eliminated_form_matches_twin_form():
    """Eliminating each twin (the form a per-subdomain kernel applies) changes no
    iterate: x^k of both forms agree to rounding for 40 sweeps, with per-wire
    admittances and on an unsymmetric circuit; W = 2g makes the line reflect
    nothing back (gamma = 0)."""
    for cfg, dims in [(1, (16, 16)), (3, (8, 8, 16))]:
        w = workloads.make(cfg, dims=dims, block=(4, 4) if cfg == 1 else None)
        L = oracle.cut_wires(w.A, w.part)[0].size
        Z = np.random.default_rng(1).uniform(0.3, 2.0, L)
        torn = oracle.tear_wires(w.A, w.part, Z)
        el = oracle.eliminate_twins(w.A, w.part, Z)
        xs_e = oracle.vtm_solve_eliminated(el, w.A, w.b[0], 40)
        sw = oracle.Sweeper(torn)
        f = torn.src @ w.b.T
        a = np.zeros((2, L, 1))
        for k in range(40):
            u, a = sw.sweep(f, a)
            x = (torn.out @ u).ravel()
            assert np.abs(x - xs_e[k]).max() <= 1e-12 * np.abs(x).max()
    A, part, _, _, _ = small_grid(4, 4, 2, 2)
    i, j, g = oracle.cut_wires(A, part)
    el = oracle.eliminate_twins(A, part, 1.0 / (2 * g))
    assert np.allclose(el.gamma, 0.0, atol=1e-15)
    assert np.allclose(el.G, np.repeat(g, 2)) and np.allclose(el.c, 0.5)


# ----------------------------------------------------------------------------- P6
@pytest.mark.parametrize("cfg,dims", [(1, None), (2, (128, 128)), (4, (96, 96)), (5, (64, 64))])
def test_lemma1_grounded_resistor_grids_are_spd(cfg, dims):
    """Lemma 1: a resistor network with a ground conductance is SPD (dense
    Cholesky succeeds; strict diagonal dominance holds)."""
    w = workloads.make(cfg, dims=dims)
    A = w.A
    assert abs(A - A.T).max() == 0
    d = A.diagonal()
    off = np.asarray(abs(A).sum(axis=1)).ravel() - np.abs(d)
    assert np.all(d > off)
    if A.shape[0] <= 5000:
        np.linalg.cholesky(A.toarray())


def test_adjoint_of_symmetric_is_forward_and_unsymmetric_is_transpose():
    """VTM on A^T (the torn A^T is the transposed torn A when every unsymmetric
    entry lies inside one sub-circuit) converges to the direct adjoint A^-T g;
    for symmetric A it is the forward solve iterate by iterate."""
    w = workloads.make(3, dims=(16, 16, 16))
    g = np.random.default_rng(3).standard_normal((1, w.n))
    torn_t = oracle.tear_wires(w.A.T.tocsr(), w.part, w.Z)
    torn = oracle.tear_wires(w.A, w.part, w.Z)
    assert abs(torn_t.T - torn.T.T).max() == 0
    r = oracle.vtm_solve(torn_t, w.A.T.tocsr(), g, 1e-12)
    lam = oracle.direct_adjoint(w.A, g)
    assert np.abs(r.x - lam).max() <= 1e-9 * np.abs(lam).max()
    w1 = workloads.make(1, dims=(32, 32))
    t1 = oracle.tear_wires(w1.A, w1.part, w1.Z)
    t1t = oracle.tear_wires(w1.A.T.tocsr(), w1.part, w1.Z)
    ra = oracle.vtm_solve(t1, w1.A, w1.b, 1e-10)
    rb = oracle.vtm_solve(t1t, w1.A.T.tocsr(), w1.b, 1e-10)
    assert ra.sweeps == rb.sweeps and np.array_equal(ra.x, rb.x)


# ----------------------------------------------------------------------------- P7
def test_branch_gradient_matches_finite_differences():
    """dL/dg for L = sum over probes of x_p^2: the adjoint formula
    -(lambda_i - lambda_j)(x_i - x_j) with A^T lambda = dL/dx, lambda from VTM on
    A^T, against central differences of L from direct solves."""
    w = workloads.make(5, dims=(32, 32), n_probes=64)
    torn = oracle.tear_wires(w.A, w.part, w.Z)
    x = oracle.vtm_solve(torn, w.A, w.b, 1e-13).x
    dLdx = np.zeros_like(x)
    dLdx[:, w.probes] = 2 * x[:, w.probes]
    lam = oracle.vtm_solve(oracle.tear_wires(w.A.T.tocsr(), w.part, w.Z), w.A.T.tocsr(), dLdx, 1e-13).x
    grad = oracle.branch_gradient(w.edges, x, lam)
    pick = np.random.default_rng(11).choice(w.edges.shape[0], 64, replace=False)

    def loss(g):
        A = workloads.nodal_matrix(w.n, w.edges, g, w.ground)
        xx = spla.splu(sp.csc_matrix(A)).solve(w.b.ravel())
        return np.sum(xx[w.probes] ** 2)

    fd = []
    for e in pick:
        h = 1e-5 * w.g[e]
        gp, gm = w.g.copy(), w.g.copy()
        gp[e] += h
        gm[e] -= h
        fd.append((loss(gp) - loss(gm)) / (2 * h))
    fd = np.array(fd)
    assert np.abs(fd - grad[pick]).max() <= 1e-5 * np.abs(grad).max()


def test_matrix_gradient_matches_finite_differences():
    """dL/dA per stored entry (-lambda_i x_j, summed over columns) for
    L = sum over probes of x_p^2 on the unsymmetric 3-D workload, against
    central differences of L from direct solves: every controlled-source gain
    (a single one-sided entry, Section IX eq. 15) and some diagonal and branch
    entries, with two right-hand sides."""
    w = workloads.make(3, dims=(8, 8, 16), nrhs=2)
    A = sp.csr_matrix(w.A)
    probes = np.random.default_rng(3).choice(w.n, 64, replace=False)
    x = oracle.direct_solve(A, w.b)
    dLdx = np.zeros_like(x)
    dLdx[:, probes] = 2 * x[:, probes]
    grad = oracle.matrix_gradient(A, x, oracle.direct_adjoint(A, dLdx))
    assert grad.shape == (A.nnz,)
    rows = np.repeat(np.arange(w.n), np.diff(A.indptr))
    k_node, c_node, _ = w.vccs
    vccs_entries = [int(np.nonzero((rows == k) & (A.indices == c))[0][0]) for k, c in zip(k_node, c_node)]
    rng = np.random.default_rng(5)
    pick = sorted(set(vccs_entries) | set(rng.choice(A.nnz, 24, replace=False).tolist()))

    def loss(Ak):
        xx = spla.splu(sp.csc_matrix(Ak)).solve(w.b.T)
        return np.sum(xx[probes] ** 2)

    fd = []
    for k in pick:
        h = 1e-5 * abs(A.data[k])
        Ap, Am = A.copy(), A.copy()
        Ap.data[k] += h
        Am.data[k] -= h
        fd.append((loss(Ap) - loss(Am)) / (2 * h))
    fd = np.array(fd)
    assert len(vccs_entries) >= 20
    assert np.abs(fd - grad[pick]).max() <= 1e-6 * np.abs(grad[pick]).max()


# ----------------------------------------------------------------------------- failure paths
def test_untearable_cross_coupling_is_rejected():
    """A controlled source between two sub-circuits is not a two-terminal
    conductance and cannot be replaced by a line."""
    A, part, _, _, _ = small_grid(4, 4, 2, 2)
    A = A.tolil()
    A[0, 2] += 0.3          # nodes 0 and 2 lie in different 2x2 blocks
    with pytest.raises(oracle.UntearableError):
        oracle.cut_wires(A.tocsr(), part)


def test_maxiter_and_zero_rhs():
    A, part, b, _, _ = small_grid()
    torn = oracle.tear_wires(A, part, 1.0)
    r = oracle.vtm_solve(torn, A, b, 1e-14, max_sweeps=5)
    assert r.status == "maxiter" and r.sweeps == 5
    r0 = oracle.vtm_solve(torn, A, np.zeros_like(b), 1e-10)
    assert r0.status == "ok" and r0.sweeps == 0 and not r0.x.any()


def test_refinement_reaches_tolerance():
    """Refinement schedule (outer FP64 residual, inner VTM to a fixed drop) ends at
    the requested residual and at the direct solution.  Parity unpinned beyond that."""
    w = workloads.make(5, dims=(64, 64))
    torn = oracle.tear_wires(w.A, w.part, w.Z)
    rr = oracle.vtm_refine(torn, w.A, w.b, 1e-8, inner_drop=1e-5)
    assert rr.status == "ok" and rr.relres.max() <= 1e-8 and rr.outer >= 2
    xs = oracle.direct_solve(w.A, w.b)
    assert np.abs(rr.x - xs).max() <= 1e-6 * np.abs(xs).max()


def test_refinement_steps_are_plain_vtm_on_the_residual():
    """Each outer step of the refinement schedule is plain VTM (Section VI) on the
    current residual r = b - A x from zero waves: it stops at the first check
    (every 8 sweeps) where plain VTM on r meets the step's target, max(drop,
    tol / (2 ||r|| / ||b||)), and adds that VTM iterate to x.  Two steps are
    rebuilt here from vtm_solve alone (its own pins hold it to the paper)."""
    w = workloads.make(5, dims=(64, 64))
    torn = oracle.tear_wires(w.A, w.part, w.Z)
    tol, drop = 1e-8, 1e-5
    x = np.zeros_like(w.b)
    for step in (1, 2):
        rel = oracle.relative_residual(w.A, w.b, x).max()
        target = max(drop, 0.5 * tol / rel)
        r = w.b - (w.A @ x.T).T
        plain = oracle.vtm_solve(torn, w.A, r, target)
        assert plain.status == "ok"
        stop = 8 * -(-plain.sweeps // 8)
        x = x + oracle.vtm_solve(torn, w.A, r, 0.0, max_sweeps=stop).x
        rr = oracle.vtm_refine(torn, w.A, w.b, tol, inner_drop=drop, max_outer=step)
        assert rr.inner_sweeps[step - 1] == stop
        assert np.allclose(rr.x, x, rtol=0, atol=1e-13 * np.abs(x).max())


@pytest.mark.parametrize("cfg,kw", [(1, dict()), (3, dict(dims=(16, 16, 16))), (4, dict(dims=(48, 48)))])
def test_interface_residual_equals_untorn_residual(cfg, kw):
    """The residual of a VTM iterate lives on the port nodes: computed from the
    waves of the sweep alone, it equals b - A x^k on the untorn A (zero off the
    port nodes), for symmetric and unsymmetric A alike."""
    w = workloads.make(cfg, **kw)
    el = oracle.eliminate_twins(w.A, w.part, w.Z)
    waves = []
    xs = oracle.vtm_solve_eliminated(el, w.A, w.b[0], 12, waves=waves)
    ports = np.zeros(w.n, bool)
    ports[el.port_node] = True
    for k in (0, 3, 11):
        r = w.b[0] - w.A @ xs[k]
        ri = oracle.interface_residual(el, w.n, *waves[k])
        scale = np.abs(w.b[0]).max()
        assert np.abs(r[~ports]).max() <= 1e-12 * scale
        assert np.abs(ri - r).max() <= 1e-11 * scale
        assert np.abs(ri[ports]).max() > 1e-6 * scale    # not trivially zero
