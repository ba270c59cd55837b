"""Parity of tearing at interfacial nodes (vtm_setup_vertex, through the C ABI)
with the oracle's level-one vertex tear (Section V, Steps 1-4; Section IX).

Iterates are compared element by element after the same number of sweeps, to
the FP64 bound of the edge-cut tests (1e-11 of max |x|): each sweep rounds
dense dot products of at most a few hundred terms and the iteration contracts.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import workloads

pytestmark = pytest.mark.gpu

ITER_RTOL = 1e-11


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a HIP device"
    return T


def vtm():
    import paper_0910_0663_amd as v
    return v


def to_dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def strips(dims, width, law="loguniform", seed=0, nrhs=1, vccs=False):
    """A grid circuit cut into strips by separator layers of interfacial nodes."""
    if vccs:
        w = workloads.make(3, dims=dims, nrhs=nrhs, seed=seed)
        A, b = w.A, w.b
    else:
        rng = np.random.default_rng(seed)
        edges = workloads.grid2d_edges(*dims) if len(dims) == 2 else workloads.grid3d_edges(*dims)
        m = edges.shape[0]
        g = 10.0 ** rng.uniform(-1, 1, m) if law == "loguniform" else rng.uniform(0.5, 2.0, m)
        n = int(np.prod(dims))
        A = workloads.nodal_matrix(n, edges, g, np.full(n, workloads.GROUND_S))
        b = rng.standard_normal((nrhs, n))
    label, iface, sides = workloads.separator_strips(dims, width)
    off = A.tocoo()
    br = (off.row != off.col) & (off.data < 0)
    W = float(np.mean(-off.data[br]))   # mean branch conductance, as for the wire-cut workloads
    return A, b, label, iface, sides, W


def dense(W):
    return W.toarray() if sp.issparse(W) else W


def oracle_iterates(A, b, label, iface, sides, W, ks):
    torn = oracle.tear_at_vertices(A, label, iface, sides, dense(W))
    sw = oracle.Sweeper(torn)
    f = torn.src @ b.T
    a = np.zeros((2, torn.n_lines, b.shape[0]))
    out = {}
    for k in range(1, max(ks) + 1):
        u, a = sw.sweep(f, a)
        if k in ks:
            out[k] = (torn.out @ u).T
    return out


def solver(A, label, iface, sides, W, **kw):
    """vtm_setup_vertex for a scalar or per-line W, vtm_setup_vertex_coupled for a sparse matrix."""
    if sp.issparse(W):
        return vtm().Solver(A, label, None, iface=iface, sides=sides, W=W, **kw)
    Z = 1.0 / np.asarray(W, dtype=np.float64)
    return vtm().Solver(A, label, Z, iface=iface, sides=sides, **kw)


def gpu_iterate(torch, A, b, label, iface, sides, W, k, check_every=1, **kw):
    s = solver(A, label, iface, sides, W, nrhs_max=b.shape[0], check_every=check_every, max_sweeps=k,
               adaptive_checks=False, **kw)
    x = torch.empty(b.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(vtm().VTMError) as ei:
        s.solve(to_dev(torch, b), 1e-300, x)
    assert ei.value.name == "VTM_E_MAXITER"
    assert ei.value.report.sweeps == k
    s.close()
    return x.cpu().numpy()


def assert_close(x, ref, rtol=ITER_RTOL):
    scale = np.abs(ref).max()
    err = np.abs(x - ref).max()
    assert err <= rtol * scale, f"max err {err:.3e} vs scale {scale:.3e}"


@pytest.fixture(scope="module")
def opamp(golden_dir):
    with open(os.path.join(golden_dir, "opamp_example.json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("form", ["full", "port", "port_dense"])
def test_opamp_example_converges_with_papers_W(torch, opamp, form):
    """Section IX: the op-amp circuit of eq. (15), nodes 2 and 3 split, W2 = 0.5,
    W3 = 20000: VTM reaches A^-1 I although Jacobi and Gauss-Seidel diverge."""
    A = sp.csr_matrix(np.array(opamp["A_eq15"], dtype=np.float64))
    label, iface, sides = np.array([0, -1, -1, 1]), np.array([1, 2]), np.array([[0, 1], [0, 1]])
    W = np.array([opamp["W2"], opamp["W3"]])
    b = np.array([[1.0, 1.0, 1.0, 1.0], [0.3, -1.1, 0.7, 2.0]])
    s = solver(A, label, iface, sides, W, nrhs_max=2, check_every=1, adaptive_checks=False, local_form=form)
    x, rep = s.solve(to_dev(torch, b), 1e-12)
    xs = np.linalg.solve(A.toarray(), b.T).T
    assert np.allclose(x.cpu().numpy(), xs, rtol=1e-10, atol=1e-12)
    ref = oracle.vtm_solve(oracle.tear_at_vertices(A, label, iface, sides, W), A, b, 1e-12, max_sweeps=100)
    assert ref.status == "ok" and abs(rep.sweeps - ref.sweeps) <= 1
    # the adjoint: the same tear of A^T (the oracle tears A^T itself)
    At = A.T.tocsr()
    lam, rep = s.solve_adjoint(to_dev(torch, b), 1e-12)
    assert np.allclose(lam.cpu().numpy(), np.linalg.solve(At.toarray(), b.T).T, rtol=1e-10, atol=1e-12)
    ref = oracle.vtm_solve(oracle.tear_at_vertices(At, label, iface, sides, W), At, b, 1e-12, max_sweeps=100)
    assert ref.status == "ok" and abs(rep.sweeps - ref.sweeps) <= 1


def test_opamp_example_diverges_with_poor_W(torch, opamp):
    """Section VIII: with both admittances 0.5 the same tear diverges."""
    A = sp.csr_matrix(np.array(opamp["A_eq15"], dtype=np.float64))
    s = solver(A, np.array([0, -1, -1, 1]), np.array([1, 2]), np.array([[0, 1], [0, 1]]), np.array([0.5, 0.5]),
               check_every=1)
    with pytest.raises(vtm().VTMError) as ei:
        s.solve(to_dev(torch, np.ones(4)), 1e-12)
    assert ei.value.name == "VTM_E_DIVERGED"


@pytest.mark.parametrize("dims,width,kw", [
    ((24, 47), 10, dict()),                                 # 2-D strips of 24 x 10: packed port-node form
    ((24, 47), 10, dict(local_form="full")),
    ((24, 47), 10, dict(local_form="port_dense")),
    ((40, 47), 10, dict()),                                 # 80 ports per strip: dense port-to-port form
    ((12, 12, 23), 5, dict()),                              # 3-D slabs of 12 x 12 x 5
])
def test_separator_strip_iterates_match_oracle(torch, dims, width, kw):
    A, b, label, iface, sides, W = strips(dims, width)
    ks = [1, 2, 7]
    ref = oracle_iterates(A, b, label, iface, sides, W, ks)
    for k in ks:
        assert_close(gpu_iterate(torch, A, b, label, iface, sides, W, k, **kw), ref[k])
    # port-to-port sweeps between the first and the last
    assert_close(gpu_iterate(torch, A, b, label, iface, sides, W, 7, check_every=7, **kw), ref[7])


def test_per_line_admittance_and_several_rhs(torch):
    A, b, label, iface, sides, _ = strips((24, 35), 8, nrhs=3, seed=4)
    W = np.random.default_rng(1).uniform(0.3, 3.0, iface.size)
    ref = oracle_iterates(A, b, label, iface, sides, W, [5])
    assert_close(gpu_iterate(torch, A, b, label, iface, sides, W, 5), ref[5])


def test_batched_mfma_layout_iterates_match_oracle(torch):
    A, b, label, iface, sides, W = strips((16, 35), 8, nrhs=16, seed=6)
    ref = oracle_iterates(A, b, label, iface, sides, W, [4])
    assert_close(gpu_iterate(torch, A, b, label, iface, sides, W, 4, check_every=4), ref[4])


def test_batched_bf16_long_separator_reaches_tolerance(torch):
    """A separator of 1,024 interfacial nodes (1024 x 7 grid, two strips of 3,072
    inner nodes): each sub-circuit's 1,024-port operator leaves no room to stage h
    beside the incident waves in LDS, so the batched BF16 port-to-port sweep reads
    h at the store; BF16 refinement still reaches 1e-8 in every column."""
    A, b, label, iface, sides, W = strips((1024, 7), 3, nrhs=16, seed=3)
    s = solver(A, label, iface, sides, W, precision="bf16_refine", nrhs_max=16)
    x, rep = s.solve(to_dev(torch, b), 1e-8)
    assert rep.pp_shape[0] > 0  # the batched port-to-port form ran
    assert oracle.relative_residual(A, b, x.cpu().numpy()).max() <= 1e-8


def test_unsymmetric_slabs_iterate_and_converge(torch):
    """Controlled sources inside the slabs (unsymmetric A)."""
    A, b, label, iface, sides, W = strips((6, 10, 23), 5, vccs=True)
    ref = oracle_iterates(A, b, label, iface, sides, W, [6])
    assert_close(gpu_iterate(torch, A, b, label, iface, sides, W, 6, check_every=3), ref[6])
    r = oracle.vtm_solve(oracle.tear_at_vertices(A, label, iface, sides, W), A, b, 1e-9, max_sweeps=5000)
    assert r.status == "ok"
    s = solver(A, label, iface, sides, W, check_every=1, adaptive_checks=False)
    x, rep = s.solve(to_dev(torch, b), 1e-9)
    assert abs(rep.sweeps - r.sweeps) <= 1
    assert rep.relres_max <= 1e-9


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_separator_strips_solve_to_tolerance(torch, prec):
    """Sweep count of the FP64 path that of the oracle (within one, for rounding at the threshold);
    both precisions reach the FP64 tolerance on the untorn A."""
    A, b, label, iface, sides, W = strips((48, 59), 11, seed=2)
    tol = 1e-10
    r = oracle.vtm_solve(oracle.tear_at_vertices(A, label, iface, sides, W), A, b, tol, max_sweeps=20000)
    assert r.status == "ok"
    s = solver(A, label, iface, sides, W, precision=prec, check_every=1 if prec == "fp64" else 8,
               adaptive_checks=False)
    x, rep = s.solve(to_dev(torch, b), tol)
    assert rep.relres_max <= tol
    xs = spla.spsolve(A.tocsc(), b[0])
    assert np.abs(x.cpu().numpy()[0] - xs).max() <= 1e-7 * np.abs(xs).max()
    if prec == "fp64":
        assert abs(rep.sweeps - r.sweeps) <= 1


# ---------------------------------------------------------------- coupled lines
def coupled(dims, width, rule, alpha=1.0, **kw):
    A, b, label, iface, sides, _ = strips(dims, width, **kw)
    W = vtm().vertex_admittance(A, label, iface, sides, rule, alpha)
    return A, b, label, iface, sides, W


@pytest.mark.parametrize("rule,alpha,kw", [
    ("ob", 1.0, dict()),                                    # dense port-to-port form with B = 2 W
    ("ob", 1.0, dict(local_form="full")),
    ("wob", 0.3, dict(local_form="port_dense")),
    ("diag", 1.0, dict()),
])
def test_coupled_line_iterates_match_oracle(torch, rule, alpha, kw):
    """Section VIII rules 2-4 as coupled lines (eqs. 4-5): W over each
    separator's interfacial nodes, with the branches between them."""
    A, b, label, iface, sides, W = coupled((24, 47), 10, rule, alpha)
    ks = [1, 2, 7]
    ref = oracle_iterates(A, b, label, iface, sides, W, ks)
    for k in ks:
        assert_close(gpu_iterate(torch, A, b, label, iface, sides, W, k, **kw), ref[k])
    assert_close(gpu_iterate(torch, A, b, label, iface, sides, W, 7, check_every=7, **kw), ref[7])


def test_diagonal_W_as_coupled_lines_equals_per_line_W(torch):
    A, b, label, iface, sides, W = coupled((24, 47), 10, "diag")
    x1 = gpu_iterate(torch, A, b, label, iface, sides, W, 9, check_every=3)
    x2 = gpu_iterate(torch, A, b, label, iface, sides, W.diagonal().copy(), 9, check_every=3)
    assert_close(x1, x2)


def test_coupled_lines_batched_and_three_dimensional(torch):
    A, b, label, iface, sides, W = coupled((16, 35), 8, "ob", nrhs=16, seed=6)
    ref = oracle_iterates(A, b, label, iface, sides, W, [5])
    assert_close(gpu_iterate(torch, A, b, label, iface, sides, W, 5, check_every=5), ref[5])
    A, b, label, iface, sides, W = coupled((8, 9, 23), 5, "wob", 0.5, law="uniform")
    ref = oracle_iterates(A, b, label, iface, sides, W, [6])
    assert_close(gpu_iterate(torch, A, b, label, iface, sides, W, 6, check_every=3), ref[6])


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_coupled_lines_solve_to_tolerance(torch, prec):
    A, b, label, iface, sides, W = coupled((48, 59), 11, "wob", 0.3, seed=2)
    tol = 1e-10
    r = oracle.vtm_solve(oracle.tear_at_vertices(A, label, iface, sides, dense(W)), A, b, tol, max_sweeps=20000)
    assert r.status == "ok"
    s = solver(A, label, iface, sides, W, precision=prec, check_every=1 if prec == "fp64" else 8,
               adaptive_checks=False)
    x, rep = s.solve(to_dev(torch, b), tol)
    assert rep.relres_max <= tol
    if prec == "fp64":
        assert abs(rep.sweeps - r.sweeps) <= 1


def test_table2_ordering_on_the_gpu(torch):
    """Table II, qualitatively, on a 100 x 100 unit resistor grid cut into
    strips of 100 x 18 by five separator columns (2000 nodes per torn strip
    with its twins): the GPU's sweep counts are the oracle's, and diagonal >
    overlapped block > weighted overlapped block."""
    dims = (100, 100)
    e = workloads.grid2d_edges(*dims)
    n = int(np.prod(dims))
    A = workloads.nodal_matrix(n, e, np.ones(e.shape[0]), np.full(n, workloads.GROUND_S))
    b = np.random.default_rng(0).standard_normal((1, n))
    label, iface, sides = workloads.separator_strips(dims, 18)
    sweeps = {}
    for rule, alpha in (("diag", 1.0), ("ob", 1.0), ("wob", 0.3)):
        W = vtm().vertex_admittance(A, label, iface, sides, rule, alpha)
        r = oracle.vtm_solve(oracle.tear_at_vertices(A, label, iface, sides, W.toarray()), A, b, 1e-8,
                             max_sweeps=5000)
        s = solver(A, label, iface, sides, W, check_every=1, adaptive_checks=False)
        x, rep = s.solve(to_dev(torch, b), 1e-8)
        assert abs(rep.sweeps - r.sweeps) <= 1
        sweeps[rule] = rep.sweeps
    assert sweeps["diag"] > sweeps["ob"] > sweeps["wob"]


def test_coupled_W_is_checked(torch):
    A, b, label, iface, sides, W = coupled((12, 23), 5, "ob")
    def status(Wbad):
        with pytest.raises(vtm().VTMError) as ei:
            solver(A, label, iface, sides, sp.csr_matrix(Wbad))
        return ei.value.name
    Wd = W.toarray()
    # lines of different separators (different pairs of strips) coupled
    a, c = 0, int(np.nonzero(sides[:, 0] != sides[0, 0])[0][0])
    X = Wd.copy()
    X[a, c] = X[c, a] = -0.1
    assert status(X) == "VTM_E_ARG"
    X = Wd.copy()
    X[0, 1] += 0.1                                  # not symmetric
    assert status(X) == "VTM_E_ARG"
    X = Wd.copy()
    X[3, 3] = 0.0                                   # no positive diagonal
    assert status(X) == "VTM_E_ARG"


def test_table2_two_sub_circuits_on_the_gpu(torch):
    """Table II's Grid2d setting itself: a 100 x 100 unit resistor grid torn into
    two sub-circuits at one separator column of 100 interfacial nodes (5,050
    torn nodes each).  The GPU's sweep counts are the oracle's for the
    diagonal, overlapped-block, weighted overlapped-block and Schur complement
    approximation (two layers of the interior) W, and x is the direct
    solution."""
    dims = (100, 100)
    e = workloads.grid2d_edges(*dims)
    n = int(np.prod(dims))
    A = workloads.nodal_matrix(n, e, np.ones(e.shape[0]), np.full(n, workloads.GROUND_S))
    b = np.random.default_rng(0).standard_normal((1, n))
    label, iface, sides = workloads.separator_strips(dims, 49)
    assert iface.size == 100 and label.max() == 1
    xs = spla.spsolve(A.tocsc(), b[0])
    for rule, alpha in (("diag", 1.0), ("ob", 1.0), ("wob", 0.3), ("sca", 2)):
        W = (vtm().vertex_sca(A, label, iface, sides, 0, alpha) if rule == "sca"
             else vtm().vertex_admittance(A, label, iface, sides, rule, alpha))
        r = oracle.vtm_solve(oracle.tear_at_vertices(A, label, iface, sides, W.toarray()), A, b, 1e-8,
                             max_sweeps=5000)
        s = solver(A, label, iface, sides, W, check_every=1, adaptive_checks=False)
        x, rep = s.solve(to_dev(torch, b), 1e-8)
        assert abs(rep.sweeps - r.sweeps) <= 1, (rule, rep.sweeps, r.sweeps)
        assert np.abs(x.cpu().numpy()[0] - xs).max() <= 1e-6 * np.abs(xs).max()
        s.close()


@pytest.mark.parametrize("depth,drop,kw", [
    (2, 0.0, dict()),
    (3, 0.02, dict(local_form="full")),
    (1, 0.0, dict(precision="fp32_refine")),
])
def test_schur_complement_approximation_iterates(torch, depth, drop, kw):
    """Rule 5 of Section VIII (vtm_vertex_sca) as coupled lines: iterates equal
    the oracle's with the oracle's own partial Schur complement as W."""
    A, b, label, iface, sides, _ = strips((24, 47), 10, seed=3)
    W = vtm().vertex_sca(A, label, iface, sides, 0, depth, drop)
    torn = oracle.tear_at_vertices(A, label, iface, sides, 1.0)
    Wo = oracle.partial_schur(torn, 0, depth, drop)
    assert np.abs(W.toarray() - Wo).max() <= 1e-13 * np.abs(Wo).max()
    if kw.get("precision") == "fp32_refine":
        r = oracle.vtm_solve(oracle.tear_at_vertices(A, label, iface, sides, Wo), A, b, 1e-10, max_sweeps=5000)
        s = solver(A, label, iface, sides, W, check_every=8, **kw)
        x, rep = s.solve(to_dev(torch, b), 1e-10)
        assert r.status == "ok" and rep.relres_max <= 1e-10
        return
    ks = [1, 2, 6]
    ref = oracle_iterates(A, b, label, iface, sides, Wo, ks)
    for k in ks:
        assert_close(gpu_iterate(torch, A, b, label, iface, sides, W, k, **kw), ref[k])
    assert_close(gpu_iterate(torch, A, b, label, iface, sides, W, 6, check_every=6, **kw), ref[6])


@pytest.mark.parametrize("case", ["symmetric", "controlled_sources", "coupled"])
def test_adjoint_iterates_match_oracle_tear_of_the_transpose(torch, case):
    """vtm_solve_adjoint with tearing at interfacial nodes: x^k of VTM on the
    oracle's tear of A^T (which the split rule makes the transposed tear of A),
    and the adjoint solution at the end."""
    if case == "controlled_sources":
        A, b, label, iface, sides, W = strips((6, 10, 23), 5, vccs=True)
    elif case == "coupled":
        A, b, label, iface, sides, W = coupled((24, 47), 10, "wob", 0.5, seed=5)
    else:
        A, b, label, iface, sides, W = strips((24, 47), 10, seed=5)
    At = A.T.tocsr()
    ref = oracle_iterates(At, b, label, iface, sides, W, [1, 4])
    for k, ce in ((1, 1), (4, 1), (4, 4)):
        s = solver(A, label, iface, sides, W, check_every=ce, max_sweeps=k, adaptive_checks=False)
        lam = torch.empty(b.shape, dtype=torch.float64, device="cuda")
        with pytest.raises(vtm().VTMError) as ei:
            s.solve_adjoint(to_dev(torch, b), 1e-300, lam)
        assert ei.value.name == "VTM_E_MAXITER" and ei.value.report.sweeps == k
        assert_close(lam.cpu().numpy(), ref[k])
    s = solver(A, label, iface, sides, W, check_every=8)
    lam, rep = s.solve_adjoint(to_dev(torch, b), 1e-10)
    ls = spla.spsolve(At.tocsc(), b[0])
    assert rep.relres_max <= 1e-10
    assert np.abs(lam.cpu().numpy()[0] - ls).max() <= 1e-7 * np.abs(ls).max()


def test_table2_grid3d_two_sub_circuits_on_the_gpu(torch):
    """Table II's Grid3d setting: a 30^3 unit resistor grid torn in two at one
    30 x 30 separator plane (900 interfacial nodes; 12,600 + 900 and 13,500 +
    900 torn nodes, one right-hand side).  With W = 0.3 C the GPU needs the
    oracle's sweeps and reaches the direct solution.  Sub-circuits this large
    (their x does not fit LDS beside the right-hand side) also take the adjoint
    and two right-hand sides, which reach the direct solutions too."""
    dims = (30, 30, 30)
    e = workloads.grid3d_edges(*dims)
    n = int(np.prod(dims))
    A = workloads.nodal_matrix(n, e, np.ones(e.shape[0]), np.full(n, workloads.GROUND_S))
    b = np.random.default_rng(0).standard_normal((1, n))
    label, iface, sides = workloads.separator_strips(dims, 14)
    assert iface.size == 900 and label.max() == 1
    W = vtm().vertex_admittance(A, label, iface, sides, "wob", 0.3)
    r = oracle.vtm_solve(oracle.tear_at_vertices(A, label, iface, sides, W.toarray()), A, b, 1e-8, max_sweeps=500)
    s = solver(A, label, iface, sides, W, check_every=1, adaptive_checks=False)
    x, rep = s.solve(to_dev(torch, b), 1e-8)
    assert r.status == "ok" and abs(rep.sweeps - r.sweeps) <= 1
    xs = spla.spsolve(A.tocsc(), b[0])
    assert np.abs(x.cpu().numpy()[0] - xs).max() <= 1e-6 * np.abs(xs).max()
    lam, _ = s.solve_adjoint(to_dev(torch, b), 1e-8)  # A is symmetric: A^-T b = A^-1 b
    assert np.abs(lam.cpu().numpy()[0] - xs).max() <= 1e-6 * np.abs(xs).max()
    s.close()
    b2 = np.concatenate([b, np.random.default_rng(1).standard_normal((1, n))])
    s = solver(A, label, iface, sides, W, nrhs_max=2)
    x2, _ = s.solve(to_dev(torch, b2), 1e-8)
    s.close()
    xs2 = oracle.direct_solve(A, b2)
    assert np.abs(x2.cpu().numpy() - xs2).max() <= 1e-6 * np.abs(xs2).max()


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_coupled_lines_graph_replay_matches_eager_bitwise(torch, prec):
    """Check intervals of a solve torn at interfacial nodes with coupled lines
    (b expanded to the twins, coupled waves after each full sweep, x the twins'
    mean) replayed as captured hipGraphs give bitwise the eager result, solve
    after solve."""
    A, b, label, iface, sides, W = coupled((24, 47), 10, "wob", 0.3, seed=9)
    common = dict(precision=prec, check_every=4, adaptive_checks=False)
    eager = solver(A, label, iface, sides, W, use_graph=False, **common)
    graph = solver(A, label, iface, sides, W, use_graph=True, **common)
    bd = to_dev(torch, b)
    xe, re = eager.solve(bd, 1e-10)
    for _ in range(3):
        xg, rg = graph.solve(bd, 1e-10)
        torch.cuda.synchronize()
        assert rg.sweeps == re.sweeps and rg.outer == re.outer
        assert torch.equal(xg, xe)
    assert re.relres_max <= 1e-10


def test_no_interfacial_nodes_and_zero_columns(torch):
    """Degenerate tears: with no interfacial node the circuit is one sub-circuit
    and one sweep is the direct solve; a zero right-hand side column converges
    at once with x = 0 beside a nonzero one."""
    A, b, label, iface, sides, W = strips((12, 13), 5, nrhs=2)
    one = np.zeros(A.shape[0], dtype=np.int32)
    s = solver(A, one, np.zeros(0, np.int32), np.zeros((0, 2), np.int32), 1.0, nrhs_max=2, check_every=1)
    x, rep = s.solve(to_dev(torch, b), 1e-12)
    assert rep.sweeps == 1
    xs = np.linalg.solve(A.toarray(), b.T).T
    assert np.abs(x.cpu().numpy() - xs).max() <= 1e-12 * np.abs(xs).max()
    b2 = b.copy()
    b2[1] = 0.0
    s = solver(A, label, iface, sides, W, nrhs_max=2, check_every=1)
    x, rep = s.solve(to_dev(torch, b2), 1e-10)
    xh = x.cpu().numpy()
    assert np.all(xh[1] == 0.0) and rep.relres[0] <= 1e-10
