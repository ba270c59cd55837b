"""Host side of tearing at interfacial nodes (vtm_split_vertex, no GPU): the
library's torn system equals the oracle's tear (Section V, Steps 2-3) node for
node, and the tearing errors are reported."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads
from paper_0910_0663_amd import binding


def oracle_in_library_order(A, label, iface, sides):
    """The oracle's torn matrix and sub-circuit labels, reordered to the
    library's node ids (inner and side-a twins keep the node id, node n + l is
    the side-b twin of iface[l])."""
    torn = oracle.tear_at_vertices(A, label, iface, sides, 1.0)
    n, L = A.shape[0], len(iface)
    is_if = np.zeros(n, dtype=bool)
    is_if[iface] = True
    inner = np.nonzero(~is_if)[0]
    pos = np.empty(n + L, dtype=np.int64)
    pos[inner] = torn.src[:, inner].tocsc().indices      # an inner node's source has one entry
    pos[np.asarray(iface)] = torn.pa
    pos[n + np.arange(L)] = torn.pb
    T = torn.T.tocsr()[pos][:, pos]
    return T, torn.block_of[pos], torn.src[pos]


def assert_same_split(A, label, iface, sides):
    M, part = binding.split_vertex(A, label, iface, sides)
    T, blk, src = oracle_in_library_order(A, label, iface, sides)
    assert M.shape == T.shape
    assert np.array_equal(part, blk)
    D = (M - T).tocoo()
    assert np.abs(D.data).max(initial=0.0) <= 1e-15 * np.abs(T.data).max()
    # the torn sources: b for inner nodes, b / 2 for each twin
    n, L = A.shape[0], len(iface)
    w = np.ones(n + L)
    w[np.asarray(iface)] = 0.5
    w[n:] = 0.5
    src_expected = sp.csr_matrix((w, (np.arange(n + L), np.concatenate([np.arange(n), iface]))),
                                 shape=(n + L, n))
    assert abs(src - src_expected).max() == 0.0


@pytest.fixture(scope="module")
def opamp(golden_dir):
    with open(os.path.join(golden_dir, "opamp_example.json")) as fh:
        return json.load(fh)


def test_split_of_the_opamp_example(opamp):
    """Section IX: nodes 2 and 3 of eq. (15) split into twins; an unsymmetric
    system whose controlled-source entries attach to the twin on the side of
    the controlling or controlled inner node."""
    A = sp.csr_matrix(np.array(opamp["A_eq15"], dtype=np.float64))
    assert_same_split(A, np.array([0, -1, -1, 1]), np.array([1, 2]), np.array([[0, 1], [0, 1]]))


@pytest.mark.parametrize("dims,width,law", [
    ((12, 23), 5, "loguniform"),       # 2-D strips, separators with interface-interface branches
    ((5, 6, 17), 4, "uniform"),        # 3-D slabs
])
def test_split_of_separator_strips(dims, width, law):
    rng = np.random.default_rng(3)
    edges = workloads.grid2d_edges(*dims) if len(dims) == 2 else workloads.grid3d_edges(*dims)
    g = 10.0 ** rng.uniform(-1, 1, edges.shape[0]) if law == "loguniform" else rng.uniform(0.5, 2, edges.shape[0])
    n = int(np.prod(dims))
    A = workloads.nodal_matrix(n, edges, g, np.full(n, workloads.GROUND_S))
    label, iface, sides = workloads.separator_strips(dims, width)
    assert_same_split(A, label, iface, sides)


def test_split_with_controlled_sources_and_reversed_sides():
    """Controlled sources inside strips and next to separators, and separator
    nodes listed with their two strips in either order."""
    w = workloads.make(3, dims=(4, 9, 14))   # unsymmetric 3-D circuit with controlled sources
    label, iface, sides = workloads.separator_strips(w.dims, 4)
    flip = np.arange(iface.size) % 3 == 1
    sides = np.where(flip[:, None], sides[:, ::-1], sides)
    assert_same_split(w.A, label, iface, sides)


def test_split_errors():
    A = workloads.make(1, dims=(6, 6)).A
    label, iface, sides = workloads.separator_strips((6, 6), 2)
    def status(*args):
        with pytest.raises(binding.VTMError) as ei:
            binding.split_vertex(A, *args)
        return ei.value.name
    # an inner node coupled to a strip it does not belong to
    bad = label.copy()
    bad[0] = 1
    assert status(bad, iface, sides) == "VTM_E_UNTEARABLE"
    # an interfacial node bordering strips that do not include a neighbour's
    s2 = sides.copy()
    s2[0] = [1, 2]
    assert status(label, iface, s2) == "VTM_E_UNTEARABLE"
    # repeated interfacial node, one-sided interfacial node
    assert status(label, np.concatenate([iface, iface[:1]]), np.concatenate([sides, sides[:1]])) == "VTM_E_ARG"
    s3 = sides.copy()
    s3[0] = [0, 0]
    assert status(label, iface, s3) == "VTM_E_ARG"
    # coupling across strips that bypasses the separator
    B = A.tolil()
    B[0, 5] = B[5, 0] = -0.5
    with pytest.raises(binding.VTMError) as ei:
        binding.split_vertex(B.tocsr(), label, iface, sides)
    assert ei.value.name == "VTM_E_UNTEARABLE"


def unit_grid(dims):
    e = workloads.grid2d_edges(*dims) if len(dims) == 2 else workloads.grid3d_edges(*dims)
    n = int(np.prod(dims))
    return workloads.nodal_matrix(n, e, np.ones(e.shape[0]), np.full(n, workloads.GROUND_S))


@pytest.mark.parametrize("side", [0, 1])
def test_vertex_admittance_rules_are_the_interface_block(side):
    """Section VIII rules 1-4 on tearing at interfacial nodes: C is the block of
    the oracle's torn matrix over one side's twins (C_1 or C_2)."""
    w = workloads.make(4, dims=(14, 23))
    label, iface, sides = workloads.separator_strips(w.dims, 5)
    torn = oracle.tear_at_vertices(w.A, label, iface, sides, 1.0)
    pos = torn.pa if side == 0 else torn.pb
    Cref = torn.T.tocsr()[pos][:, pos].toarray()
    assert np.count_nonzero(Cref - np.diag(np.diag(Cref))) > 0     # branches between interfacial nodes
    W = {r: binding.vertex_admittance(w.A, label, iface, sides, r, 0.3, side).toarray()
         for r in ("ob", "wob", "diag", "identity", "scaled_mean")}
    assert np.abs(W["ob"] - Cref).max() <= 1e-15 * np.abs(Cref).max()
    assert np.abs(W["wob"] - 0.3 * Cref).max() <= 1e-15 * np.abs(Cref).max()
    assert np.array_equal(W["diag"], np.diag(np.diag(W["ob"])))
    assert np.array_equal(W["identity"], 0.3 * np.eye(iface.size))
    assert np.allclose(W["scaled_mean"], 0.3 * np.mean(w.g) * np.eye(iface.size), rtol=1e-14, atol=0)
    with pytest.raises(binding.VTMError):
        binding.vertex_admittance(w.A, label, iface, sides, "ob", 1.0, 2)


def test_table2_ordering_of_preconditioners_on_a_grid2d_like_circuit():
    """Table II (Grid2d column), qualitatively: a 100 x 100 resistor grid torn
    into two sub-circuits at one separator column of 100 interfacial nodes.
    The diagonal preconditioner needs about twice the sweeps of the overlapped
    block (963 vs 491 in the paper), and a weighted overlapped block needs
    fewer still (296)."""
    dims = (100, 100)
    A = unit_grid(dims)
    b = np.random.default_rng(0).standard_normal((1, A.shape[0]))
    label, iface, sides = workloads.separator_strips(dims, 49)
    assert iface.size == 100 and label.max() == 1
    sweeps = {}
    for rule, alpha in (("diag", 1.0), ("ob", 1.0), ("wob", 0.3)):
        W = binding.vertex_admittance(A, label, iface, sides, rule, alpha).toarray()
        r = oracle.vtm_solve(oracle.tear_at_vertices(A, label, iface, sides, W), A, b, 1e-8, max_sweeps=5000)
        assert r.status == "ok"
        sweeps[rule] = r.sweeps
    assert sweeps["diag"] > sweeps["ob"] > sweeps["wob"]
    assert 1.5 <= sweeps["diag"] / sweeps["ob"] <= 2.5


# ----------------------------------------------------------- Schur complement approximation
def test_partial_schur_reduces_to_its_special_cases():
    """Rule 5 of Section VIII in the oracle: with every inner node kept it is
    the exact Schur complement of Example 3 (computed by interface_schur over
    the whole side), with none it is the interface block C, and a matched line
    W = S_1 makes T_1 = 0, so two sweeps of the sweep operator vanish and VTM
    converges in a few sweeps (Section VIII: one reflection)."""
    dims = (12, 25)
    A = unit_grid(dims)
    label, iface, sides = workloads.separator_strips(dims, 12)
    assert label.max() == 1
    torn = oracle.tear_at_vertices(A, label, iface, sides, 1.0)
    for side in (0, 1):
        S = oracle.interface_schur(torn, side)
        assert np.allclose(oracle.partial_schur(torn, side, None), 0.5 * (S + S.T), rtol=1e-12, atol=1e-14)
        P = torn.pa if side == 0 else torn.pb
        C = torn.T.tocsr()[P][:, P].toarray()
        assert np.array_equal(oracle.partial_schur(torn, side, 0), 0.5 * (C + C.T))
    W = oracle.partial_schur(torn, 0, None)
    matched = oracle.tear_at_vertices(A, label, iface, sides, W)
    M = oracle.sweep_operator(matched)
    assert np.abs(M @ M).max() < 1e-9 * np.abs(M).max()
    b = np.random.default_rng(2).standard_normal((1, A.shape[0]))
    r = oracle.vtm_solve(matched, A, b, 1e-10, max_sweeps=50)
    assert r.status == "ok" and r.sweeps <= 3


@pytest.mark.parametrize("side", [0, 1])
def test_partial_schur_at_depth_d_is_a_block_continued_fraction(side):
    """Rule 5 at the depths between none and all, by an independent route: on a
    unit grid torn at one column of nodes, the inner nodes within d hops of one
    side's twins are the d columns beside the separator, so C - E D~^-1 F is a
    block continued fraction over those columns, eliminated from the farthest
    inwards: Z = B_far, Z <- B - Z^-1 column by column (unit couplings between
    neighbouring columns and to the twins), and S~ = C - Z^-1.  Each B is the
    column's tridiagonal block of the untorn A."""
    ny, nx, s = 9, 17, 8
    A = unit_grid((ny, nx))
    label, iface, sides = workloads.separator_strips((ny, nx), s)
    assert np.array_equal(iface, np.arange(ny) * nx + s)
    torn = oracle.tear_at_vertices(A, label, iface, sides, 1.0)
    P = torn.pa if side == 0 else torn.pb
    C = torn.T.tocsr()[P][:, P].toarray()
    Ad = A.toarray()
    step = -1 if side == 0 else 1
    for d in (1, 2, 3, 5):
        cols = [np.arange(ny) * nx + s + step * h for h in range(1, d + 1)]
        Z = Ad[np.ix_(cols[-1], cols[-1])]
        for c in reversed(cols[:-1]):
            Z = Ad[np.ix_(c, c)] - np.linalg.inv(Z)
        S = C - np.linalg.inv(Z)
        assert np.allclose(oracle.partial_schur(torn, side, d), 0.5 * (S + S.T), rtol=1e-12, atol=1e-14), d


def test_partial_schur_drops_small_entries():
    dims = (10, 21)
    A = unit_grid(dims)
    label, iface, sides = workloads.separator_strips(dims, 10)
    torn = oracle.tear_at_vertices(A, label, iface, sides, 1.0)
    full = oracle.partial_schur(torn, 0, 3)
    kept = oracle.partial_schur(torn, 0, 3, drop=0.05)
    d = np.sqrt(np.diag(full))
    big = np.abs(full) >= 0.05 * np.outer(d, d)
    np.fill_diagonal(big, True)
    assert np.array_equal(kept, np.where(big, full, 0.0))
    assert 0 < np.count_nonzero(kept) < np.count_nonzero(full)


def test_table2_sca_beats_the_overlapped_block():
    """Table II, Grid2d column: the Schur complement approximation needs fewer
    sweeps than the overlapped block (275 vs 491), and more of the interior in
    D~ means fewer sweeps still (the exact complement needs a few)."""
    dims = (100, 100)
    A = unit_grid(dims)
    b = np.random.default_rng(0).standard_normal((1, A.shape[0]))
    label, iface, sides = workloads.separator_strips(dims, 49)
    torn = oracle.tear_at_vertices(A, label, iface, sides, 1.0)
    sweeps = []
    for depth in (0, 1, 2, 4):
        W = oracle.partial_schur(torn, 0, depth)
        r = oracle.vtm_solve(oracle.tear_at_vertices(A, label, iface, sides, W), A, b, 1e-8, max_sweeps=5000)
        assert r.status == "ok"
        sweeps.append(r.sweeps)
    assert sweeps == sorted(sweeps, reverse=True) and len(set(sweeps)) == 4


@pytest.mark.parametrize("dims,width,side,depth,drop", [
    ((14, 23), 5, 0, 1, 0.0),
    ((14, 23), 5, 1, 2, 0.0),
    ((14, 23), 5, 0, 3, 0.02),
    ((14, 23), 5, 1, None, 0.0),
    ((12, 12, 11), 5, 0, 2, 0.0),
    ((12, 12, 11), 5, 1, 3, 0.02),
])
def test_vertex_sca_equals_the_oracle(dims, width, side, depth, drop):
    """vtm_vertex_sca against the oracle's partial_schur: same entries (to
    rounding of the dense solves) and the same pattern after dropping."""
    if len(dims) == 2:
        A = workloads.make(4, dims=dims).A
    else:
        e = workloads.grid3d_edges(*dims)
        n = int(np.prod(dims))
        A = workloads.nodal_matrix(n, e, np.random.default_rng(1).uniform(0.5, 2, e.shape[0]), np.full(n, 0.01))
    label, iface, sides = workloads.separator_strips(dims, width)
    torn = oracle.tear_at_vertices(A, label, iface, sides, 1.0)
    Wo = oracle.partial_schur(torn, side, depth, drop)
    Wl = binding.vertex_sca(A, label, iface, sides, side, depth, drop).toarray()
    assert np.array_equal(Wo != 0, Wl != 0)
    assert np.abs(Wo - Wl).max() <= 1e-13 * np.abs(Wo).max()
    with pytest.raises(binding.VTMError):
        binding.vertex_sca(A, label, iface, sides, side, depth, -1.0)
