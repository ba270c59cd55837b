"""Parity of the HIP path (called through the C ABI) with the CPU oracle.

Tolerances (FP64 path): iterates are compared element by element after the
same number of sweeps.  Each sweep rounds a dense dot product of at most n_s
terms (relative error <= n_s * 2^-53 ~ 3e-14 for n_s = 256) and the iteration
contracts errors by rho < 1 per sweep, so the accumulated difference stays
below n_s * 2^-53 / (1 - rho); with rho <= 0.99 that is <= 3e-12.  The tests
use 1e-11 relative to max |x|.
"""
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


def oracle_iterates(w, ks, b=None, transpose=False):
    A = w.A.T.tocsr() if transpose else w.A
    torn = oracle.tear_wires(A, w.part, w.Z)
    sw = oracle.Sweeper(torn)
    b = w.b if b is None else b
    f = torn.src @ b.T
    a = np.zeros((2, torn.n_lines, b.shape[0]))
    out = {}
    for k in range(1, max(ks) + 1):
        u, a = sw.sweep(f, a)
        if k in ks:
            out[k] = (torn.out @ u).T
    return out


def gpu_iterate(torch, w, k, b=None, adjoint=False, nrhs_max=None, check_every=1, **kw):
    """x^k of the HIP path: max_sweeps = k with an unreachable tolerance.  With
    check_every = k the sweeps between the first and the last are port-to-port."""
    b = w.b if b is None else b
    s = vtm().Solver(w.A, w.part, w.Z, nrhs_max=nrhs_max or b.shape[0], check_every=check_every, max_sweeps=k,
                     adaptive_checks=False, **kw)
    x = torch.empty((b.shape[0], w.n), dtype=torch.float64, device="cuda")
    fn = s.solve_adjoint if adjoint else s.solve
    with pytest.raises(vtm().VTMError) as ei:
        fn(to_dev(torch, b), 1e-300, x)
    assert ei.value.name == "VTM_E_MAXITER"
    assert ei.value.report.sweeps == k
    s.close()
    return x.cpu().numpy()


def assert_close(x, ref, rtol=ITER_RTOL):
    scale = np.abs(ref).max()
    err = np.abs(x - ref).max()
    assert err <= rtol * scale, f"max err {err:.3e} vs scale {scale:.3e}"


@pytest.mark.parametrize("cfg,kw", [
    (1, dict()),
    (3, dict(dims=(16, 16, 16))),
    (4, dict(dims=(64, 64), nrhs=3)),
    (2, dict(dims=(64, 64))),
])
def test_iterates_match_oracle(torch, cfg, kw):
    """x^k of the GPU equals the oracle's x^k element by element (several tiles,
    uneven sub-circuits, an unsymmetric circuit, several right-hand sides)."""
    w = workloads.make(cfg, **kw)
    ks = [1, 2, 7, 40]
    ref = oracle_iterates(w, ks)
    for k in ks:
        assert_close(gpu_iterate(torch, w, k), ref[k])


@pytest.mark.parametrize("cfg,kw,prec", [
    (1, dict(), "fp64"),
    (2, dict(dims=(64, 64)), "fp64"),
    (3, dict(dims=(16, 16, 16)), "fp64"),
    (4, dict(dims=(64, 64)), "fp64"),
])
def test_port_to_port_iterates_match_oracle(torch, cfg, kw, prec):
    """Sweeps that stream only the port-to-port operator (Appendix, eqs. 23-26)
    give the oracle's iterates: x^k after a first full sweep, k - 2 port-to-port
    sweeps and a last full sweep."""
    w = workloads.make(cfg, **kw)
    ks = [2, 9, 40]
    ref = oracle_iterates(w, ks)
    for k in ks:
        for form in ("port", "port_dense"):
            assert_close(gpu_iterate(torch, w, k, check_every=k, local_form=form), ref[k])


@pytest.mark.parametrize("dims,block", [((72, 72), (9, 9)), ((96, 96), (12, 12)), ((100, 100), (16, 16))])
def test_packed_split_sweep_iterates_match_oracle(torch, dims, block):
    """Sub-circuits with 32 to 64 port nodes (9x9, 12x12, 16x16 blocks, the last
    grid with ragged edge blocks) take the packed sweep with one wavefront per
    diagonal chunk; some chunks lie past a sub-circuit's last diagonal.  The
    iterates equal the oracle's."""
    w = workloads.make(2, dims=dims, block=block)
    ks = [2, 9]
    ref = oracle_iterates(w, ks)
    for k in ks:
        assert_close(gpu_iterate(torch, w, k, check_every=k, local_form="port"), ref[k])


def test_port_to_port_and_full_forms_agree(torch):
    """The local forms (full inverse, packed symmetric port-node operator, dense
    port operator) reach the tolerance after the same sweeps and agree."""
    w = workloads.make(2, dims=(256, 256))
    xs = []
    for form in ("full", "port", "port_dense"):
        s = vtm().Solver(w.A, w.part, w.Z, check_every=8, adaptive_checks=False, local_form=form, timing=True)
        x, rep = s.solve(to_dev(torch, w.b), w.tol)
        xs.append((x.cpu().numpy(), rep, s.port_operator_bytes))
    (xf, rf, bf), (xp, rp, bp), (xd, rd, bd) = xs
    assert rf.sweeps == rp.sweeps == rd.sweeps
    assert rp.pp_launches > 0 and rd.pp_launches > 0 and rf.pp_launches == 0
    # 8 x 8 blocks: 28 port nodes (406 packed entries) against 32 ports (1024)
    assert bf == 0 and bp < bd / 2
    assert_close(xp, xf)
    assert_close(xd, xf)


def _with_isolated_component(nrhs):
    """A 32x32 grid cut into 4x4 sub-circuits of 8x8, plus a separate 8x8 grid
    that forms one sub-circuit with no cut wire (k = q = 0 ports), 17 sub-circuits
    in all (an odd count leaves the last pair of the packed sweep half empty)."""
    import types
    rng = np.random.default_rng(11)
    e1 = workloads.grid2d_edges(32, 32)
    e2 = workloads.grid2d_edges(8, 8) + 32 * 32
    edges = np.concatenate([e1, e2])
    n = 32 * 32 + 64
    g = rng.uniform(0.5, 2.0, size=edges.shape[0])
    A = workloads.nodal_matrix(n, edges, g, np.full(n, workloads.GROUND_S))
    part = np.concatenate([workloads.block_partition_2d(32, 32, 8, 8), np.full(64, 16)]).astype(np.int32)
    b = rng.standard_normal((nrhs, n))
    return types.SimpleNamespace(A=A, b=b, part=part, Z=1.0 / g.mean(), n=n, tol=1e-10)


@pytest.mark.parametrize("nrhs", [1, 20])
def test_sub_circuit_without_ports_in_every_form(torch, nrhs):
    """A sub-circuit with no cut wire next to ordinary ones: every local form
    (packed, port-node, port operator, full; MFMA tiles for 20 right-hand sides)
    gives the oracle's iterates, and the solve reaches its tolerance."""
    w = _with_isolated_component(nrhs)
    ks = [1, 2, 7]
    ref = oracle_iterates(w, ks)
    for form in ("port", "port_dense", "full"):
        for k in ks:
            assert_close(gpu_iterate(torch, w, k, check_every=k, local_form=form), ref[k])
    s = vtm().Solver(w.A, w.part, w.Z, nrhs_max=nrhs)
    x, rep = s.solve(to_dev(torch, w.b), w.tol)
    assert oracle.relative_residual(w.A, w.b, x.cpu().numpy()).max() <= w.tol
    s.close()


def _strong_one_sided_couplings(w, scale, seed):
    """w with one-sided entries larger than the diagonal added inside its
    sub-circuits (controlled sources of large gain), so that the elimination of
    every local matrix has to pivot."""
    rng = np.random.default_rng(seed)
    A = w.A.tolil()
    d = w.A.diagonal()
    for s_ in range(w.n_sub):
        nodes = np.nonzero(w.part == s_)[0]
        for i in rng.choice(nodes, size=len(nodes) // 2, replace=False):
            j = rng.choice(nodes[nodes != i])
            A[i, j] = A[i, j] + scale * d[i] * rng.choice([-1.0, 1.0])
    w.A = A.tocsr()
    return w


@pytest.mark.parametrize("kind", ["pivoting 64-node", "ragged 63-node", "pivoting 125-node panels"])
def test_register_setup_iterates_match_oracle(torch, kind):
    """Sub-circuits of up to 64 nodes are inverted by one wavefront each: with
    one-sided entries larger than the diagonal (every elimination pivots) on
    4x4x4 blocks, and on 7x9 blocks (63 nodes, a ragged register row), the first
    iterates in the full and port-to-port forms equal the oracle's (exact local
    solves by sparse LU).  The same pivoting on 256 blocks of 5x5x5 exercises the
    panel elimination with a row per thread (panels of 32 columns, the last one
    29 wide)."""
    if kind == "pivoting 64-node":
        w = _strong_one_sided_couplings(workloads.make(3, dims=(8, 8, 8), block=(4, 4, 4)), 3.0, 4)
        assert np.bincount(w.part).max() == 64
    elif kind.startswith("pivoting 125"):
        w = _strong_one_sided_couplings(workloads.make(3, dims=(40, 40, 20), block=(5, 5, 5)), 3.0, 5)
        assert w.n_sub == 256 and np.bincount(w.part).min() == 125
    else:
        w = workloads.make(1, dims=(63, 63), block=(7, 9))
        assert np.bincount(w.part).max() == 63
    ks = [1, 3]
    ref = oracle_iterates(w, ks)
    for k in ks:
        assert_close(gpu_iterate(torch, w, k, local_form="full"), ref[k])
        assert_close(gpu_iterate(torch, w, k, check_every=k), ref[k])


def test_singular_sub_circuit_is_reported(torch):
    """A node with no branch and no ground, alone in its sub-circuit, makes that
    sub-circuit's matrix singular: setup fails with VTM_E_SINGULAR, for FP64 and
    for the batched (MFMA tile) setup alike."""
    base = workloads.make(1, dims=(16, 16), block=(8, 8))
    n = base.n + 1
    A = sp.bmat([[base.A, None], [None, sp.csr_matrix((1, 1))]], format="csr")
    part = np.concatenate([base.part, [base.n_sub]]).astype(np.int32)
    for kw in (dict(), dict(nrhs_max=16), dict(precision="fp32_refine")):
        with pytest.raises(vtm().VTMError) as ei:
            vtm().Solver(A, part, base.Z, **kw)
        assert ei.value.name == "VTM_E_SINGULAR", kw
    assert n == A.shape[0]


@pytest.mark.parametrize("kw", [dict(), dict(nrhs=16)])
def test_largest_sub_circuits(torch, kw):
    """Two sub-circuits of 8,192 nodes (inverted in blocked global-memory
    Gauss-Jordan with 64-column panels; the full sweep stages 128 KiB of LDS):
    iterates equal the oracle's in the port (128 ports each, dense operator)
    and full forms; with 16 right-hand sides the FP64 handle keeps the
    column-group layout because an 8,192-row block does not fit the batched
    sweep's LDS staging."""
    w = workloads.make(1, dims=(128, 128), block=(128, 64), **kw)
    assert w.n_sub == 2 and np.bincount(w.part).max() == 8192
    ks = [3]
    ref = oracle_iterates(w, ks)
    for form in ("port", "full"):
        for k in ks:
            assert_close(gpu_iterate(torch, w, k, check_every=k, local_form=form), ref[k])


def test_sub_circuits_at_the_size_limit(torch):
    """Two sub-circuits of 16,384 nodes, the planner's limit: each FP64 inverse
    is exactly 2^31 bytes, the largest range the setup's buffer loads and stores
    address (an offset of 2^31 marks a masked lane), inverted with 64-column
    panels whose pivot steps are launches of their own.  The solve (port-to-port,
    128 ports each) reaches the sparse LU's solution, and so do two right-hand
    sides at once (full sweeps, one column a workgroup, x read back from HBM for
    the waves: the right-hand side alone fills 128 KiB of LDS)."""
    w = workloads.make(1, dims=(128, 256), block=(128, 128), nrhs=2)
    assert w.n_sub == 2 and np.bincount(w.part).max() == 16384
    xs = oracle.direct_solve(w.A, w.b)
    s = vtm().Solver(w.A, w.part, w.Z)
    x, rep = s.solve(to_dev(torch, w.b[:1]), 1e-10)
    s.close()
    assert oracle.relative_residual(w.A, w.b[:1], x.cpu().numpy()).max() <= 1e-10
    assert np.abs(x.cpu().numpy()[0] - xs[0]).max() <= 1e-6 * np.abs(xs[0]).max()
    s = vtm().Solver(w.A, w.part, w.Z, nrhs_max=2)
    x, rep = s.solve(to_dev(torch, w.b), 1e-10)
    s.close()
    assert oracle.relative_residual(w.A, w.b, x.cpu().numpy()).max() <= 1e-10
    assert np.abs(x.cpu().numpy() - xs).max() <= 1e-6 * np.abs(xs).max()


def test_large_unsymmetric_sub_circuits_several_rhs_and_adjoint(torch):
    """An unsymmetric circuit (controlled sources) in two 13,824-node blocks,
    above the 10,240 nodes whose x fits LDS beside the right-hand side: two
    right-hand sides and the adjoint (the stored inverses read transposed) reach
    the sparse LU's solutions of A x = b and A^T lambda = g."""
    w = workloads.make(3, dims=(24, 24, 48), block=(24, 24, 24), nrhs=2)
    assert w.n_sub == 2 and np.bincount(w.part).min() > 10240
    s = vtm().Solver(w.A, w.part, w.Z, nrhs_max=2)
    x, rep = s.solve(to_dev(torch, w.b), 1e-10)
    xs = oracle.direct_solve(w.A, w.b)
    assert oracle.relative_residual(w.A, w.b, x.cpu().numpy()).max() <= 1e-10
    assert np.abs(x.cpu().numpy() - xs).max() <= 1e-6 * np.abs(xs).max()
    g = np.random.default_rng(11).standard_normal((1, w.n))
    lam, rep = s.solve_adjoint(to_dev(torch, g), 1e-10)
    s.close()
    lam_ref = oracle.direct_adjoint(w.A, g)
    assert oracle.relative_residual(w.A.T.tocsr(), g, lam.cpu().numpy()).max() <= 1e-10
    assert np.abs(lam.cpu().numpy() - lam_ref).max() <= 1e-6 * np.abs(lam_ref).max()


@pytest.mark.parametrize("cfg,kw,rule,alpha", [
    (1, dict(), "ob", 1.0),                        # packed sweep with a different W per port
    (1, dict(), "wob", 0.125),
    (3, dict(dims=(16, 16, 16)), "wob", 0.25),     # port-node form, controlled sources
    (4, dict(dims=(64, 64), nrhs=20), "wob", 0.25),  # MFMA tiles
])
def test_per_wire_admittance_iterates_match_oracle(torch, cfg, kw, rule, alpha):
    """Lines of different admittance (Section VIII's overlapped-block rules,
    one W per wire from vtm_line_admittance): iterates equal the oracle's in the
    port-to-port and full forms."""
    w = workloads.make(cfg, **kw)
    w.Z = 1.0 / vtm().line_admittance(w.A, w.part, rule, alpha)
    ks = [1, 5, 20]
    ref = oracle_iterates(w, ks)
    for form in ("port", "full"):
        for k in ks:
            assert_close(gpu_iterate(torch, w, k, check_every=k, local_form=form), ref[k])


def test_timing_modes_count_every_launch(torch):
    """Per-launch events (timing 1) and one event pair per run of port-to-port
    sweeps (timing 2) count the same launches: the first and the rebuilding
    full sweep, and every other sweep as port-to-port; both give the same x."""
    w = workloads.make(2, dims=(256, 256))
    xs = []
    for mode in (1, 2):
        s = vtm().Solver(w.A, w.part, w.Z, check_every=8, timing=mode)
        x, rep = s.solve(to_dev(torch, w.b), w.tol)
        assert rep.sweep_launches == 2 and rep.pp_launches == rep.sweeps - 1, (mode, rep)
        assert rep.pp_kernel_ms > 0 and rep.sweep_kernel_ms > 0
        xs.append(x.cpu().numpy())
        s.close()
    assert np.array_equal(xs[0], xs[1])


def test_64sq_grid_sweeps_and_solution(torch):
    """64x64 grid, 4x4 sub-circuits of 16x16, tol 1e-10, residual checked every
    sweep: the same sweep count as the oracle (within one for rounding at the
    threshold), the same iterate, and the fixed point of the direct solve."""
    w = workloads.make(1)
    r = oracle.vtm_solve(oracle.tear_wires(w.A, w.part, w.Z), w.A, w.b, w.tol)
    s = vtm().Solver(w.A, w.part, w.Z, check_every=1, adaptive_checks=False)
    x, rep = s.solve(to_dev(torch, w.b), w.tol)
    assert abs(rep.sweeps - r.sweeps) <= 1
    ref = oracle_iterates(w, [rep.sweeps])[rep.sweeps]
    assert_close(x.cpu().numpy(), ref)
    assert oracle.relative_residual(w.A, w.b, x.cpu().numpy()).max() <= w.tol
    xs = oracle.direct_solve(w.A, w.b)
    assert np.abs(x.cpu().numpy() - xs).max() <= 1e-8 * np.abs(xs).max()


@pytest.mark.parametrize("adaptive", [False, True])
def test_log_uniform_grid_of_8x8_blocks_scaled_down(torch, adaptive):
    """The 8x8-sub-circuit, log-uniform-conductance workload at 256x256 with a
    check every 8 sweeps (and with checks thinned out far from the tolerance):
    the GPU stops within [oracle, oracle + 7] sweeps and its iterate matches the
    oracle's at that count."""
    w = workloads.make(2, dims=(256, 256))
    r = oracle.vtm_solve(oracle.tear_wires(w.A, w.part, w.Z), w.A, w.b, w.tol)
    s = vtm().Solver(w.A, w.part, w.Z, check_every=8, adaptive_checks=adaptive)
    x, rep = s.solve(to_dev(torch, w.b), w.tol)
    assert r.sweeps <= rep.sweeps <= r.sweeps + 7
    ref = oracle_iterates(w, [rep.sweeps])[rep.sweeps]
    assert_close(x.cpu().numpy(), ref)


def test_zero_rhs_and_single_subcircuit(torch):
    w = workloads.make(1, dims=(32, 32))
    s = vtm().Solver(w.A, w.part, w.Z)
    x, rep = s.solve(torch.zeros((1, w.n), dtype=torch.float64, device="cuda"), 1e-10)
    assert rep.sweeps == 0 and not x.any().item()
    one = vtm().Solver(w.A, np.zeros(w.n, np.int32), 1.0, check_every=1)
    assert one.n_wires == 0
    x1, rep1 = one.solve(to_dev(torch, w.b), 1e-13)
    assert rep1.sweeps == 1
    assert_close(x1.cpu().numpy(), np.linalg.solve(w.A.toarray(), w.b.ravel())[None], rtol=1e-12)


def test_maxiter_divergence_and_arguments(torch):
    V = vtm()
    w = workloads.make(1, dims=(32, 32))
    s = V.Solver(w.A, w.part, w.Z, check_every=4, max_sweeps=10)
    with pytest.raises(V.VTMError) as ei:
        s.solve(to_dev(torch, w.b), 1e-12)
    assert ei.value.name == "VTM_E_MAXITER" and ei.value.report.sweeps == 10
    # divergence forced from the host: any residual above 1e-3 counts as diverged,
    # and the first iterate's residual is far above that
    d = V.Solver(w.A, w.part, w.Z, check_every=1, divergence=1e-3)
    with pytest.raises(V.VTMError) as ei:
        d.solve(to_dev(torch, w.b), 1e-12)
    assert ei.value.name == "VTM_E_DIVERGED" and ei.value.report.sweeps == 1
    with pytest.raises(V.VTMError) as ei:
        s.solve(to_dev(torch, np.ones((2, w.n))), 1e-8)   # nrhs above nrhs_max
    assert ei.value.name == "VTM_E_ARG"
    A = w.A.tolil()
    A[0, 900] = 0.2
    with pytest.raises(V.VTMError) as ei:
        V.Solver(A.tocsr(), w.part, w.Z)
    assert ei.value.name == "VTM_E_UNTEARABLE"


def test_resume_from_waves_is_bitwise_continuation(torch):
    """The iteration state is the wave vector: stopping after 24 sweeps,
    exporting and re-importing the waves, and continuing gives bitwise the same
    iterate as an uninterrupted run (full local form throughout: a resumed solve
    has no zero-wave first sweep to take the port-to-port source term from)."""
    V = vtm()
    w = workloads.make(1)
    b = to_dev(torch, w.b)
    kw = dict(check_every=8, adaptive_checks=False, local_form="full")
    full = V.Solver(w.A, w.part, w.Z, **kw)
    x_full, rep_full = full.solve(b, w.tol)
    part = V.Solver(w.A, w.part, w.Z, max_sweeps=24, **kw)
    x_tmp = torch.empty_like(b)
    with pytest.raises(V.VTMError):
        part.solve(b, w.tol, x_tmp)
    waves = part.get_waves()
    cont = V.Solver(w.A, w.part, w.Z, **kw)
    cont.set_waves(waves)
    x_cont, rep_cont = cont.solve(b, w.tol)
    assert rep_cont.sweeps + 24 == rep_full.sweeps
    assert torch.equal(x_cont, x_full)
    # a refining handle has no wave checkpoint (its state is x with an inner solve's waves)
    r = V.Solver(w.A, w.part, w.Z, precision="fp32_refine")
    r.solve(b, w.tol)
    for call in (r.get_waves, lambda: r.set_waves(waves)):
        with pytest.raises(V.VTMError) as ei:
            call()
        assert ei.value.name == "VTM_E_UNSUPPORTED"
    r.close()


def test_repeat_runs_are_bitwise_identical(torch):
    V = vtm()
    w = workloads.make(4, dims=(96, 96), nrhs=2)
    s = V.Solver(w.A, w.part, w.Z, nrhs_max=2)
    b = to_dev(torch, w.b)
    x1, r1 = s.solve(b, 1e-9)
    x2, r2 = s.solve(b, 1e-9)
    assert r1.sweeps == r2.sweeps and torch.equal(x1, x2)


def test_adjoint_matches_oracle_on_unsymmetric_circuit(torch):
    """VTM on A^T with the stored inverses read transposed: iterates equal the
    oracle's VTM on the torn A^T, and the converged result is A^-T g."""
    w = workloads.make(3, dims=(16, 16, 16))
    g = np.random.default_rng(5).standard_normal((1, w.n))
    ks = [1, 3, 25]
    ref = oracle_iterates(w, ks, b=g, transpose=True)
    for k in ks:
        # port-node sweeps on the transposed operator, checked every sweep or only at k; full sweeps
        assert_close(gpu_iterate(torch, w, k, b=g, adjoint=True), ref[k])
        assert_close(gpu_iterate(torch, w, k, b=g, adjoint=True, check_every=k), ref[k])
        assert_close(gpu_iterate(torch, w, k, b=g, adjoint=True, local_form="full"), ref[k])
    s = vtm().Solver(w.A, w.part, w.Z)
    lam, rep = s.solve_adjoint(to_dev(torch, g), 1e-11)
    lam_ref = oracle.direct_adjoint(w.A, g)
    assert np.abs(lam.cpu().numpy() - lam_ref).max() <= 1e-8 * np.abs(lam_ref).max()


@pytest.mark.parametrize("cfg,dims", [(3, (16, 16, 32)), (5, (128, 128))])
def test_fp32_refinement_reaches_fp64_tolerance(torch, cfg, dims):
    """FP32 inverses and sweeps inside FP64 refinement reach relative residual
    1e-8 (recomputed here in FP64 on the host) and the direct solution within
    the conditioning bound of that residual."""
    w = workloads.make(cfg, dims=dims)
    s = vtm().Solver(w.A, w.part, w.Z, precision="fp32_refine")
    x, rep = s.solve(to_dev(torch, w.b), w.tol)
    xh = x.cpu().numpy()
    assert oracle.relative_residual(w.A, w.b, xh).max() <= w.tol
    assert rep.outer >= 1
    xs = oracle.direct_solve(w.A, w.b)
    assert np.abs(xh - xs).max() <= 2e-6 * np.abs(xs).max()
    # a column count that is not a multiple of four (the staging's scalar path)
    x6, rep6 = s.solve(to_dev(torch, w.b[:6]), w.tol)
    assert oracle.relative_residual(w.A, w.b[:6], x6.cpu().numpy()).max() <= w.tol


@pytest.mark.parametrize("form", ["port", "port_dense", "full"])
def test_fp32_refinement_with_timing_in_every_local_form(torch, form):
    """Timed FP32 refinement (per-launch events on every sweep, including the
    full sweep that rebuilds each correction) reaches the FP64 tolerance in
    every local form and reports its port-to-port launches."""
    w = workloads.make(5, dims=(128, 128))
    s = vtm().Solver(w.A, w.part, w.Z, precision="fp32_refine", local_form=form, timing=True)
    x, rep = s.solve(to_dev(torch, w.b), w.tol)
    assert oracle.relative_residual(w.A, w.b, x.cpu().numpy()).max() <= w.tol
    assert rep.outer >= 1 and rep.sweep_launches >= 1
    assert (rep.pp_launches > 0) == (form != "full")
    s.close()


def test_gradient_through_autograd_matches_oracle(torch):
    """dL/db and dL/dg for L = sum over probes of x^2 through VTMSolve, against the
    oracle's adjoint formula with direct solves."""
    from paper_0910_0663_amd import Circuit, VTMSolve
    w = workloads.make(5, dims=(64, 64), n_probes=256)
    circ = Circuit(w.n, w.edges, w.ground, w.part, w.Z, tol=1e-10, precision="fp64")
    g = torch.tensor(w.g, dtype=torch.float64, device="cuda", requires_grad=True)
    b = torch.tensor(w.b[0], dtype=torch.float64, device="cuda", requires_grad=True)
    x = VTMSolve.apply(b, g, circ)
    probes = torch.as_tensor(w.probes, device="cuda")
    loss = (x[probes] ** 2).sum()
    loss.backward()
    xs = oracle.direct_solve(w.A, w.b)
    dLdx = np.zeros_like(xs)
    dLdx[:, w.probes] = 2 * xs[:, w.probes]
    lam = oracle.direct_adjoint(w.A, dLdx)
    gref = oracle.branch_gradient(w.edges, xs, lam)
    assert np.abs(b.grad.cpu().numpy() - lam[0]).max() <= 1e-7 * np.abs(lam).max()
    assert np.abs(g.grad.cpu().numpy() - gref).max() <= 1e-7 * np.abs(gref).max()


def test_full_size_2048sq_residual(torch):
    """The bench workload at full size (2048^2 nodes, 65,536 sub-circuits of 8x8,
    check every 8 sweeps): the returned x meets the FP64 relative residual 1e-8
    recomputed on the host from the untorn A."""
    w = workloads.make(2)
    s = vtm().Solver(w.A, w.part, w.Z, check_every=8)
    x, rep = s.solve(to_dev(torch, w.b), w.tol)
    assert rep.checks < 40
    print(f"full-size sweeps {rep.sweeps} relres {rep.relres_max:.3e} solve_ms {rep.solve_ms:.1f}", flush=True)
    rel = oracle.relative_residual(w.A, w.b, x.cpu().numpy()).max()
    assert rel <= w.tol
    assert abs(rel - rep.relres_max) <= 1e-3 * rel


def test_full_size_1024sq_64rhs_bf16_refinement_residual(torch):
    """The batched bench workload at full size (1024^2 nodes, 4,290 uneven
    sub-circuits, 64 right-hand sides): BF16 sweeps on the matrix cores inside
    FP64 refinement give every column relative residual <= 1e-8, recomputed on the
    host from the untorn A."""
    w = workloads.make(4)
    s = vtm().Solver(w.A, w.part, w.Z, precision="bf16_refine", nrhs_max=w.nrhs)
    x, rep = s.solve(to_dev(torch, w.b), w.tol)
    print(f"full-size bf16: sweeps {rep.sweeps} outer {rep.outer} relres {rep.relres_max:.3e}", flush=True)
    rel = oracle.relative_residual(w.A, w.b, x.cpu().numpy())
    assert rel.shape == (64,) and rel.max() <= w.tol
    assert 2 <= rep.outer <= 8, rep.outer   # see test_batched_bf16_refinement_reaches_fp64_tolerance


def test_full_size_128cube_fp32_refinement_residual(torch):
    """The unsymmetric bench workload at full size (128^3 nodes with 124,846
    controlled sources, 4,096 sub-circuits of 8^3): FP32 sweeps inside FP64
    refinement reach relative residual 1e-8, recomputed on the host."""
    w = workloads.make(3)
    s = vtm().Solver(w.A, w.part, w.Z, precision="fp32_refine")
    x, rep = s.solve(to_dev(torch, w.b), w.tol)
    print(f"full-size fp32 3-D: sweeps {rep.sweeps} outer {rep.outer} relres {rep.relres_max:.3e}", flush=True)
    assert oracle.relative_residual(w.A, w.b, x.cpu().numpy()).max() <= w.tol
    assert rep.outer >= 1


def test_full_size_512sq_gradient_matches_oracle(torch):
    """The gradient bench workload at full size (512^2 grid, 4,096 probes, 523,264
    branches; FP32 sweeps with FP64 refinement to 1e-8): dL/dg of every branch
    against the oracle's adjoint formula with direct solves (whose formula a CPU
    test pins by central differences).  The bound allows the solves' own error
    (kappa(A) times the tolerance)."""
    from paper_0910_0663_amd import Circuit, VTMSolve
    w = workloads.make(5)
    circ = Circuit(w.n, w.edges, w.ground, w.part, w.Z, tol=w.tol, precision="fp32_refine")
    g = torch.tensor(w.g, dtype=torch.float64, device="cuda", requires_grad=True)
    b = torch.tensor(w.b[0], dtype=torch.float64, device="cuda")
    x = VTMSolve.apply(b, g, circ)
    probes = torch.as_tensor(w.probes, device="cuda")
    (x[probes] ** 2).sum().backward()
    xs = oracle.direct_solve(w.A, w.b)
    dLdx = np.zeros_like(xs)
    dLdx[:, w.probes] = 2 * xs[:, w.probes]
    gref = oracle.branch_gradient(w.edges, xs, oracle.direct_adjoint(w.A, dLdx))
    assert g.grad.shape[0] == len(w.edges) == 523264
    assert np.abs(g.grad.cpu().numpy() - gref).max() <= 1e-4 * np.abs(gref).max()


@pytest.mark.parametrize("cfg,centres,R,k,kw", [
    # the bench workload: corner, edge and interior sub-circuits; one full sweep,
    # port-to-port sweeps on the packed symmetric operator, one full sweep
    (2, [0, 128, 256 * 128 + 128, 65535], 8, 9, dict()),
    # 128^3 with controlled sources (unsymmetric): dense port-to-port operators
    # between 384 ports of 8^3 sub-circuits; corner, interior and far corner
    (3, [0, 8 * 256 + 8 * 16 + 8, 4095], 2, 3, dict(precision="fp64")),
    # 64 right-hand sides on uneven sub-circuits: FP64 inverses as MFMA tiles
    (4, [0, "mid", -1], 3, 4, dict(nrhs_max=64)),
])
def test_full_size_sampled_iterates_match_windowed_oracle(torch, cfg, centres, R, k, kw):
    """At full size, x^k on sampled sub-circuits equals the oracle's, run on the
    window of sub-circuits within R >= k - 1 hops of each sample (exact for
    k <= R + 1: the oracle side is pinned against the whole-problem oracle on
    smaller grids)."""
    from oracle_window import window_iterate
    w = workloads.make(cfg)
    print(f"{w.name}: n={w.n} subs={w.n_sub} nrhs={w.nrhs} k={k}", flush=True)
    x = gpu_iterate(torch, w, k, check_every=k, **kw)
    for c in centres:
        c = w.n_sub // 2 if c == "mid" else c % w.n_sub
        nodes = np.nonzero(w.part == c)[0]
        assert_close(x[:, nodes], window_iterate(w, c, R, k))


# ----------------------------------------------------------------------------- batched (MFMA) forms
def test_batched_fp64_mfma_iterates_match_oracle(torch):
    """FP64 handles sized for 16+ right-hand sides store the inverses as MFMA
    tiles (v_mfma_f64_16x16x4f64); their iterates equal the oracle's, on uneven
    sub-circuits padded to the tile size, including a ragged last block of
    right-hand sides and a single right-hand side."""
    w = workloads.make(4, dims=(96, 96), nrhs=20)
    ks = [1, 3, 17]
    ref = oracle_iterates(w, ks)
    for k in ks:
        assert_close(gpu_iterate(torch, w, k, nrhs_max=20), ref[k])
    w1 = workloads.make(4, dims=(96, 96), nrhs=1)
    ref1 = oracle_iterates(w1, [5])
    assert_close(gpu_iterate(torch, w1, 5, nrhs_max=16), ref1[5])
    # checks every 8 sweeps: sweeps in between store x on port rows only
    s = vtm().Solver(w.A, w.part, w.Z, nrhs_max=20, check_every=8, adaptive_checks=False)
    x, rep = s.solve(to_dev(torch, w.b), 1e-9)
    assert rep.sweeps % 8 == 0
    assert_close(x.cpu().numpy(), oracle_iterates(w, [rep.sweeps])[rep.sweeps])


def test_batched_ragged_tiles_match_oracle(torch):
    """A node count and a column count that are not multiples of the 64 x 64 tiles
    of the renumbering transposes (8,100 nodes, 17 right-hand sides): the iterates
    still equal the oracle's."""
    w = workloads.make(4, dims=(90, 90), nrhs=17)
    assert w.A.shape[0] % 64 != 0
    ref = oracle_iterates(w, [4])
    assert_close(gpu_iterate(torch, w, 4, nrhs_max=17), ref[4])


def test_batched_bf16_refinement_reaches_fp64_tolerance(torch):
    """BF16 inverses x BF16 right-hand sides on MFMA with FP32 accumulation,
    inside FP64 refinement: every column reaches relative residual 1e-8
    (recomputed in FP64 on the host) and the direct solution."""
    w = workloads.make(4, dims=(192, 192), nrhs=32)
    s = vtm().Solver(w.A, w.part, w.Z, precision="bf16_refine", nrhs_max=32)
    x, rep = s.solve(to_dev(torch, w.b), w.tol)
    xh = x.cpu().numpy()
    assert oracle.relative_residual(w.A, w.b, xh).max() <= w.tol
    # a BF16 inner solve reaches its 1e-2 target or stalls where the BF16 inverse stops
    # it, measured between 1/20 and 1/40 of the outer residual; with at least a
    # 10-fold reduction per correction, relres 1 -> 1e-8 takes at most 8 corrections.
    # A kernel that skipped work would stall far earlier and need more.
    assert 3 <= rep.outer <= 8, rep.outer
    xs = oracle.direct_solve(w.A, w.b)
    assert np.abs(xh - xs).max() <= 2e-6 * np.abs(xs).max()


# ----------------------------------------------------------------------------- hipGraph replay
@pytest.mark.parametrize("cfg,kw,prec,nr", [
    (1, dict(), "fp64", 1),
    (5, dict(dims=(128, 128)), "fp32_refine", 1),
    (4, dict(dims=(96, 96), nrhs=16), "bf16_refine", 16),
])
def test_graph_replay_matches_eager_bitwise(torch, cfg, kw, prec, nr):
    """Check intervals replayed as captured hipGraphs give bitwise the eager
    result with the same check schedule, solve after solve (each solve replays
    its graphs many times, with the host's own eager work and synchronisations
    in between)."""
    V = vtm()
    w = workloads.make(cfg, **kw)
    b = to_dev(torch, w.b)
    common = dict(precision=prec, nrhs_max=nr, check_every=4, adaptive_checks=False)
    eager = V.Solver(w.A, w.part, w.Z, use_graph=False, **common)
    graph = V.Solver(w.A, w.part, w.Z, use_graph=True, **common)
    xe, re = eager.solve(b, w.tol)
    for _ in range(3):
        xg, rg = graph.solve(b, w.tol)
        torch.cuda.synchronize()
        assert rg.sweeps == re.sweeps and rg.outer == re.outer
        assert torch.equal(xg, xe)
    assert oracle.relative_residual(w.A, w.b, xe.cpu().numpy()).max() <= w.tol


@pytest.mark.parametrize("form", ["port", "full"])
def test_adjoint_of_symmetric_circuit_is_the_forward_solve(torch, form):
    """A symmetric A: vtm_solve_adjoint(g) is vtm_solve(g) (same sweeps, same
    result to the rounding of reading the stored inverses transposed)."""
    w = workloads.make(1)
    s = vtm().Solver(w.A, w.part, w.Z, check_every=1, adaptive_checks=False, local_form=form)
    b = to_dev(torch, w.b)
    x, rx = s.solve(b, w.tol)
    lam, rl = s.solve_adjoint(b, w.tol)
    assert rx.sweeps == rl.sweeps
    assert_close(lam.cpu().numpy(), x.cpu().numpy())
