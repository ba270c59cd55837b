"""The C-ABI boundary beyond solve: dL/dA on the caller's CSR pattern and
finite-difference checks of the gradients, the adjoint of batched (MFMA tile)
handles, and the residual history of vtm_report.

Tolerances: the gradient kernels evaluate the oracle's formulas on the same
inputs, so they agree to rounding (each entry is a sum of nrhs products: 1e-14
relative).  Gradients from solves carry the solves' error, at most
kappa(A) * tol relative (A15); against central differences (truncation
O(h^2), h = 1e-5 of the entry) that bounds the difference.  Batched FP64
iterates use the 1e-11 bound of the other FP64 iterate tests; BF16 ones the
rounding model of test_gpu_lowprec.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import workloads

pytestmark = pytest.mark.gpu

ITER_RTOL = 1e-11
U_BF16 = 2.0 ** -8


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


def assert_close(x, ref, rtol):
    scale = np.abs(ref).max()
    err = np.abs(x - ref).max()
    assert err <= rtol * scale, f"max err {err:.3e} vs {rtol:.1e} * {scale:.3e}"


def oracle_iterates(A, part, Z, b, ks):
    torn = oracle.tear_wires(A, part, Z)
    sw = oracle.Sweeper(torn)
    f = torn.src @ b.T
    a = np.zeros((2, torn.n_lines, b.shape[0]))
    out = {}
    for k in range(1, max(ks) + 1):
        u, a = sw.sweep(f, a)
        if k in ks:
            out[k] = (torn.out @ u).T
    return out


def stop_after(torch, s, fn_name, b, k):
    """Run a solver stopped after exactly k sweeps (MAXITER); returns x."""
    x = torch.empty(b.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(vtm().VTMError) as ei:
        getattr(s, fn_name)(to_dev(torch, b), 1e-300, x)
    assert ei.value.name == "VTM_E_MAXITER" and ei.value.report.sweeps == k, ei.value
    return x.cpu().numpy()


# ----------------------------------------------------------------------------- dL/dA
def _with_duplicates(A):
    """The same matrix as a CSR whose rows hold their entries in reverse order and
    where every diagonal entry is stored as two halves (duplicates are summed)."""
    A = sp.csr_matrix(A)
    rows, cols, vals = [], [], []
    for i in range(A.shape[0]):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        for q in range(hi - 1, lo - 1, -1):
            j, v = A.indices[q], A.data[q]
            if j == i:
                rows += [i, i]
                cols += [j, j]
                vals += [0.5 * v, 0.5 * v]
            else:
                rows.append(i)
                cols.append(j)
                vals.append(v)
    indptr = np.zeros(A.shape[0] + 1, dtype=np.int64)
    np.add.at(indptr, np.asarray(rows) + 1, 1)
    return sp.csr_matrix((np.asarray(vals), np.asarray(cols), np.cumsum(indptr)), shape=A.shape)


def test_grad_entries_and_branches_match_oracle(torch):
    """vtm_grad's dL/dA on the caller's CSR (unsorted rows, duplicated diagonal
    entries) and dL/dg per branch, from the same x and lambda as the oracle's
    formulas, two right-hand sides, unsymmetric A with controlled sources."""
    w = workloads.make(3, dims=(16, 16, 16), nrhs=2)
    A = _with_duplicates(w.A)
    assert A.nnz == w.A.nnz + w.n and not A.has_canonical_format
    s = vtm().Solver(A, w.part, w.Z, nrhs_max=2)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((2, w.n))
    lam = rng.standard_normal((2, w.n))
    dg, dA = s.grad(to_dev(torch, x), to_dev(torch, lam), torch.as_tensor(w.edges, device="cuda"), nnz=A.nnz)
    ref_A = oracle.matrix_gradient(A, x, lam)
    ref_g = oracle.branch_gradient(w.edges, x, lam)
    assert_close(dA.cpu().numpy(), ref_A, 1e-14)
    assert_close(dg.cpu().numpy(), ref_g, 1e-14)
    # dL/dA alone (no branch list)
    _, dA2 = s.grad(to_dev(torch, x), to_dev(torch, lam), None, nnz=A.nnz)
    assert torch.equal(dA, dA2)
    s.close()


def test_controlled_source_gains_gradient_matches_finite_differences(torch):
    """L = sum over probes of x^2 on a 32^3 grid with controlled sources, x and
    lambda from FP32 sweeps in FP64 refinement to 1e-10: dL/dA of 32
    controlled-source gains (single one-sided entries of A, eq. 15) against
    central differences of L through direct solves."""
    w = workloads.make(3, dims=(32, 32, 32))
    A = sp.csr_matrix(w.A)
    probes = np.random.default_rng(3).choice(w.n, 512, replace=False)
    s = vtm().Solver(A, w.part, w.Z, precision="fp32_refine")
    x, _ = s.solve(to_dev(torch, w.b), 1e-10)
    g = torch.zeros_like(x)
    g[0, probes] = 2.0 * x[0, probes]
    lam, _ = s.solve_adjoint(g, 1e-10)
    _, dA = s.grad(x, lam, None, nnz=A.nnz)
    dA = dA.cpu().numpy()
    s.close()
    rows = np.repeat(np.arange(w.n), np.diff(A.indptr))
    k_node, c_node, _ = w.vccs
    pick = np.random.default_rng(9).choice(k_node.size, 32, replace=False)
    entries = [int(np.nonzero((rows == k_node[p]) & (A.indices == c_node[p]))[0][0]) for p in pick]
    # L(a_kc +- h) exactly from one sparse LU: the change h e_k e_c^T gives
    # x(h) = x - h x_c A^-1 e_k / (1 + h (A^-1 e_k)_c)  (Sherman-Morrison)
    lu = spla.splu(sp.csc_matrix(A))
    xs = lu.solve(w.b.ravel())
    fd = []
    for k in entries:
        r, c = rows[k], A.indices[k]
        e = np.zeros(w.n)
        e[r] = 1.0
        z = lu.solve(e)
        h = 1e-5 * abs(A.data[k])
        vals = [np.sum((xs - dh * xs[c] / (1.0 + dh * z[c]) * z)[probes] ** 2) for dh in (h, -h)]
        fd.append((vals[0] - vals[1]) / (2 * h))
    fd = np.array(fd)
    print(f"max |fd| {np.abs(fd).max():.3e}, max diff {np.abs(fd - dA[entries]).max():.3e}", flush=True)
    # kappa(A) < 3e3 here (branch sums over the 0.01 S ground); solves to 1e-10 leave
    # at most 3e-7 relative in x and in lambda
    assert np.abs(fd - dA[entries]).max() <= 1e-6 * np.abs(fd).max()


def test_full_size_512sq_branch_gradient_matches_finite_differences(torch):
    """The gradient workload at full size (512^2, 4,096 probes, FP32 sweeps with FP64
    refinement to 1e-8): dL/dg of 64 random branches against central differences
    (h = 1e-5 g) of L.  L(g +- h) is computed exactly from one sparse LU of A by
    the Sherman-Morrison formula: a branch change dg adds dg u u^T, u = e_i - e_j,
    so x(g + dg) = x - dg (u^T x) A^-1 u / (1 + dg u^T A^-1 u)."""
    from paper_0910_0663_amd import Circuit, VTMSolve
    w = workloads.make(5)
    circ = Circuit(w.n, w.edges, w.ground, w.part, w.Z, tol=w.tol, precision="fp32_refine")
    g = torch.tensor(w.g, dtype=torch.float64, device="cuda", requires_grad=True)
    b = torch.tensor(w.b[0], dtype=torch.float64, device="cuda")
    x = VTMSolve.apply(b, g, circ)
    probes = torch.as_tensor(w.probes, device="cuda")
    (x[probes] ** 2).sum().backward()
    grad = g.grad.cpu().numpy()
    lu = spla.splu(sp.csc_matrix(w.A))
    xs = lu.solve(w.b.ravel())
    pick = np.random.default_rng(13).choice(w.edges.shape[0], 64, replace=False)
    fd = []
    for e in pick:
        i, j = w.edges[e]
        u = np.zeros(w.n)
        u[i], u[j] = 1.0, -1.0
        z = lu.solve(u)
        h = 1e-5 * w.g[e]
        vals = []
        for dg in (h, -h):
            xp = xs - dg * (xs[i] - xs[j]) / (1.0 + dg * (z[i] - z[j])) * z
            vals.append(np.sum(xp[w.probes] ** 2))
        fd.append((vals[0] - vals[1]) / (2 * h))
    fd = np.array(fd)
    print(f"max |fd| {np.abs(fd).max():.3e}, max diff {np.abs(fd - grad[pick]).max():.3e}", flush=True)
    # the solves' own error bounds the difference: kappa(A) tol, kappa < 2e3 on this grid
    # (largest eigenvalue below 4 x 2 x 2 S, smallest above the 0.01 S ground)
    assert np.abs(fd - grad[pick]).max() <= 2e-5 * np.abs(grad).max()


# ----------------------------------------------------------------------------- batched adjoint
def test_batched_fp64_adjoint_iterates_match_oracle_transpose(torch):
    """An unsymmetric A on a handle with MFMA tiles (FP64, 16 right-hand sides):
    the adjoint sweeps use the transposed tiles, and x^k equals the oracle's VTM
    iterate on the torn A^T; the converged lambda is A^-T g."""
    w = workloads.make(3, dims=(16, 16, 16))
    g = np.random.default_rng(5).standard_normal((16, w.n))
    At = w.A.T.tocsr()
    ks = [1, 3, 9]
    ref = oracle_iterates(At, w.part, w.Z, g, ks)
    for k in ks:
        s = vtm().Solver(w.A, w.part, w.Z, nrhs_max=16, check_every=k, max_sweeps=k, adaptive_checks=False)
        assert s.inverse_bytes > 0
        assert_close(stop_after(torch, s, "solve_adjoint", g, k), ref[k], ITER_RTOL)
        s.close()
    s = vtm().Solver(w.A, w.part, w.Z, nrhs_max=16)
    lam, rep = s.solve_adjoint(to_dev(torch, g), 1e-11)
    lam_ref = oracle.direct_adjoint(w.A, g)
    assert np.abs(lam.cpu().numpy() - lam_ref).max() <= 1e-8 * np.abs(lam_ref).max()
    s.close()


def test_batched_bf16_adjoint_iterates_and_refinement(torch):
    """BF16 tiles of K^-T: the inner iterate of the adjoint (one outer step, k
    sweeps) against the oracle's iterate on the torn A^T at the BF16 rounding
    bound (5.5 sqrt(k) u sqrt(2/3) of max|x|), and the refined adjoint reaches
    1e-8 on A^T."""
    w = workloads.make(3, dims=(16, 16, 16))
    g = np.random.default_rng(6).standard_normal((16, w.n))
    At = w.A.T.tocsr()
    for k in (1, 4):
        ref = oracle_iterates(At, w.part, w.Z, g, [k])[k]
        s = vtm().Solver(w.A, w.part, w.Z, precision="bf16_refine", nrhs_max=16, check_every=k, max_sweeps=k,
                         max_outer=1, adaptive_checks=False)
        x = stop_after(torch, s, "solve_adjoint", g, k)
        s.close()
        assert_close(x, ref, 5.5 * math.sqrt(k) * U_BF16 * math.sqrt(2.0 / 3.0))
    s = vtm().Solver(w.A, w.part, w.Z, precision="bf16_refine", nrhs_max=16)
    lam, rep = s.solve_adjoint(to_dev(torch, g), 1e-8)
    assert oracle.relative_residual(At, g, lam.cpu().numpy()).max() <= 1e-8
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16_refine"])
def test_batched_adjoint_of_symmetric_circuit_is_the_forward_solve(torch, prec):
    """Symmetric A on tiles: the adjoint runs the same tiles and port-to-port
    operators as the forward solve, so lambda(g) is bitwise x(g)."""
    w = workloads.make(4, dims=(96, 96), nrhs=20)
    s = vtm().Solver(w.A, w.part, w.Z, precision=prec, nrhs_max=20)
    b = to_dev(torch, w.b)
    x, rx = s.solve(b, 1e-9)
    lam, rl = s.solve_adjoint(b, 1e-9)
    assert rx.sweeps == rl.sweeps and rx.outer == rl.outer
    assert torch.equal(x, lam)
    s.close()


# ----------------------------------------------------------------------------- residual history
def test_residual_history_of_plain_solve_matches_oracle(torch):
    """Checked every sweep in the full form, the history is the oracle's
    residual after every sweep (plus the check of x = 0): 1 exactly, then
    falling to the tolerance; the last entry is the final relres."""
    w = workloads.make(1)
    r = oracle.vtm_solve(oracle.tear_wires(w.A, w.part, w.Z), w.A, w.b, w.tol)
    s = vtm().Solver(w.A, w.part, w.Z, check_every=1, adaptive_checks=False, local_form="full")
    x, rep = s.solve(to_dev(torch, w.b), w.tol)
    h = rep.history
    assert h.size == rep.checks == rep.sweeps + 1
    assert h[0] == 1.0 and list(rep.history_sweeps) == list(range(rep.sweeps + 1))
    assert h[-1] == rep.relres_max <= w.tol
    n = min(len(r.history), h.size - 1)
    ratio = h[1:n + 1] / np.asarray(r.history[:n])
    assert np.abs(ratio - 1.0).max() <= 1e-3, np.abs(ratio - 1.0).max()
    s.close()


def test_residual_history_of_port_checks_and_refinement(torch):
    """Port-to-port form with adaptive checks: the history has one entry per
    check, sweeps increasing, ending at the final relres.  BF16 refinement: one
    entry per outer step, each correction at least 10-fold (the bound behind
    the outer-step count of the refinement tests)."""
    w = workloads.make(2, dims=(256, 256))
    s = vtm().Solver(w.A, w.part, w.Z)
    _, rep = s.solve(to_dev(torch, w.b), w.tol)
    assert rep.history.size == rep.checks and np.all(np.diff(rep.history_sweeps) >= 0)
    assert rep.history_sweeps[-1] == rep.sweeps and rep.history[-1] == rep.relres_max
    s.close()
    w4 = workloads.make(4, dims=(192, 192), nrhs=32)
    s = vtm().Solver(w4.A, w4.part, w4.Z, precision="bf16_refine", nrhs_max=32)
    _, rep = s.solve(to_dev(torch, w4.b), w4.tol)
    h = rep.history
    print("bf16 outer residuals", h, flush=True)
    assert h.size == rep.outer + 1 and h[0] == 1.0 and h[-1] <= w4.tol
    # every correction but the last cuts the residual 10-fold; the last one's inner
    # target is only what the tolerance needs, 0.5 tol / relres
    assert np.all(h[1:-1] <= 0.1 * h[:-2]) and h[-1] <= w4.tol
    s.close()
