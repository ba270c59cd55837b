"""vtm_refresh (new conductances on the same pattern and partition, no new
tearing plan) against a handle freshly set up with the same values: the same
kernels on the same layout, so every solve must agree bitwise.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


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


def new_values(w, seed):
    """The workload's circuit with every branch conductance scaled by U[0.8, 1.25]
    (same branches, same controlled sources: the same sparsity pattern)."""
    g = w.g * np.random.default_rng(seed).uniform(0.8, 1.25, w.g.size)
    return workloads.nodal_matrix(w.n, w.edges, g, w.ground, w.vccs), g


@pytest.mark.parametrize("cfg,kw,prec,nr", [
    (2, dict(dims=(256, 256)), "fp64", 1),              # packed symmetric port-node operators
    (3, dict(dims=(16, 16, 16)), "fp64", 1),           # unsymmetric: port-node operators, transposed CSR
    (3, dict(dims=(16, 16, 16)), "fp32_refine", 1),    # blocked inversion (512-node sub-circuits), FP32
    (5, dict(dims=(128, 128)), "fp32_refine", 1),      # packed, eight wavefronts per sub-circuit
    (4, dict(dims=(96, 96), nrhs=20), "bf16_refine", 20),  # MFMA tiles, batched port-to-port operators
    (4, dict(dims=(96, 96), nrhs=20), "fp64", 20),
])
def test_refresh_equals_fresh_setup(torch, cfg, kw, prec, nr):
    w = workloads.make(cfg, **kw)
    A2, g2 = new_values(w, 1)
    Z2 = 1.0 / g2.mean()
    b = to_dev(torch, w.b)
    s = vtm().Solver(w.A, w.part, w.Z, precision=prec, nrhs_max=nr)
    x0, r0 = s.solve(b, w.tol)
    # new conductances, same impedance; then new conductances and a new impedance
    for Z in (None, Z2):
        s.refresh(A2, Z)
        fresh = vtm().Solver(A2, w.part, w.Z if Z is None else Z, precision=prec, nrhs_max=nr)
        x1, r1 = s.solve(b, w.tol)
        xf, rf = fresh.solve(b, w.tol)
        fresh.close()
        assert (r1.sweeps, r1.outer, r1.checks) == (rf.sweeps, rf.outer, rf.checks)
        assert np.array_equal(r1.relres, rf.relres)
        assert torch.equal(x1, xf)
        assert oracle.relative_residual(A2, w.b, x1.cpu().numpy()).max() <= w.tol
    # back to the first values: the first solve again, bitwise
    s.refresh(w.A, w.Z)
    x2, r2 = s.solve(b, w.tol)
    assert r2.sweeps == r0.sweeps and torch.equal(x2, x0)
    s.close()


def test_refresh_per_wire_impedance_and_adjoint(torch):
    """Per-wire impedances (Section VIII's weighted overlapped block) given at
    refresh, and the adjoint afterwards, against a fresh handle."""
    w = workloads.make(2, dims=(128, 128))
    A2, _ = new_values(w, 2)
    Wn = vtm().line_admittance(A2, w.part, "wob", 0.25)
    s = vtm().Solver(w.A, w.part, w.Z)
    s.refresh(A2, 1.0 / Wn)
    fresh = vtm().Solver(A2, w.part, 1.0 / Wn)
    b = to_dev(torch, w.b)
    for fn in ("solve", "solve_adjoint"):
        x1, r1 = getattr(s, fn)(b, w.tol)
        xf, rf = getattr(fresh, fn)(b, w.tol)
        assert r1.sweeps == rf.sweeps and torch.equal(x1, xf)
    s.close()
    fresh.close()


def test_refresh_rejects_what_a_new_setup_would_need(torch):
    """A changed pattern (an off-diagonal entry becoming zero), a changed symmetry,
    a cut that is no longer a conductance, a wrong entry count, and a handle torn
    at interfacial nodes; after each error the handle still solves as before."""
    V = vtm()
    w = workloads.make(2, dims=(64, 64))
    s = V.Solver(w.A, w.part, w.Z)
    b = to_dev(torch, w.b)
    x0, _ = s.solve(b, w.tol)
    A = w.A.tocsr()
    rows = np.repeat(np.arange(w.n), np.diff(A.indptr))
    off = np.nonzero(rows != A.indices)[0]
    cut = off[w.part[rows[off]] != w.part[A.indices[off]]][0]
    inner = off[w.part[rows[off]] == w.part[A.indices[off]]][0]
    cases = []
    v = A.data.copy()
    v[inner] = 0.0
    cases.append((v, "VTM_E_ARG"))                  # pattern change
    v = A.data.copy()
    v[inner] *= 1.5
    cases.append((v, "VTM_E_UNSUPPORTED"))          # no longer symmetric
    v = A.data.copy()
    v[cut] = 0.3
    j = np.nonzero((rows == A.indices[cut]) & (A.indices == rows[cut]))[0][0]
    v[j] = 0.3
    cases.append((v, "VTM_E_UNTEARABLE"))           # a cut coupling that is not a conductance
    for vals, name in cases:
        with pytest.raises(V.VTMError) as ei:
            s.refresh(vals)
        assert ei.value.name == name
    with pytest.raises(ValueError):
        s.refresh(A.data[:-1])
    x1, _ = s.solve(b, w.tol)
    assert torch.equal(x0, x1)
    s.close()
    wv = workloads.make(2, dims=(24, 47))
    label, iface, sides = workloads.separator_strips((24, 47), 10)
    t = V.Solver(wv.A, label, 1.0, iface=iface, sides=sides)
    with pytest.raises(V.VTMError) as ei:
        t.refresh(wv.A)
    assert ei.value.name == "VTM_E_UNSUPPORTED"
    t.close()


def test_circuit_refreshes_its_handle_when_conductances_change(torch):
    """autograd.Circuit keeps one handle and refreshes it when g changes; the
    gradient after a change equals that of a circuit built for the new g."""
    from paper_0910_0663_amd import Circuit, VTMSolve
    w = workloads.make(5, dims=(64, 64), n_probes=256)
    probes = torch.as_tensor(w.probes, device="cuda")
    b = torch.tensor(w.b[0], dtype=torch.float64, device="cuda")

    def grad(circ, g_np):
        g = torch.tensor(g_np, dtype=torch.float64, device="cuda", requires_grad=True)
        x = VTMSolve.apply(b, g, circ)
        (x[probes] ** 2).sum().backward()
        return g.grad

    c = Circuit(w.n, w.edges, w.ground, w.part, w.Z, tol=1e-10, precision="fp64")
    grad(c, w.g)
    first = c._solver
    g2 = w.g * np.random.default_rng(4).uniform(0.8, 1.25, w.g.size)
    d1 = grad(c, g2)
    assert c._solver is first
    d2 = grad(Circuit(w.n, w.edges, w.ground, w.part, w.Z, tol=1e-10, precision="fp64"), g2)
    assert torch.equal(d1, d2)
