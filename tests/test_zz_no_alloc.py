"""vtm_solve_noalloc (the solve that allocates nothing; its residual reductions use
the library's static device workspace) against vtm_solve, through the C ABI.

Both run the same kernels in the same order, so x must be bitwise equal and
the reports identical.  Two calls in a row, the second with a smaller input,
check that nothing the first call left in the shared workspace leaks into
the second.
"""
import ctypes as C

import numpy as np
import pytest

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


def abi_solve(torch, s, fn, b, tol):
    """One call of vtm_solve or vtm_solve_noalloc through ctypes; returns status, x, report."""
    b = b.contiguous()
    x = torch.full_like(b, float("nan"))
    rel = np.zeros(b.shape[0])
    rep = vtm().binding.Report(relres=rel.ctypes.data_as(C.POINTER(C.c_double)))
    st = fn(s._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), b.shape[0], float(tol), C.byref(rep))
    torch.cuda.synchronize()
    return st, x, (rep.sweeps, rep.outer, rep.checks, rep.relres_max), rel.copy()


def compare(torch, s, b, tol):
    L = vtm().lib()
    st0, x0, r0, rel0 = abi_solve(torch, s, L.vtm_solve, b, tol)
    st1, x1, r1, rel1 = abi_solve(torch, s, L.vtm_solve_noalloc, b, tol)
    assert st0 == 0 and st1 == 0, (st0, st1, L.vtm_last_error())
    assert r0 == r1, (r0, r1)
    assert np.array_equal(rel0, rel1)
    assert torch.equal(x0, x1)
    return r0


@pytest.mark.parametrize("prec", ["bf16_refine", "fp64"])
def test_noalloc_solve_equals_solve_twice_second_smaller(torch, prec):
    """64 right-hand sides (every residual workgroup's partial sums in use), then
    5 on the same handle, then a smaller circuit on another handle."""
    w = workloads.make(4, dims=(160, 160), nrhs=64)
    s = vtm().Solver(w.A, w.part, w.Z, precision=prec, nrhs_max=64)
    b = torch.as_tensor(w.b, dtype=torch.float64, device="cuda")
    big = compare(torch, s, b, 1e-8)
    small = compare(torch, s, b[:5], 1e-8)
    assert big[0] > 0 and small[0] > 0
    s.close()
    w2 = workloads.make(1, dims=(48, 48))
    s2 = vtm().Solver(w2.A, w2.part, w2.Z, precision="fp64" if prec == "fp64" else "fp32_refine")
    compare(torch, s2, torch.as_tensor(w2.b, dtype=torch.float64, device="cuda"), 1e-10)
    s2.close()


def test_noalloc_limits(torch):
    """More than 64 right-hand sides, graphs or timing events: VTM_E_UNSUPPORTED."""
    V = vtm()
    w = workloads.make(4, dims=(64, 64), nrhs=65)
    s = V.Solver(w.A, w.part, w.Z, nrhs_max=65)
    b = torch.as_tensor(w.b, dtype=torch.float64, device="cuda")
    with pytest.raises(V.VTMError) as ei:
        s.solve_noalloc(b, 1e-8)
    assert ei.value.name == "VTM_E_UNSUPPORTED"
    x, rep = s.solve_noalloc(b[:64], 1e-8)
    assert rep.relres_max <= 1e-8
    s.close()
    for kw in (dict(use_graph=True), dict(timing=True)):
        t = V.Solver(w.A, w.part, w.Z, **kw)
        with pytest.raises(V.VTMError) as ei:
            t.solve_noalloc(b[:1], 1e-8)
        assert ei.value.name == "VTM_E_UNSUPPORTED"
        t.close()
