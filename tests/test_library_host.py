"""Host-side checks of the C-ABI library: it loads, exports every symbol that
include/vtm.h declares, and its tearing planner (host code, no device work)
agrees with the oracle's independently derived eliminated-twin form."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads
import paper_0910_0663_amd as vtm
from paper_0910_0663_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "vtm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vtm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "vtm_setup" in names and "vtm_solve" in names and "vtm_solve_adjoint" in names
    assert "vtm_grad" in names
    L = vtm.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(vtm.EXPORTS) == names


@pytest.mark.parametrize("cfg,kw", [
    (1, dict()),
    (3, dict(dims=(16, 16, 16))),
    (4, dict(dims=(96, 96))),
    (2, dict(dims=(64, 64))),
])
def test_plan_matches_oracle(cfg, kw):
    w = workloads.make(cfg, **kw)
    i, j, g = oracle.cut_wires(w.A, w.part)
    pl = vtm.plan(w.A, w.part, w.Z)
    assert pl["n_sub"] == w.n_sub
    assert np.array_equal(pl["wires"][:, 0], i) and np.array_equal(pl["wires"][:, 1], j)
    el = oracle.eliminate_twins(w.A, w.part, w.Z)
    for key in ("G", "c", "beta", "gamma"):
        assert np.allclose(pl[key], getattr(el, key)[0::2], rtol=1e-15, atol=0), key


def test_plan_per_wire_impedance():
    w = workloads.make(1, dims=(32, 32))
    L = oracle.cut_wires(w.A, w.part)[0].size
    Z = np.random.default_rng(0).uniform(0.2, 5.0, L)
    pl = vtm.plan(w.A, w.part, Z)
    el = oracle.eliminate_twins(w.A, w.part, Z)
    assert np.allclose(pl["beta"], el.beta[0::2], rtol=1e-15)
    assert np.allclose(pl["gamma"], el.gamma[0::2], rtol=1e-15, atol=1e-16)


def test_plan_cut_counts_of_full_size_partitions():
    """Cut wires of the block partitions follow from the geometry: for a 2-D grid
    of ny x nx nodes in blocks, (block columns - 1) * ny + (block rows - 1) * nx."""
    for (ny, nx), (by, bx) in [((64, 64), (16, 16)), ((128, 96), (8, 8)), ((40, 24), (8, 12))]:
        e = workloads.grid2d_edges(ny, nx)
        n = ny * nx
        A = workloads.nodal_matrix(n, e, np.ones(e.shape[0]), np.full(n, 0.01))
        part = workloads.block_partition_2d(ny, nx, by, bx)
        pl = vtm.plan(A, part, 1.0)
        assert pl["wires"].shape[0] == (nx // bx - 1) * ny + (ny // by - 1) * nx


def _status_of(call):
    with pytest.raises(vtm.VTMError) as ei:
        call()
    return ei.value.name


def test_plan_rejects_bad_input():
    w = workloads.make(1, dims=(16, 16), block=(4, 4))
    A = w.A.tolil()
    A[0, 200] = 0.3                      # one-sided coupling across sub-circuits
    assert _status_of(lambda: vtm.plan(A.tocsr(), w.part, 1.0)) == "VTM_E_UNTEARABLE"
    B = w.A.tolil()
    B[0, 200] = B[200, 0] = 0.3          # symmetric but positive: not a conductance
    assert _status_of(lambda: vtm.plan(B.tocsr(), w.part, 1.0)) == "VTM_E_UNTEARABLE"
    bad = w.part.copy()
    bad[bad == 1] = 2                    # label 1 unused
    assert _status_of(lambda: vtm.plan(w.A, bad, 1.0)) == "VTM_E_ARG"
    assert _status_of(lambda: vtm.plan(w.A, w.part, -1.0)) == "VTM_E_ARG"
    assert _status_of(lambda: vtm.plan(w.A, w.part, [1.0, 2.0])) == "VTM_E_ARG"
    C = w.A.copy()
    C.data[3] = np.nan
    assert _status_of(lambda: vtm.plan(C, w.part, 1.0)) == "VTM_E_ARG"
    big = np.zeros(w.n, dtype=np.int32)
    e = workloads.grid2d_edges(129, 129)   # one sub-circuit of 16,641 nodes: above the 16,384 limit
    A129 = workloads.nodal_matrix(129 * 129, e, np.ones(e.shape[0]), np.full(129 * 129, 0.01))
    assert _status_of(lambda: vtm.plan(A129, np.zeros(129 * 129, np.int32), 1.0)) == "VTM_E_UNSUPPORTED"
    assert big.size == w.n


def test_plan_merges_duplicates_and_ignores_row_order():
    """Duplicate CSR entries are summed and column order inside a row is free."""
    w = workloads.make(1, dims=(16, 16), block=(4, 4))
    coo = w.A.tocoo()
    rng = np.random.default_rng(1)
    k = rng.permutation(coo.nnz)
    r, c, v = coo.row[k], coo.col[k], coo.data[k]
    half = v / 2
    dup = sp.coo_matrix((np.concatenate([half, half]), (np.concatenate([r, r]), np.concatenate([c, c]))),
                        shape=w.A.shape)
    rows = np.concatenate([r, r])
    order = np.argsort(rows, kind="stable")
    indptr = np.searchsorted(rows[order], np.arange(w.n + 1))
    A2 = sp.csr_matrix((dup.data[order], dup.col[order], indptr), shape=w.A.shape)
    assert not A2.has_sorted_indices
    p1 = vtm.plan(w.A, w.part, w.Z)
    p2 = vtm.plan(A2, w.part, w.Z)
    assert np.array_equal(p1["wires"], p2["wires"])
    assert np.allclose(p1["G"], p2["G"], rtol=1e-15)


@pytest.mark.parametrize("cfg,kw", [(1, dict()), (2, dict(dims=(64, 64))), (4, dict(dims=(96, 96)))])
def test_line_admittance_rules(cfg, kw):
    """Section VIII's rules per cut wire.  The scaled mean reproduces the
    generator's own W = mean branch conductance; the overlapped block W = C is
    each twin's own diagonal in the oracle's tear (2g of the split midpoint, on
    both sides); the weighted block and alpha I scale as stated."""
    w = workloads.make(cfg, **kw)
    W_mean = vtm.line_admittance(w.A, w.part, "scaled_mean", 1.0)
    assert np.allclose(W_mean, 1.0 / w.Z, rtol=1e-13, atol=0)
    assert np.allclose(vtm.line_admittance(w.A, w.part, "scaled_mean", 0.25), 0.25 / w.Z, rtol=1e-13, atol=0)
    torn = oracle.tear_wires(w.A, w.part, w.Z)
    T = torn.T.tocsr()
    W_ob = vtm.line_admittance(w.A, w.part, "ob")
    assert np.allclose(W_ob, T[torn.pa, torn.pa].A1, rtol=1e-14, atol=0)
    assert np.allclose(W_ob, T[torn.pb, torn.pb].A1, rtol=1e-14, atol=0)
    assert np.allclose(vtm.line_admittance(w.A, w.part, "wob", 0.125), 0.125 * W_ob, rtol=1e-15, atol=0)
    assert np.all(vtm.line_admittance(w.A, w.part, "identity", 0.7) == 0.7)


def test_line_admittance_bad_arguments():
    w = workloads.make(1)
    L = vtm.lib()
    assert _status_of(lambda: vtm.line_admittance(w.A, w.part, "ob", 0.0)) == "VTM_E_ARG"
    hc = binding._HostCsr(w.A)
    part = np.ascontiguousarray(w.part, dtype=np.int32)
    out = np.zeros(10)
    st = L.vtm_line_admittance(ctypes.byref(hc.s), part.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 2, 1.0,
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 10)
    assert L.vtm_status_str(st).decode() == "VTM_E_ARG"    # wrong wire count
    st = L.vtm_line_admittance(ctypes.byref(hc.s), part.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 7, 1.0,
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 10)
    assert L.vtm_status_str(st).decode() == "VTM_E_ARG"    # unknown rule
