"""ctypes binding of libvtm.so (include/vtm.h): argument marshalling only.

Every step of the iteration runs in the library's HIP kernels; torch supplies
device memory and the current stream.  Importing this module does not load the
library; the first call does, and raises if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvtm.so")

FP64, FP32_REFINE, BF16_REFINE = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32_refine": FP32_REFINE, "bf16_refine": BF16_REFINE}

STATUS = ["VTM_OK", "VTM_E_ARG", "VTM_E_UNTEARABLE", "VTM_E_SINGULAR", "VTM_E_DIVERGED",
          "VTM_E_MAXITER", "VTM_E_HIP", "VTM_E_OOM", "VTM_E_UNSUPPORTED"]

EXPORTS = ["vtm_default_options", "vtm_setup", "vtm_solve", "vtm_solve_adjoint", "vtm_grad",
           "vtm_get_waves", "vtm_set_waves", "vtm_info", "vtm_destroy", "vtm_status_str",
           "vtm_last_error", "vtm_plan", "vtm_line_admittance", "vtm_setup_vertex",
           "vtm_split_vertex", "vtm_setup_vertex_coupled", "vtm_vertex_admittance", "vtm_vertex_sca",
           "vtm_solve_noalloc", "vtm_refresh"]


class VTMError(RuntimeError):
    def __init__(self, status: int, message: str, report=None):
        self.status = status
        self.name = STATUS[status] if 0 <= status < len(STATUS) else str(status)
        self.report = report
        super().__init__(f"{self.name}: {message}")


class Csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.POINTER(C.c_int64)),
                ("col", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_double))]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("nrhs_max", C.c_int32), ("check_every", C.c_int32),
                ("max_outer", C.c_int32), ("max_sweeps", C.c_int64), ("divergence", C.c_double),
                ("inner_drop", C.c_double), ("use_graph", C.c_int32), ("timing", C.c_int32),
                ("adaptive_checks", C.c_int32), ("batch_row_tiles", C.c_int32),
                ("batch_rhs_block", C.c_int32), ("local_form", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("sweeps", C.c_int64), ("outer", C.c_int32), ("checks", C.c_int32),
                ("relres_max", C.c_double), ("solve_ms", C.c_double), ("sweep_kernel_ms", C.c_double),
                ("sweep_launches", C.c_int64), ("batch_row_tiles", C.c_int32), ("batch_rhs_block", C.c_int32),
                ("pp_kernel_ms", C.c_double), ("pp_launches", C.c_int64), ("pp_shape", C.c_int32 * 3),
                ("relres", C.POINTER(C.c_double)), ("history", C.POINTER(C.c_double)),
                ("history_sweeps", C.POINTER(C.c_int64)), ("history_cap", C.c_int32),
                ("history_len", C.c_int32), ("history_total", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    """Load libvtm.so (built in-tree by ``paper_0910_0663_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_0910_0663_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    L.vtm_default_options.argtypes = [C.POINTER(Options)]
    L.vtm_default_options.restype = None
    L.vtm_setup.argtypes = [C.POINTER(Csr), C.POINTER(C.c_int32), dp, i64, C.POINTER(Options), vp,
                            C.POINTER(vp)]
    L.vtm_setup.restype = C.c_int
    L.vtm_setup_vertex.argtypes = [C.POINTER(Csr), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), i64, dp, i64, C.POINTER(Options), vp, C.POINTER(vp)]
    L.vtm_setup_vertex.restype = C.c_int
    for name in ("vtm_solve", "vtm_solve_adjoint", "vtm_solve_noalloc"):
        f = getattr(L, name)
        f.argtypes = [vp, vp, vp, i32, C.c_double, C.POINTER(Report)]
        f.restype = C.c_int
    L.vtm_grad.argtypes = [vp, vp, vp, i32, vp, i64, vp, vp]
    L.vtm_grad.restype = C.c_int
    L.vtm_refresh.argtypes = [vp, dp, dp, i64]
    L.vtm_refresh.restype = C.c_int
    L.vtm_get_waves.argtypes = [vp, vp, i32]
    L.vtm_get_waves.restype = C.c_int
    L.vtm_set_waves.argtypes = [vp, vp, i32]
    L.vtm_set_waves.restype = C.c_int
    L.vtm_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64),
                           C.POINTER(i64)]
    L.vtm_info.restype = C.c_int
    L.vtm_destroy.argtypes = [vp]
    L.vtm_destroy.restype = None
    L.vtm_status_str.argtypes = [C.c_int]
    L.vtm_status_str.restype = C.c_char_p
    L.vtm_last_error.argtypes = []
    L.vtm_last_error.restype = C.c_char_p
    L.vtm_plan.argtypes = [C.POINTER(Csr), C.POINTER(C.c_int32), dp, i64, C.POINTER(i64), C.POINTER(i64),
                           C.POINTER(C.c_int32), dp]
    L.vtm_plan.restype = C.c_int
    L.vtm_line_admittance.argtypes = [C.POINTER(Csr), C.POINTER(C.c_int32), C.c_int32, C.c_double, dp, i64]
    L.vtm_line_admittance.restype = C.c_int
    L.vtm_split_vertex.argtypes = [C.POINTER(Csr), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), i64, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64),
                                   C.POINTER(C.c_int32), dp, C.POINTER(C.c_int32)]
    L.vtm_split_vertex.restype = C.c_int
    L.vtm_setup_vertex_coupled.argtypes = [C.POINTER(Csr), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                           C.POINTER(C.c_int32), i64, C.POINTER(Csr), C.POINTER(Options), vp,
                                           C.POINTER(vp)]
    L.vtm_setup_vertex_coupled.restype = C.c_int
    L.vtm_vertex_admittance.argtypes = [C.POINTER(Csr), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_int32), i64, C.c_int32, C.c_double, C.c_int32,
                                        C.POINTER(i64), C.POINTER(i64), C.POINTER(C.c_int32), dp]
    L.vtm_vertex_admittance.restype = C.c_int
    L.vtm_vertex_sca.argtypes = [C.POINTER(Csr), C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                 i64, C.c_int32, C.c_int32, C.c_double, C.POINTER(i64), C.POINTER(i64),
                                 C.POINTER(C.c_int32), dp]
    L.vtm_vertex_sca.restype = C.c_int
    _lib = L
    return L


def _check(status: int, report=None):
    if status != 0:
        raise VTMError(status, lib().vtm_last_error().decode(), report)


class _HostCsr:
    """Keeps numpy arrays alive while a vtm_csr points at them."""

    def __init__(self, A):
        import scipy.sparse as sp
        A = sp.csr_matrix(A)
        self.rowptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
        self.col = np.ascontiguousarray(A.indices, dtype=np.int32)
        self.val = np.ascontiguousarray(A.data, dtype=np.float64)
        self.n = A.shape[0]
        if A.shape[0] != A.shape[1]:
            raise ValueError("A must be square")
        self.s = Csr(self.n, self.val.size, self.rowptr.ctypes.data_as(C.POINTER(C.c_int64)),
                     self.col.ctypes.data_as(C.POINTER(C.c_int32)),
                     self.val.ctypes.data_as(C.POINTER(C.c_double)))


def _z_array(Z):
    z = np.ascontiguousarray(np.atleast_1d(np.asarray(Z, dtype=np.float64)))
    return z, z.ctypes.data_as(C.POINTER(C.c_double)), z.size


def plan(A, part, Z) -> dict:
    """Host-only tearing plan (vtm_plan): cut wires and their port coefficients."""
    L = lib()
    hc = _HostCsr(A)
    part = np.ascontiguousarray(part, dtype=np.int32)
    z, zp, nz = _z_array(Z)
    ns, nw = C.c_int64(), C.c_int64()
    pp = part.ctypes.data_as(C.POINTER(C.c_int32))
    _check(L.vtm_plan(C.byref(hc.s), pp, zp, nz, C.byref(ns), C.byref(nw), None, None))
    wires = np.zeros((nw.value, 2), dtype=np.int32)
    coef = np.zeros((nw.value, 4), dtype=np.float64)
    _check(L.vtm_plan(C.byref(hc.s), pp, zp, nz, None, None, wires.ctypes.data_as(C.POINTER(C.c_int32)),
                      coef.ctypes.data_as(C.POINTER(C.c_double))))
    return dict(n_sub=ns.value, wires=wires, G=coef[:, 0], c=coef[:, 1], beta=coef[:, 2],
                gamma=coef[:, 3])


def split_vertex(A, label, iface, sides):
    """Host-only: the system torn at interfacial nodes (vtm_split_vertex), as a
    scipy CSR matrix of n + len(iface) nodes (duplicates summed) and its
    sub-circuit labels."""
    import scipy.sparse as sp
    L = lib()
    hc = _HostCsr(A)
    i32p = C.POINTER(C.c_int32)
    label = np.ascontiguousarray(label, dtype=np.int32)
    iface = np.ascontiguousarray(iface, dtype=np.int32)
    sides = np.ascontiguousarray(sides, dtype=np.int32).reshape(-1, 2)
    args = (C.byref(hc.s), label.ctypes.data_as(i32p), iface.ctypes.data_as(i32p), sides.ctypes.data_as(i32p),
            iface.size)
    nt, nnz = C.c_int64(), C.c_int64()
    _check(L.vtm_split_vertex(*args, C.byref(nt), C.byref(nnz), None, None, None, None))
    rowptr = np.zeros(nt.value + 1, dtype=np.int64)
    col = np.zeros(nnz.value, dtype=np.int32)
    val = np.zeros(nnz.value, dtype=np.float64)
    part = np.zeros(nt.value, dtype=np.int32)
    _check(L.vtm_split_vertex(*args, None, None, rowptr.ctypes.data_as(C.POINTER(C.c_int64)),
                              col.ctypes.data_as(i32p), val.ctypes.data_as(C.POINTER(C.c_double)),
                              part.ctypes.data_as(i32p)))
    M = sp.csr_matrix((val, col, rowptr), shape=(nt.value, nt.value))
    M.sum_duplicates()
    return M, part


def vertex_sca(A, label, iface, sides, side=0, depth=1, drop=0.0):
    """Schur complement approximation W over the interfacial nodes (rule 5 of
    Section VIII; vtm_vertex_sca), as a scipy CSR matrix in iface order;
    depth=None keeps every inner node (the exact Schur complement)."""
    import scipy.sparse as sp
    L = lib()
    hc = _HostCsr(A)
    i32p = C.POINTER(C.c_int32)
    label = np.ascontiguousarray(label, dtype=np.int32)
    iface = np.ascontiguousarray(iface, dtype=np.int32)
    sides = np.ascontiguousarray(sides, dtype=np.int32).reshape(-1, 2)
    args = (C.byref(hc.s), label.ctypes.data_as(i32p), iface.ctypes.data_as(i32p), sides.ctypes.data_as(i32p),
            iface.size, int(side), -1 if depth is None else int(depth), float(drop))
    nnz = C.c_int64()
    _check(L.vtm_vertex_sca(*args, C.byref(nnz), None, None, None))
    rowptr = np.zeros(iface.size + 1, dtype=np.int64)
    col = np.zeros(nnz.value, dtype=np.int32)
    val = np.zeros(nnz.value, dtype=np.float64)
    _check(L.vtm_vertex_sca(*args, None, rowptr.ctypes.data_as(C.POINTER(C.c_int64)), col.ctypes.data_as(i32p),
                            val.ctypes.data_as(C.POINTER(C.c_double))))
    return sp.csr_matrix((val, col, rowptr), shape=(iface.size, iface.size))


ADMITTANCE_RULES = {"scaled_mean": 0, "identity": 1, "ob": 2, "wob": 3, "diag": 4}


def vertex_admittance(A, label, iface, sides, rule="ob", alpha=1.0, side=0):
    """W over the interfacial nodes under a rule of Section VIII
    (vtm_vertex_admittance), as a scipy CSR matrix in iface order."""
    import scipy.sparse as sp
    L = lib()
    hc = _HostCsr(A)
    i32p = C.POINTER(C.c_int32)
    label = np.ascontiguousarray(label, dtype=np.int32)
    iface = np.ascontiguousarray(iface, dtype=np.int32)
    sides = np.ascontiguousarray(sides, dtype=np.int32).reshape(-1, 2)
    args = (C.byref(hc.s), label.ctypes.data_as(i32p), iface.ctypes.data_as(i32p), sides.ctypes.data_as(i32p),
            iface.size, ADMITTANCE_RULES[rule], float(alpha), int(side))
    nnz = C.c_int64()
    _check(L.vtm_vertex_admittance(*args, C.byref(nnz), None, None, None))
    rowptr = np.zeros(iface.size + 1, dtype=np.int64)
    col = np.zeros(nnz.value, dtype=np.int32)
    val = np.zeros(nnz.value, dtype=np.float64)
    _check(L.vtm_vertex_admittance(*args, None, rowptr.ctypes.data_as(C.POINTER(C.c_int64)),
                                   col.ctypes.data_as(i32p), val.ctypes.data_as(C.POINTER(C.c_double))))
    return sp.csr_matrix((val, col, rowptr), shape=(iface.size, iface.size))


def line_admittance(A, part, rule="scaled_mean", alpha=1.0):
    """Characteristic admittance of every cut wire under a rule of Section VIII
    (vtm_line_admittance), in the canonical wire order; pass Z = 1 / W."""
    L = lib()
    hc = _HostCsr(A)
    part = np.ascontiguousarray(part, dtype=np.int32)
    pp = part.ctypes.data_as(C.POINTER(C.c_int32))
    nw = plan(A, part, 1.0)["wires"].shape[0]
    W = np.zeros(nw, dtype=np.float64)
    _check(L.vtm_line_admittance(C.byref(hc.s), pp, ADMITTANCE_RULES[rule], float(alpha),
                                 W.ctypes.data_as(C.POINTER(C.c_double)), nw))
    return W


@dataclass
class SolveReport:
    sweeps: int
    outer: int
    checks: int
    relres_max: float
    solve_ms: float
    relres: np.ndarray
    sweep_kernel_ms: float = 0.0
    sweep_launches: int = 0
    batch_shape: tuple = (0, 0)
    pp_kernel_ms: float = 0.0
    pp_launches: int = 0
    pp_shape: tuple = (0, 0, 0)
    history: np.ndarray = None          # max relative residual per check (per outer step when refining)
    history_sweeps: np.ndarray = None   # sweeps run by each entry


def _ptr(t) -> int:
    return t.data_ptr()


class Solver:
    """A torn circuit on the current HIP device (vtm_setup).

    A: scipy sparse (host), part: int labels per node, Z: scalar or per cut wire.
    With ``iface`` and ``sides`` given, the circuit is torn at those interfacial
    nodes instead (vtm_setup_vertex): ``part`` then labels the inner nodes and
    ``Z`` is the impedance of each twin-joining line (scalar or per interfacial
    node); or ``W``, a scipy sparse admittance matrix over the interfacial
    nodes, couples the lines (vtm_setup_vertex_coupled; Z is then ignored).
    """

    HISTORY_CAP = 4096   # residual-history entries kept per solve

    def __init__(self, A, part, Z, precision="fp64", nrhs_max=1, check_every=8,
                 max_sweeps=1_000_000, divergence=1e6, inner_drop=0.0, max_outer=30,
                 use_graph=False, timing=False, adaptive_checks=True, batch_shape=(0, 0), local_form="port",
                 stream=None, iface=None, sides=None, W=None):
        import torch
        L = lib()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the VTM library runs on the GPU only")
        self._torch = torch
        opt = Options()
        L.vtm_default_options(C.byref(opt))
        opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        opt.nrhs_max = int(nrhs_max)
        opt.check_every = int(check_every)
        opt.max_sweeps = int(max_sweeps)
        opt.divergence = float(divergence)
        opt.inner_drop = float(inner_drop)
        opt.max_outer = int(max_outer)
        opt.use_graph = 1 if use_graph else 0
        opt.timing = int(timing) if isinstance(timing, int) and not isinstance(timing, bool) else (1 if timing else 0)
        opt.adaptive_checks = 1 if adaptive_checks else 0
        opt.batch_row_tiles, opt.batch_rhs_block = int(batch_shape[0]), int(batch_shape[1])
        opt.local_form = {"full": 0, "port": 1, "port_dense": 2}[local_form] if isinstance(local_form, str) else int(local_form)
        self.precision = precision
        self.nrhs_max = int(nrhs_max)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        hc = _HostCsr(A)
        self.n = hc.n
        self.nnz = int(hc.val.size)   # entries of A as given (the dL/dA of grad)
        part = np.ascontiguousarray(part, dtype=np.int32)
        if part.size != self.n:
            raise ValueError("part must have one label per node")
        h = C.c_void_p()
        if iface is None:
            z, zp, nz = _z_array(Z)
            _check(L.vtm_setup(C.byref(hc.s), part.ctypes.data_as(C.POINTER(C.c_int32)), zp, nz, C.byref(opt),
                               C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        else:
            iface = np.ascontiguousarray(iface, dtype=np.int32)
            sides = np.ascontiguousarray(sides, dtype=np.int32).reshape(-1, 2)
            if sides.shape[0] != iface.size:
                raise ValueError("sides must hold two sub-circuits per interfacial node")
            i32p = C.POINTER(C.c_int32)
            if W is not None:
                wc = _HostCsr(W)
                _check(L.vtm_setup_vertex_coupled(C.byref(hc.s), part.ctypes.data_as(i32p),
                                                  iface.ctypes.data_as(i32p), sides.ctypes.data_as(i32p),
                                                  iface.size, C.byref(wc.s), C.byref(opt),
                                                  C.c_void_p(self.stream.cuda_stream), C.byref(h)))
            else:
                w, wp, nw_ = _z_array(1.0 / np.asarray(Z, dtype=np.float64))
                _check(L.vtm_setup_vertex(C.byref(hc.s), part.ctypes.data_as(i32p), iface.ctypes.data_as(i32p),
                                          sides.ctypes.data_as(i32p), iface.size, wp, nw_, C.byref(opt),
                                          C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        n, ns, nw, kb, pb, sb = (C.c_int64() for _ in range(6))
        _check(L.vtm_info(h, C.byref(n), C.byref(ns), C.byref(nw), C.byref(kb), C.byref(pb), C.byref(sb)))
        self.n_sub, self.n_wires, self.inverse_bytes = ns.value, nw.value, kb.value
        self.port_operator_bytes, self.port_sweep_bytes = pb.value, sb.value

    # -- helpers ---------------------------------------------------------------
    def _vec(self, t, name):
        torch = self._torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
            raise TypeError(f"{name} must be a float64 tensor on the GPU")
        if t.dim() == 1:
            t = t.unsqueeze(0)
        if t.dim() != 2 or t.shape[1] != self.n:
            raise ValueError(f"{name} must have shape [n] or [nrhs, n]")
        return t.contiguous()

    def _run(self, fn, b, tol, x):
        b = self._vec(b, "b")
        nrhs = b.shape[0]
        if x is None:
            x = self._torch.empty_like(b)
        rel = np.zeros(nrhs)
        hist = np.zeros(self.HISTORY_CAP)
        hsw = np.zeros(self.HISTORY_CAP, dtype=np.int64)
        rep = Report(relres=rel.ctypes.data_as(C.POINTER(C.c_double)),
                     history=hist.ctypes.data_as(C.POINTER(C.c_double)),
                     history_sweeps=hsw.ctypes.data_as(C.POINTER(C.c_int64)), history_cap=self.HISTORY_CAP)
        with self._torch.cuda.stream(self.stream):
            st = fn(self._h, C.c_void_p(_ptr(b)), C.c_void_p(_ptr(x)), nrhs, float(tol), C.byref(rep))
        k = rep.history_len
        r = SolveReport(rep.sweeps, rep.outer, rep.checks, rep.relres_max, rep.solve_ms, rel.copy(),
                        rep.sweep_kernel_ms, rep.sweep_launches, (rep.batch_row_tiles, rep.batch_rhs_block),
                        rep.pp_kernel_ms, rep.pp_launches, tuple(rep.pp_shape), hist[:k].copy(), hsw[:k].copy())
        _check(st, r)
        return x, r

    # -- API -------------------------------------------------------------------
    def solve(self, b, tol, x=None):
        """x with A x = b to relative residual tol (vtm_solve)."""
        return self._run(lib().vtm_solve, b, tol, x)

    def solve_noalloc(self, b, tol, x=None):
        """As solve, through vtm_solve_noalloc (no device allocation in the call;
        at most 64 right-hand sides; x should be preallocated by the caller)."""
        return self._run(lib().vtm_solve_noalloc, b, tol, x)

    def solve_adjoint(self, g, tol, lam=None):
        """lambda with A^T lambda = g (vtm_solve_adjoint)."""
        return self._run(lib().vtm_solve_adjoint, g, tol, lam)

    def grad(self, x, lam, branch_ij=None, nnz=None):
        """dL/dg per branch (vtm_grad); branch_ij int32 [m, 2] on the GPU (or None).
        With nnz (the entry count of the A given at setup) also dL/dA per entry of
        that CSR, returned as a second tensor."""
        torch = self._torch
        x = self._vec(x, "x")
        lam = self._vec(lam, "lambda")
        if branch_ij is None:
            ij = torch.zeros((0, 2), dtype=torch.int32, device=x.device)
        else:
            ij = branch_ij.to(device=x.device, dtype=torch.int32).contiguous()
        out = torch.empty(ij.shape[0], dtype=torch.float64, device=x.device)
        dA = torch.empty(int(nnz), dtype=torch.float64, device=x.device) if nnz is not None else None
        _check(lib().vtm_grad(self._h, C.c_void_p(_ptr(x)), C.c_void_p(_ptr(lam)), x.shape[0],
                              C.c_void_p(_ptr(ij)) if ij.shape[0] else None, ij.shape[0],
                              C.c_void_p(_ptr(out)) if ij.shape[0] else None,
                              C.c_void_p(_ptr(dA)) if dA is not None else None))
        return out if dA is None else (out, dA)

    def refresh(self, A, Z=None):
        """New values of A on the pattern given at setup (vtm_refresh): A is a
        scipy CSR with the same rowptr and column arrays, or the new values
        array itself; Z (optional) new line impedances, scalar or per cut wire."""
        import scipy.sparse as sp
        vals = sp.csr_matrix(A).data if sp.issparse(A) else np.asarray(A)
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        if vals.size != self.nnz:
            raise ValueError("A must have the entries of the matrix given at setup")
        if Z is None:
            zp, nz = None, 0
        else:
            z, zp, nz = _z_array(Z)
        _check(lib().vtm_refresh(self._h, vals.ctypes.data_as(C.POINTER(C.c_double)), zp, nz))

    def get_waves(self, nrhs=1):
        w = self._torch.empty((nrhs, 2 * self.n_wires), dtype=self._torch.float64, device="cuda")
        _check(lib().vtm_get_waves(self._h, C.c_void_p(_ptr(w)), nrhs))
        return w

    def set_waves(self, w):
        w = w.contiguous()
        _check(lib().vtm_set_waves(self._h, C.c_void_p(_ptr(w)), w.shape[0]))

    def close(self):
        if getattr(self, "_h", None):
            lib().vtm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
