"""Differentiation through a VTM solve: ``VTMSolve.apply(b, g, circuit)``.

Forward: build the nodal matrix of the circuit for branch conductances g,
tear and factor it (vtm_setup, only when g changed) and solve A x = b
(vtm_solve).  Backward: lambda = A^-T dL/dx by VTM on the torn A^T with the
same stored inverses (vtm_solve_adjoint); dL/db = lambda and
dL/dg_e = -(lambda_i - lambda_j)(x_i - x_j) (vtm_grad).
"""
from __future__ import annotations

import numpy as np
import torch

import scipy.sparse as sp

from .binding import Solver


def nodal_matrix(n, edges, g, ground, vccs=None):
    """Nodal-analysis matrix of a current-driven circuit (Section II, eq. 1): a
    branch of conductance g between i and j stamps +g on A_ii and A_jj and -g on
    A_ij and A_ji; a conductance to ground stamps the diagonal; a voltage-
    controlled current source (k, c, gain) stamps the single entry A_kc (the
    op-amp example, eq. 15).  CSR with sorted columns, duplicates summed."""
    edges = np.asarray(edges, dtype=np.int64)
    i, j = edges[:, 0], edges[:, 1]
    g = np.asarray(g, dtype=np.float64)
    diag = np.arange(n)
    rows = [i, j, i, j, diag]
    cols = [i, j, j, i, diag]
    vals = [g, g, -g, -g, np.asarray(ground, dtype=np.float64)]
    if vccs is not None:
        k, c, gm = vccs
        rows.append(np.asarray(k))
        cols.append(np.asarray(c))
        vals.append(np.asarray(gm, dtype=np.float64))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


class Circuit:
    """Grid-like circuit structure: branches, ground conductances, partition, line impedance."""

    def __init__(self, n, edges, ground, part, Z, tol=1e-8, precision="fp32_refine", vccs=None,
                 **solver_kw):
        self.n = int(n)
        self.edges = np.asarray(edges, dtype=np.int64)
        self.ground = np.asarray(ground, dtype=np.float64)
        self.part = np.asarray(part, dtype=np.int32)
        self.Z = Z
        self.tol = float(tol)
        self.precision = precision
        self.vccs = vccs
        self.solver_kw = solver_kw
        self._key = None
        self._solver = None
        self._ij = None
        self.last_forward = None
        self.last_adjoint = None

    def solver(self, g: torch.Tensor) -> Solver:
        """The handle for conductances g: set up once, then refreshed in place
        (vtm_refresh: same pattern and partition, no new tearing plan) whenever g
        changes."""
        gh = g.detach().to("cpu", torch.float64).numpy()
        key = gh.tobytes()
        if key != self._key:
            A = nodal_matrix(self.n, self.edges, gh, self.ground, self.vccs)
            if self._solver is None:
                self._solver = Solver(A, self.part, self.Z, precision=self.precision, **self.solver_kw)
            else:
                self._solver.refresh(A)
            self._key = key
        return self._solver

    def branch_ij(self, device) -> torch.Tensor:
        if self._ij is None or self._ij.device != device:
            self._ij = torch.as_tensor(self.edges.astype(np.int32), device=device)
        return self._ij


class VTMSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, g, circuit: Circuit):
        solver = circuit.solver(g)
        x, rep = solver.solve(b.detach(), circuit.tol)
        circuit.last_forward = rep
        ctx.circuit = circuit
        ctx.solver = solver
        ctx.b_shape = b.shape
        ctx.save_for_backward(x)
        return x.reshape(b.shape)

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        solver, circuit = ctx.solver, ctx.circuit
        gx = gx.reshape(x.shape).to(torch.float64).contiguous()
        lam, rep = solver.solve_adjoint(gx, circuit.tol)
        circuit.last_adjoint = rep
        grad_b = lam.reshape(ctx.b_shape) if ctx.needs_input_grad[0] else None
        grad_g = solver.grad(x, lam, circuit.branch_ij(x.device)) if ctx.needs_input_grad[1] else None
        return grad_b, grad_g, None
