"""Oracle: a plain, slow, FP64 CPU implementation of the Virtual Transmission Method.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the
benchmark's CPU-baseline leg may import, call or execute anything in this
package.  It shares no code with the HIP library (no kernels, headers, helpers,
tables or pre/post-processing); the only thing both sides use is the seeded
input generator in ``workloads``.

Method: F. Wei and H. Yang, "Transmission Line Inspires A New Distributed
Algorithm to Solve the Linear System of Circuit" (arXiv 0910.0663).

* Section V (wire tearing, Steps 1-4; eqs. 6-8): interfacial nodes are split
  into twins; branches and sources at an interfacial node are split between the
  twins; each twin pair is joined by a lossless line.
* Section VI (eqs. 9-14): every sub-circuit solves its own system with the
  line's equivalent circuit (admittance W on the twin, incident wave
  ``W u_other - i_other`` of the previous step as a source); all line delays are
  one step; boundary variables start at zero.
* Section VIII: Schur complements S_i (input admittances) and reflection
  matrices T_i = (W - S_i)(W + S_i)^-1; the convergence factor is
  sqrt(rho(T_1 T_2)).
* Appendix (eqs. 22-30): the iteration's fixed point is the solution of the
  untorn system.

The configurations this library targets partition *nodes* and tear every cut
*branch* ("edge-cut").  The oracle reconciles that with the paper's node
splitting by the exact circuit identity i --g-- j  ==  i --2g-- m --2g-- j: the
new middle node m is the interfacial node of Step 1 (level-one tearing).

Everything is float64.  Sub-circuit solves use a sparse LU of the block-diagonal
matrix of all sub-circuit systems (one library call that solves every
sub-circuit independently; the paper allows any sequential local solver).

Parity status of each function is stated in its docstring; every function is
pinned by the CPU tests in ``tests/test_oracle_*.py`` unless it says
"parity unpinned".
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class UntearableError(ValueError):
    """The partition couples two sub-circuits by something other than a
    two-terminal conductance (a cut cannot be replaced by a line)."""


# --------------------------------------------------------------------------- #
# Wire tearing (Section V)
# --------------------------------------------------------------------------- #
@dataclass
class Torn:
    """A circuit after level-one wire tearing.

    The stacked local vector holds every sub-circuit's unknowns, sub-circuit by
    sub-circuit: its inner nodes, then its twin nodes.
    """
    T: sp.csc_matrix            # block-diagonal sub-circuit matrices, eqs. (7)/(8) (no line terms)
    src: sp.csr_matrix          # local sources f = src @ b   (Step 3 split of the sources)
    out: sp.csr_matrix          # node voltages x = out @ u
    pa: np.ndarray              # position of the side-a twin of every line
    pb: np.ndarray              # position of the side-b twin of every line
    W: np.ndarray               # line admittance: [L] (uncoupled lines) or [L, L] (coupled)
    block_of: np.ndarray        # sub-circuit of every local unknown
    n_blocks: int
    meta: dict = field(default_factory=dict)

    @property
    def n_lines(self) -> int:
        return self.pa.size


def tear_at_vertices(A, label, iface, sides, W, split=0.5) -> Torn:
    """Level-one wire tearing of ``A x = b`` (Section V, Steps 1-4).

    label[v]   sub-circuit of every non-interfacial node (ignored for interface nodes)
    iface      interfacial nodes (Step 1)
    sides      [len(iface), 2]: the two sub-circuits that share each interfacial
               node (level-one: exactly two); side 0 is called "a", side 1 "b"
    W          line admittance: one per interfacial node, or a dense SPD matrix
               over the interfacial nodes (coupled lines, eqs. 4-5)
    split      share of the side-a twin in what Step 3 splits (the interfacial
               node's ground conductance, its source and interface-interface
               branches); the paper's example uses equal halves

    Step 3 reading: a two-terminal branch (A[v,w] == A[w,v] < 0) from an
    interfacial node v to an inner node w is not split: it joins w to the twin
    of v on w's side, and its conductance moves to that twin's diagonal.  What
    is left of A[v,v] (ground) is split.  A one-sided entry (a controlled
    source, A[v,w] or A[w,v] alone) also attaches to the twin on w's side; this
    is how the paper's op-amp example writes eqs. (16)-(17).
    """
    A = sp.csr_matrix(A, dtype=np.float64)
    A.eliminate_zeros()
    n = A.shape[0]
    label = np.asarray(label, dtype=np.int64)
    iface = np.asarray(iface, dtype=np.int64)
    sides = np.asarray(sides, dtype=np.int64).reshape(-1, 2)
    L = iface.size
    is_if = np.zeros(n, dtype=bool)
    is_if[iface] = True
    line_of = -np.ones(n, dtype=np.int64)
    line_of[iface] = np.arange(L)
    n_blocks = int(max(label[~is_if].max(initial=-1), sides.max(initial=-1))) + 1

    # ---- positions in the stacked local vector: inner nodes, then twins ----
    inner_nodes = np.nonzero(~is_if)[0]
    # (block, kind, key) sort: kind 0 = inner (key node id), kind 1 = twin (key line id)
    tw_block = sides.ravel()                                 # twin k = 2*l + s
    tw_line = np.repeat(np.arange(L), 2)
    blk = np.concatenate([label[inner_nodes], tw_block])
    kind = np.concatenate([np.zeros(inner_nodes.size, np.int64), np.ones(2 * L, np.int64)])
    key = np.concatenate([inner_nodes, tw_line])
    order = np.lexsort((key, kind, blk))
    N = order.size
    pos = np.empty(N, dtype=np.int64)
    pos[order] = np.arange(N)
    pos_inner = -np.ones(n, dtype=np.int64)
    pos_inner[inner_nodes] = pos[:inner_nodes.size]
    pos_twin = pos[inner_nodes.size:].reshape(L, 2)          # [line, side]
    block_of = blk[order]

    def twin_on_side_of(v, w):
        """Twin of interfacial node v that lies in the sub-circuit of inner node w."""
        l = line_of[v]
        s = np.where(sides[l, 0] == label[w], 0, np.where(sides[l, 1] == label[w], 1, -1))
        if np.any(s < 0):
            raise UntearableError("interfacial node coupled to a sub-circuit it does not border")
        return pos_twin[l, s]

    coo = A.tocoo()
    r, c, v = coo.row.astype(np.int64), coo.col.astype(np.int64), coo.data
    rows, cols, vals = [], [], []

    # inner-inner entries stay inside their sub-circuit
    m = ~is_if[r] & ~is_if[c]
    if np.any(label[r[m]] != label[c[m]]):
        raise UntearableError("two sub-circuits are coupled directly, not through an interfacial node")
    rows.append(pos_inner[r[m]]); cols.append(pos_inner[c[m]]); vals.append(v[m])

    # interface-row / inner-column and inner-row / interface-column entries
    m = is_if[r] & ~is_if[c]
    rows.append(twin_on_side_of(r[m], c[m])); cols.append(pos_inner[c[m]]); vals.append(v[m])
    m = ~is_if[r] & is_if[c]
    rows.append(pos_inner[r[m]]); cols.append(twin_on_side_of(c[m], r[m])); vals.append(v[m])

    # diagonal of interfacial nodes: branch conductances to each side, plus the split remainder
    Ad = A.diagonal()
    branch_side = np.zeros((L, 2))
    m = is_if[r] & ~is_if[c]
    mirror = np.asarray(A[c[m], r[m]]).ravel()
    twoterm = (mirror == v[m]) & (v[m] < 0)
    lr = line_of[r[m]][twoterm]
    s_of = np.where(sides[lr, 0] == label[c[m]][twoterm], 0, 1)
    np.add.at(branch_side, (lr, s_of), -v[m][twoterm])
    rem = Ad[iface] - branch_side.sum(axis=1)
    diag_tw = branch_side + np.stack([split * rem, (1.0 - split) * rem], axis=1)
    rows.append(pos_twin.ravel()); cols.append(pos_twin.ravel()); vals.append(diag_tw.ravel())

    # interface-interface off-diagonal entries are split between the common sides
    m = is_if[r] & is_if[c] & (r != c)
    if np.any(m):
        lr, lc = line_of[r[m]], line_of[c[m]]
        if np.any(np.sort(sides[lr], axis=1) != np.sort(sides[lc], axis=1)):
            raise UntearableError("interface-interface entry between different side pairs")
        same = sides[lr, 0] == sides[lc, 0]
        for s in (0, 1):
            w_s = split if s == 0 else 1.0 - split
            sc = np.where(same, s, 1 - s)
            rows.append(pos_twin[lr, s]); cols.append(pos_twin[lc, sc]); vals.append(w_s * v[m])

    T = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsc()
    T.sum_duplicates()

    # sources: inner nodes keep theirs, interfacial sources are split (Step 3)
    src_r = np.concatenate([pos_inner[inner_nodes], pos_twin[:, 0], pos_twin[:, 1]])
    src_c = np.concatenate([inner_nodes, iface, iface])
    src_v = np.concatenate([np.ones(inner_nodes.size), np.full(L, split), np.full(L, 1.0 - split)])
    src = sp.csr_matrix((src_v, (src_r, src_c)), shape=(N, n))

    # node voltages: inner nodes directly, interfacial nodes as the mean of their twins
    out_r = np.concatenate([inner_nodes, iface, iface])
    out_c = np.concatenate([pos_inner[inner_nodes], pos_twin[:, 0], pos_twin[:, 1]])
    out_v = np.concatenate([np.ones(inner_nodes.size), np.full(2 * L, 0.5)])
    out = sp.csr_matrix((out_v, (out_r, out_c)), shape=(n, N))

    W = np.asarray(W, dtype=np.float64)
    if W.ndim == 0:
        W = np.full(L, float(W))
    return Torn(T=T, src=src, out=out, pa=pos_twin[:, 0].copy(), pb=pos_twin[:, 1].copy(),
                W=W, block_of=block_of, n_blocks=n_blocks)


def cut_wires(A, part):
    """Branches cut by a node partition, in canonical order (i < j ascending).

    Every pair of nodes in different sub-circuits must be coupled by a
    two-terminal conductance, A[i, j] == A[j, i] < 0, so that it can be torn
    into a line; anything else raises :class:`UntearableError`.
    Returns (i, j, g) with g = -A[i, j].
    """
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    part = np.asarray(part)
    coo = A.tocoo()
    m = part[coo.row] != part[coo.col]
    r, c, v = coo.row[m].astype(np.int64), coo.col[m].astype(np.int64), coo.data[m]
    up = r < c
    lo = ~up
    ku = r[up] * A.shape[0] + c[up]
    kl = c[lo] * A.shape[0] + r[lo]
    ou, ol = np.argsort(ku), np.argsort(kl)
    if ku.size != kl.size or np.any(ku[ou] != kl[ol]) or np.any(v[up][ou] != v[lo][ol]):
        raise UntearableError("cross-partition coupling is not symmetric")
    g = -v[up][ou]
    if np.any(g <= 0):
        raise UntearableError("cross-partition coupling is not a positive conductance")
    return r[up][ou], c[up][ou], g


def expand_midpoints(A, wires):
    """Replace every cut branch i --g-- j by i --2g-- m --2g-- j with a new node m
    (no ground, no source).  Exact: eliminating m gives back g between i and j.
    Returns the (n + n_wires) square matrix; node n + e is the middle of wire e."""
    A = sp.csr_matrix(A, dtype=np.float64)
    n = A.shape[0]
    i, j, g = wires
    k = i.size
    mid = n + np.arange(k)
    rows = [i, j, i, j, i, mid, j, mid, mid]
    cols = [j, i, i, j, mid, i, mid, j, mid]
    vals = [g, g, g, g, -2 * g, -2 * g, -2 * g, -2 * g, 4 * g]
    D = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n + k, n + k))
    Aexp = sp.bmat([[A, None], [None, sp.csr_matrix((k, k))]]).tocsr() + D.tocsr()
    Aexp.eliminate_zeros()
    return Aexp.tocsr()


def tear_wires(A, part, Z, color=None) -> Torn:
    """Tear every branch cut by the node partition ``part`` into a lossless line
    of impedance Z (scalar, or one per cut wire in canonical order).

    Each cut branch is first split at its middle (:func:`expand_midpoints`); the
    middle node is the interfacial node, shared by exactly two sub-circuits
    (level-one tearing).  Side a of a line is the sub-circuit of its lower node,
    or the colour-0 sub-circuit when a 2-colouring ``color[sub]`` is given.
    """
    part = np.asarray(part, dtype=np.int64)
    n = A.shape[0]
    wires = cut_wires(A, part)
    i, j, g = wires
    Aexp = expand_midpoints(A, wires)
    k = i.size
    label = np.concatenate([part, -np.ones(k, np.int64)])
    sides = np.stack([part[i], part[j]], axis=1)
    if color is not None:
        color = np.asarray(color)
        flip = color[sides[:, 0]] != 0
        sides[flip] = sides[flip][:, ::-1]
    Z = np.asarray(Z, dtype=np.float64)
    W = 1.0 / (np.full(k, float(Z)) if Z.ndim == 0 else Z)
    torn = tear_at_vertices(Aexp, label, n + np.arange(k), sides, W, split=0.5)
    torn.src = torn.src[:, :n].tocsr()
    torn.out = torn.out[:n, :].tocsr()
    torn.meta.update(wires=wires, n=n)
    return torn


# --------------------------------------------------------------------------- #
# The iteration (Section VI)
# --------------------------------------------------------------------------- #
def line_matrix(torn: Torn) -> sp.csc_matrix:
    """Sub-circuit matrices with each line's equivalent circuit: admittance W on
    its twins (the ``C + W`` block of eqs. 10-11 and 13-14)."""
    T = torn.T.tocoo()
    rows, cols, vals = [T.row], [T.col], [T.data]
    W = torn.W
    for p in (torn.pa, torn.pb):
        if W.ndim == 1:
            rows.append(p); cols.append(p); vals.append(W)
        else:
            rr, cc = np.meshgrid(p, p, indexing="ij")
            rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(W.ravel())
    N = torn.T.shape[0]
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsc()
    M.sum_duplicates()
    return M


def _wmul(W, u):
    return W[:, None] * u if W.ndim == 1 else W @ u


@dataclass
class Result:
    x: np.ndarray                   # node voltages [nrhs, n]
    sweeps: int
    status: str                     # "ok" | "diverged" | "maxiter"
    relres: np.ndarray              # final relative residual per column
    history: list                   # max relative residual after every sweep
    waves: Optional[np.ndarray] = None


class Sweeper:
    """Runs VTM sweeps on a torn circuit: each sweep solves every sub-circuit
    with the incident waves of the previous sweep, then sends each twin's
    outgoing wave down its line (eqs. 11 and 14, all delays equal to 1)."""

    def __init__(self, torn: Torn):
        self.torn = torn
        self.lu = spla.splu(line_matrix(torn), permc_spec="COLAMD")

    def sweep(self, f, a):
        """f: local sources [N, k]; a: incident waves [2, L, k] (into side a, side b).
        Returns local voltages u [N, k] and the next incident waves."""
        t = self.torn
        rhs = f.copy()
        rhs[t.pa] += a[0]
        rhs[t.pb] += a[1]
        u = self.lu.solve(rhs)
        ua, ub = u[t.pa], u[t.pb]
        # line currents into the twins: i = -W u + (W u_other - i_other)_{k-1}
        ia = a[0] - _wmul(t.W, ua)
        ib = a[1] - _wmul(t.W, ub)
        # what leaves each twin, W u - i, reaches the other twin one step later
        a_next = np.stack([_wmul(t.W, ub) - ib, _wmul(t.W, ua) - ia])
        return u, a_next


def relative_residual(A, b, x):
    """||b - A x||_2 / ||b||_2 per column ([k, n] arrays); ||b - A x|| when b = 0."""
    r = b - (A @ x.T).T
    rn = np.linalg.norm(r, axis=1)
    bn = np.linalg.norm(b, axis=1)
    return np.where(bn > 0, rn / np.where(bn > 0, bn, 1.0), rn)


def vtm_solve(torn: Torn, A, b, tol, max_sweeps=100000, diverge=1e6, a0=None,
              sweeper: Optional[Sweeper] = None) -> Result:
    """Synchronous VTM from zero boundary variables (Section VI) until every
    column satisfies ||b - A x||_2 / ||b||_2 <= tol on the untorn A, checked
    after every sweep.  Diverged = a non-finite residual or one above
    ``diverge``; maxiter = ``max_sweeps`` sweeps without convergence."""
    b = np.atleast_2d(np.asarray(b, dtype=np.float64))
    sw = sweeper or Sweeper(torn)
    f = (torn.src @ b.T)
    L, k = torn.n_lines, b.shape[0]
    a = np.zeros((2, L, k)) if a0 is None else np.array(a0, dtype=np.float64).reshape(2, L, k)
    x = np.zeros_like(b)
    rel = relative_residual(A, b, x)
    hist = []
    if np.all(rel <= tol):
        return Result(x, 0, "ok", rel, hist, a)
    for s in range(1, max_sweeps + 1):
        u, a = sw.sweep(f, a)
        x = (torn.out @ u).T
        rel = relative_residual(A, b, x)
        hist.append(float(rel.max()))
        if not np.all(np.isfinite(rel)) or rel.max() > diverge:
            return Result(x, s, "diverged", rel, hist, a)
        if np.all(rel <= tol):
            return Result(x, s, "ok", rel, hist, a)
    return Result(x, max_sweeps, "maxiter", rel, hist, a)


def sweep_operator(torn: Torn) -> np.ndarray:
    """The linear map from the incident waves of one sweep to those of the next
    (sources zero), as a dense [2L, 2L] matrix over (side a lines, side b lines).
    Small problems only."""
    sw = Sweeper(torn)
    L = torn.n_lines
    N = torn.T.shape[0]
    E = np.eye(2 * L).reshape(2, L, 2 * L)
    _, a_next = sw.sweep(np.zeros((N, 2 * L)), E)
    return a_next.reshape(2 * L, 2 * L)


# --------------------------------------------------------------------------- #
# Input admittances and reflection matrices (Section VIII, Appendix eqs. 22-30)
# --------------------------------------------------------------------------- #
def interface_schur(torn: Torn, side: int) -> np.ndarray:
    """S = C - E D^-1 F of the sub-circuits holding the twins of one side
    (Example 3), over those twins in line order; the line terms are excluded.
    Needs every sub-circuit to hold twins of one side only (a 2-coloured tear)."""
    P = torn.pa if side == 0 else torn.pb
    other = torn.pb if side == 0 else torn.pa
    blocks = np.unique(torn.block_of[P])
    if np.intersect1d(blocks, torn.block_of[other]).size:
        raise ValueError("sub-circuits hold twins of both sides; tear with a 2-colouring")
    in_side = np.isin(torn.block_of, blocks)
    is_tw = np.zeros(torn.T.shape[0], dtype=bool)
    is_tw[P] = True
    inner = np.nonzero(in_side & ~is_tw)[0]
    T = torn.T.tocsr()
    C = T[P][:, P].toarray()
    if inner.size == 0:
        return C
    E = T[P][:, inner].toarray()
    F = T[inner][:, P].toarray()
    D = T[inner][:, inner].toarray()
    return C - E @ np.linalg.solve(D, F)


def partial_schur(torn: Torn, side: int, depth=None, drop: float = 0.0) -> np.ndarray:
    """Rule 5 of Section VIII, the Schur complement approximation: for every
    group of lines whose twins lie in the same two sub-circuits (in the same
    order), W_group = C - E~ D~^-1 F~ over the twins of one side, where D~ keeps
    only the inner nodes of that side's sub-circuit within ``depth`` hops of
    those twins (in the torn matrix's graph; None keeps them all, which gives
    the exact Schur complement S of Example 3, 0 keeps none, giving C).

    Readings where the paper is silent: the submatrix is chosen by graph
    distance from the interface; the result is symmetrized, (S~ + S~^T) / 2;
    "dropping the small elements" sets an off-diagonal entry to zero when
    |w_ij| < drop * sqrt(|w_ii w_jj|).  Returns a dense [L, L] matrix (zero
    between lines of different groups)."""
    P = torn.pa if side == 0 else torn.pb
    L = P.size
    N = torn.T.shape[0]
    T = torn.T.tocsr()
    G = (abs(T) + abs(T).T).tocsr()                     # adjacency, both directions
    is_twin = np.zeros(N, dtype=bool)
    is_twin[torn.pa] = True
    is_twin[torn.pb] = True
    W = np.zeros((L, L))
    key = np.stack([torn.block_of[torn.pa], torn.block_of[torn.pb]], axis=1)
    _, group = np.unique(key, axis=0, return_inverse=True)
    for g in np.unique(group):
        lines = np.nonzero(group == g)[0]
        Pg = P[lines]
        blk = torn.block_of[Pg[0]]
        inner_ok = (torn.block_of == blk) & ~is_twin
        # breadth-first search from the twins over inner nodes of the sub-circuit
        chosen = np.zeros(N, dtype=bool)
        frontier = Pg
        hop = 0
        while frontier.size and (depth is None or hop < depth):
            nb = np.unique(G[frontier].indices)
            nb = nb[inner_ok[nb] & ~chosen[nb]]
            chosen[nb] = True
            frontier = nb
            hop += 1
        Dn = np.nonzero(chosen)[0]
        C = T[Pg][:, Pg].toarray()
        if Dn.size:
            E = T[Pg][:, Dn].toarray()
            F = T[Dn][:, Pg].toarray()
            D = T[Dn][:, Dn].toarray()
            S = C - E @ np.linalg.solve(D, F)
        else:
            S = C
        S = 0.5 * (S + S.T)
        if drop > 0.0:
            d = np.sqrt(np.abs(np.diag(S)))
            small = np.abs(S) < drop * np.outer(d, d)
            np.fill_diagonal(small, False)
            S[small] = 0.0
        W[np.ix_(lines, lines)] = S
    return W


def reflection(S: np.ndarray, W) -> np.ndarray:
    """Voltage reflection matrix T = (W - S)(W + S)^-1 (Section VIII)."""
    Wm = np.diag(W) if np.ndim(W) == 1 else np.asarray(W)
    return (Wm - S) @ np.linalg.inv(Wm + S)


def spectral_radius(M) -> float:
    return float(np.max(np.abs(np.linalg.eigvals(M)))) if np.size(M) else 0.0


# --------------------------------------------------------------------------- #
# Eliminated-twin form: what a per-subdomain kernel applies (derived independently)
# --------------------------------------------------------------------------- #
@dataclass
class Eliminated:
    """Tear of a node partition with the twin of every cut wire eliminated.

    For a cut wire of conductance g and line admittance W, the twin equation
    2g (v - u_i) + W v = a gives v = (2g u_i + a) / (2g + W).  Substituted in
    node i's row, the cut branch g becomes a port conductance G = 2gW/(2g+W) on
    the diagonal and the incident wave enters the right-hand side as c*a with
    c = 2g/(2g+W).  The outgoing wave W v - i = 2W v - a becomes
    beta*u_i + gamma*a with beta = 4gW/(2g+W), gamma = (W - 2g)/(2g+W).
    """
    subs: list            # per sub-circuit: node ids (ascending)
    K: list               # per sub-circuit: dense local matrix
    port_node: np.ndarray  # owner node of each port (port 2e: lower node of wire e, 2e+1: upper)
    c: np.ndarray
    beta: np.ndarray
    gamma: np.ndarray
    G: np.ndarray
    g: np.ndarray          # conductance of the port's cut wire


def eliminate_twins(A, part, Z) -> Eliminated:
    A = sp.csr_matrix(A, dtype=np.float64)
    part = np.asarray(part, dtype=np.int64)
    i, j, g = cut_wires(A, part)
    Z = np.asarray(Z, dtype=np.float64)
    W = 1.0 / (np.full(i.size, float(Z)) if Z.ndim == 0 else Z)
    G = 2 * g * W / (2 * g + W)
    c = 2 * g / (2 * g + W)
    beta = 4 * g * W / (2 * g + W)
    gamma = (W - 2 * g) / (2 * g + W)
    port_node = np.stack([i, j], axis=1).ravel()
    dmod = np.zeros(A.shape[0])
    np.add.at(dmod, i, G - g)
    np.add.at(dmod, j, G - g)
    subs, K = [], []
    for s in range(int(part.max()) + 1):
        nodes = np.nonzero(part == s)[0]
        Ks = A[nodes][:, nodes].toarray()
        Ks[np.diag_indices_from(Ks)] += dmod[nodes]
        subs.append(nodes)
        K.append(Ks)
    rep = lambda v: np.repeat(v, 2)
    return Eliminated(subs=subs, K=K, port_node=port_node, c=rep(c), beta=rep(beta),
                      gamma=rep(gamma), G=rep(G), g=rep(g))


def vtm_solve_eliminated(el: Eliminated, A, b, n_sweeps, waves=None):
    """Run ``n_sweeps`` sweeps of the eliminated-twin form from zero waves; returns
    the iterates x^1..x^n (one column right-hand side).  A list passed as
    ``waves`` receives, per sweep, the incident and outgoing wave of every port."""
    b = np.asarray(b, dtype=np.float64).ravel()
    n = b.size
    P = el.port_node.size
    a = np.zeros(P)                # incident wave at every port
    twin = np.arange(P) ^ 1
    xs = []
    for _ in range(n_sweeps):
        rhs = b.copy()
        np.add.at(rhs, el.port_node, el.c * a)
        x = np.empty(n)
        for nodes, Ks in zip(el.subs, el.K):
            x[nodes] = np.linalg.solve(Ks, rhs[nodes])
        out = el.beta * x[el.port_node] + el.gamma * a
        if waves is not None:
            waves.append((a, out))
        a = out[twin]
        xs.append(x)
    return xs


def interface_residual(el: Eliminated, n, a, out):
    """b - A x^k of the eliminated form's iterate, from port quantities alone.

    Each local solve satisfies its sub-circuit's rows of K x = b + sum c a, and
    K differs from A's diagonal block only by G - g at port nodes, while the
    only couplings of A across sub-circuits are the cut wires (-g to the far
    node j).  So row i of b - A x vanishes off the port nodes, and at a port
    node it is the sum over its ports of (G - g) x_i + g x_j - c a.  The node
    voltages follow from the waves of the same sweep (out = beta x_i + gamma a):
    x_i = (out_p - gamma_p a_p) / beta_p, and x_j from the twin port.
    ``a``/``out``: incident and outgoing waves of every port in that sweep."""
    twin = np.arange(el.port_node.size) ^ 1
    xi = (out - el.gamma * a) / el.beta
    d = (el.G - el.g) * xi + el.g * xi[twin] - el.c * a
    r = np.zeros(n)
    np.add.at(r, el.port_node, d)
    return r


# --------------------------------------------------------------------------- #
# Direct solves, refinement, adjoint and gradients
# --------------------------------------------------------------------------- #
def direct_solve(A, b):
    """x* = A^-1 b by sparse LU of the untorn matrix (the VTM fixed point)."""
    b = np.atleast_2d(np.asarray(b, dtype=np.float64))
    lu = spla.splu(sp.csc_matrix(A, dtype=np.float64))
    return lu.solve(b.T).T


def direct_adjoint(A, g):
    """lambda = A^-T g by sparse LU."""
    return direct_solve(sp.csr_matrix(A).T, g)


@dataclass
class RefineResult:
    x: np.ndarray
    outer: int
    inner_sweeps: list
    relres: np.ndarray
    status: str


def vtm_refine(torn: Torn, A, b, tol, inner_drop, max_outer=60, max_inner=100000,
               check_every=8, sweeper: Optional[Sweeper] = None) -> RefineResult:
    """Iterative refinement around VTM (not in the paper; the schedule the
    library uses for its low-precision forms): r = b - A x; an inner VTM on
    A d = r from zero waves, its residual ||r - A d|| / ||r|| checked every
    ``check_every`` sweeps, stops when every column is below
    max(inner_drop, tol ||b|| / (2 ||r||)) or when two checks in a row bring no
    column 20% below its best; then x += d; until ||b - A x|| / ||b|| <= tol.
    The oracle runs the inner solves in FP64 (the schedule, not the precision,
    is what it reproduces).  Pinned by rebuilding its steps from plain VTM on
    each residual (the same stopping sweeps and iterates), and by the final
    residual and the direct solution it must agree with."""
    b = np.atleast_2d(np.asarray(b, dtype=np.float64))
    sw = sweeper or Sweeper(torn)
    x = np.zeros_like(b)
    inner = []
    L, k = torn.n_lines, b.shape[0]
    for outer in range(max_outer + 1):
        rel = relative_residual(A, b, x)
        if np.all(rel <= tol):
            return RefineResult(x, outer, inner, rel, "ok")
        if outer == max_outer:
            break
        target = np.maximum(inner_drop, 0.5 * tol / np.where(rel > 0, rel, 1.0))
        r = b - (A @ x.T).T
        rn = np.linalg.norm(r, axis=1)
        f = torn.src @ r.T
        a = np.zeros((2, L, k))
        best, since, d = np.full(k, np.inf), 0, np.zeros_like(b)
        for s in range(1, max_inner + 1):
            u, a = sw.sweep(f, a)
            if s % check_every and s != max_inner:
                continue
            d = (torn.out @ u).T
            e = np.linalg.norm(r - (A @ d.T).T, axis=1) / np.where(rn > 0, rn, 1.0)
            improved = np.any(e < 0.8 * best)
            best = np.minimum(best, e)
            since = 0 if improved else since + 1
            if np.all(e <= target) or since >= 2:
                break
        inner.append(s)
        x = x + d
    return RefineResult(x, max_outer, inner, relative_residual(A, b, x), "maxiter")


def branch_gradient(edges, x, lam):
    """dL/dg for every branch (i, j) of conductance g, from A x = b and
    A^T lambda = dL/dx:  dL/dg = -(lambda_i - lambda_j)(x_i - x_j), summed over
    right-hand sides ([k, n] arrays)."""
    x = np.atleast_2d(x)
    lam = np.atleast_2d(lam)
    i, j = edges[:, 0], edges[:, 1]
    return -np.sum((lam[:, i] - lam[:, j]) * (x[:, i] - x[:, j]), axis=0)


def matrix_gradient(A, x, lam):
    """dL/dA for every stored entry of A, in A's CSR entry order, from A x = b and
    A^T lambda = dL/dx: perturbing one entry a_ij moves x by -A^-1 e_i x_j, so
    dL/da_ij = -lambda_i x_j, summed over right-hand sides ([k, n] arrays).  A
    controlled source of gain g_m at (k, c) is such an entry (Section IX, eq.
    15).  Not in the paper (the differentiation the library adds); pinned by
    central differences of the loss through direct solves."""
    A = sp.csr_matrix(A)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    x = np.atleast_2d(x)
    lam = np.atleast_2d(lam)
    return -np.sum(lam[:, rows] * x[:, A.indices], axis=0)


# --------------------------------------------------------------------------- #
# Classical stationary methods (only to show where they fail, Section IX)
# --------------------------------------------------------------------------- #
def jacobi_matrix(A) -> np.ndarray:
    A = np.asarray(sp.csr_matrix(A).toarray())
    D = np.diag(np.diag(A))
    return -np.linalg.solve(D, A - D)


def gauss_seidel_matrix(A) -> np.ndarray:
    A = np.asarray(sp.csr_matrix(A).toarray())
    L = np.tril(A)
    return -np.linalg.solve(L, A - L)
