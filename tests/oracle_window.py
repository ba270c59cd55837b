"""Windowed oracle problems: the oracle's iterate on a few sampled sub-circuits
of a workload too large for the oracle as a whole (test infrastructure; oracle
side only).

x^k on a sub-circuit depends only on the sub-circuits within k - 1 hops of it
in the graph whose edges are the cut wires: the first sweep is local (every
incident wave is zero, Section VI), and each later sweep carries waves one
wire further (eq. 5 with unit delay).  A window holding every sub-circuit
within R hops of a centre therefore reproduces the centre's x^k for k <= R + 1,
provided each wire that leaves the window keeps the port it has in the whole
problem.  With its incident wave held at zero, such a port is a conductance
G = 2 g W / (2 g + W) from its node to ground (the line's twin, tied to the
node by 2 g and to ground by W, eliminated), so the window's nodal matrix
carries G - g on that node's diagonal in place of the dropped branch.
"""
from collections import deque

import numpy as np

import oracle


def window(w, centre, R):
    """Nodes (sorted global ids), nodal matrix, right-hand sides and relabelled
    partition of the window of radius ``R`` hops around sub-circuit ``centre``."""
    part = np.asarray(w.part, dtype=np.int64)
    e = np.asarray(w.edges, dtype=np.int64)
    pi, pj = part[e[:, 0]], part[e[:, 1]]
    cut = pi != pj
    nbr = {}
    for a, b in zip(pi[cut], pj[cut]):
        nbr.setdefault(int(a), set()).add(int(b))
        nbr.setdefault(int(b), set()).add(int(a))
    hops = {int(centre): 0}
    todo = deque([int(centre)])
    while todo:
        s = todo.popleft()
        if hops[s] == R:
            continue
        for t in nbr.get(s, ()):
            if t not in hops:
                hops[t] = hops[s] + 1
                todo.append(t)
    inside = np.zeros(w.n_sub, dtype=bool)
    inside[list(hops)] = True
    nodes = np.nonzero(inside[part])[0]
    local = -np.ones(w.n, dtype=np.int64)
    local[nodes] = np.arange(nodes.size)
    A = w.A[nodes][:, nodes].tolil()
    W = 1.0 / w.Z
    ii, jj = inside[part[e[:, 0]]], inside[part[e[:, 1]]]
    for side, other, leaving in ((0, 1, ii & ~jj), (1, 0, jj & ~ii)):
        for node, g in zip(e[leaving, side], w.g[leaving]):
            G = 2.0 * g * W / (2.0 * g + W)
            A[local[node], local[node]] += G - g
    labels, part_w = np.unique(part[nodes], return_inverse=True)
    return dict(nodes=nodes, A=A.tocsr(), b=w.b[:, nodes], part=part_w.astype(np.int32), subs=labels,
                centre_nodes=local[np.nonzero(part == centre)[0]])


def window_iterate(w, centre, R, k, b=None):
    """The oracle's x^k on the nodes of sub-circuit ``centre`` (global order of
    those nodes), from the window of radius R; requires k <= R + 1."""
    assert k <= R + 1, "the window is exact only for k <= R + 1"
    win = window(w, centre, R)
    bb = win["b"] if b is None else b[:, win["nodes"]]
    torn = oracle.tear_wires(win["A"], win["part"], w.Z)
    r = oracle.vtm_solve(torn, win["A"], bb, 0.0, max_sweeps=k)
    assert r.sweeps == k
    return r.x[:, win["centre_nodes"]]
