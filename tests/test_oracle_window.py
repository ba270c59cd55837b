"""Pins of the windowed oracle used for sampled parity at full size: on
workloads small enough for the whole-problem oracle, the window of radius R
around a sub-circuit reproduces that sub-circuit's iterate x^k for every
k <= R + 1 (waves travel one cut wire per sweep), and stops reproducing it one
sweep later, once waves from outside the window would have arrived."""
import numpy as np
import pytest

import oracle
import workloads
from oracle_window import window, window_iterate


def full_iterate(w, k):
    torn = oracle.tear_wires(w.A, w.part, w.Z)
    return oracle.vtm_solve(torn, w.A, w.b, 0.0, max_sweeps=k).x


@pytest.mark.parametrize("cfg,kw,centre,R", [
    (2, dict(dims=(64, 64)), 27, 2),                 # 8 x 8 sub-circuits of 8 x 8
    (3, dict(dims=(24, 24, 24)), 13, 1),             # 3^3 sub-circuits of 8^3, with controlled sources
    (4, dict(dims=(96, 96), nrhs=2), 5, 1),          # uneven random cuts, two right-hand sides
])
def test_window_reproduces_centre_iterates(cfg, kw, centre, R):
    w = workloads.make(cfg, **kw)
    nodes = np.nonzero(w.part == centre)[0]
    for k in range(1, R + 2):
        ref = full_iterate(w, k)[:, nodes]
        x = window_iterate(w, centre, R, k)
        assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max(), k
    # one sweep past the radius, the centre sees waves the window cannot supply
    k = R + 2
    ref = full_iterate(w, k)[:, nodes]
    win = window(w, centre, R)
    torn = oracle.tear_wires(win["A"], win["part"], w.Z)
    x = oracle.vtm_solve(torn, win["A"], win["b"], 0.0, max_sweeps=k).x[:, win["centre_nodes"]]
    assert np.abs(x - ref).max() > 1e-9 * np.abs(ref).max()


def test_window_leaving_wire_is_a_grounded_port():
    """A window that is a single sub-circuit: its first iterate is the local
    solve with every cut wire replaced by G = 2gW/(2g+W) to ground."""
    w = workloads.make(1)
    win = window(w, 5, 0)
    assert win["subs"].tolist() == [5]
    x1 = window_iterate(w, 5, 0, 1)
    nodes = np.nonzero(w.part == 5)[0]
    A = w.A[nodes][:, nodes].toarray()
    W = 1.0 / w.Z
    inside = np.zeros(w.n, bool)
    inside[nodes] = True
    for (i, j), g in zip(w.edges, w.g):
        if inside[i] != inside[j]:
            node = i if inside[i] else j
            loc = np.searchsorted(nodes, node)
            A[loc, loc] += 2 * g * W / (2 * g + W) - g
    ref = np.linalg.solve(A, w.b[0, nodes])
    assert np.allclose(x1[0], ref, rtol=1e-12, atol=0)
