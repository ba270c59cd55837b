"""Synthetic resistor-grid circuits: the stand-ins for the structured test matrices
(Grid2d, Grid3d) of the paper's experiments (Section X, Table I), sized to the
five workloads this library is measured on.

A circuit here is a current-driven resistor network (Section II): branch
conductances on the edges of a 2-D 5-point or 3-D 7-point grid, a conductance
to ground at every node (so that ``A`` is SPD by Lemma 1), independent current
sources ``b`` and, for the unsymmetric workload, voltage-controlled current
sources stamped as single matrix entries the way the paper's op-amp example
(eq. 15) writes them.

Every random draw comes from ``numpy.random.default_rng(seed)`` in one fixed
order: branch conductances (canonical edge order) -> right-hand sides ->
controlled sources -> random cuts -> probe nodes.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp

GROUND_S = 0.01  # conductance to ground at every node, siemens


# --------------------------------------------------------------------------- #
# Grid graphs
# --------------------------------------------------------------------------- #
def grid2d_edges(ny: int, nx: int) -> np.ndarray:
    """Edges of an ny x nx 5-point grid, node id = row * nx + col.

    Returned as int64 [m, 2] with i < j, sorted by (i, j) ascending (the
    canonical edge order all conductance draws follow).
    """
    ids = np.arange(ny * nx, dtype=np.int64).reshape(ny, nx)
    right = np.stack([ids[:, :-1].ravel(), ids[:, 1:].ravel()], axis=1)
    down = np.stack([ids[:-1, :].ravel(), ids[1:, :].ravel()], axis=1)
    e = np.concatenate([right, down], axis=0)
    order = np.lexsort((e[:, 1], e[:, 0]))
    return np.ascontiguousarray(e[order])


def grid3d_edges(nz: int, ny: int, nx: int) -> np.ndarray:
    """Edges of an nz x ny x nx 7-point grid, node id = (z * ny + y) * nx + x,
    canonical order as in :func:`grid2d_edges`."""
    ids = np.arange(nz * ny * nx, dtype=np.int64).reshape(nz, ny, nx)
    ex = np.stack([ids[:, :, :-1].ravel(), ids[:, :, 1:].ravel()], axis=1)
    ey = np.stack([ids[:, :-1, :].ravel(), ids[:, 1:, :].ravel()], axis=1)
    ez = np.stack([ids[:-1, :, :].ravel(), ids[1:, :, :].ravel()], axis=1)
    e = np.concatenate([ex, ey, ez], axis=0)
    order = np.lexsort((e[:, 1], e[:, 0]))
    return np.ascontiguousarray(e[order])


def nodal_matrix(n: int, edges: np.ndarray, g: np.ndarray, ground: np.ndarray,
                 vccs: Optional[tuple] = None) -> sp.csr_matrix:
    """Nodal-analysis matrix of a current-driven circuit (Section II, eq. 1).

    A branch of conductance g between i and j stamps +g on both diagonals and
    -g on (i, j) and (j, i); a ground conductance stamps the diagonal; a
    voltage-controlled current source (k, c, gm) stamps the single entry
    A[k, c] += gm.  Returns CSR with sorted column indices, duplicates summed.
    """
    i, j = edges[:, 0], edges[:, 1]
    rows = [i, j, i, j, np.arange(n)]
    cols = [i, j, j, i, np.arange(n)]
    vals = [g, g, -g, -g, np.asarray(ground, dtype=np.float64)]
    if vccs is not None:
        k, c, gm = vccs
        rows.append(k)
        cols.append(c)
        vals.append(gm)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


# --------------------------------------------------------------------------- #
# Partitions
# --------------------------------------------------------------------------- #
def _axis_labels(length: int, widths) -> np.ndarray:
    lab = np.empty(length, dtype=np.int64)
    pos = 0
    for k, w in enumerate(widths):
        lab[pos:pos + w] = k
        pos += w
    assert pos == length
    return lab


def block_partition_2d(ny: int, nx: int, by, bx) -> np.ndarray:
    """Tensor-product partition of a 2-D grid into rectangles.

    ``by``/``bx`` are either a block size (int) or an explicit list of widths.
    Label = block_row * n_block_cols + block_col (row-major over blocks).
    """
    wy = _widths(ny, by)
    wx = _widths(nx, bx)
    ly = _axis_labels(ny, wy)
    lx = _axis_labels(nx, wx)
    return (ly[:, None] * len(wx) + lx[None, :]).ravel().astype(np.int32)


def block_partition_3d(nz: int, ny: int, nx: int, bz: int, by: int, bx: int) -> np.ndarray:
    wz, wy, wx = _widths(nz, bz), _widths(ny, by), _widths(nx, bx)
    lz, ly, lx = _axis_labels(nz, wz), _axis_labels(ny, wy), _axis_labels(nx, wx)
    lab = (lz[:, None, None] * len(wy) + ly[None, :, None]) * len(wx) + lx[None, None, :]
    return lab.ravel().astype(np.int32)


def separator_strips(dims, width: int):
    """Node separators for tearing at interfacial nodes (Section V, Step 1):
    the grid (2-D or 3-D, node numbering as in :func:`grid2d_edges` /
    :func:`grid3d_edges`) is cut along its last axis into strips (slabs) of
    ``width`` inner layers, consecutive strips divided by one layer of
    interfacial nodes (the last strip takes what is left, and one more layer
    when a single layer would remain).  Every interfacial
    node borders exactly the two strips on either side of its layer.

    Returns ``label`` (int32 [n]: strip of every inner node, -1 on separator
    layers), ``iface`` (int32, ascending node ids) and ``sides`` (int32
    [len(iface), 2]: the strips before and after the node's layer)."""
    dims = tuple(int(d) for d in dims)
    nx = dims[-1]
    lay = np.full(nx, -1, dtype=np.int64)     # strip of each layer, -1 for a separator
    sep_of = np.full(nx, -1, dtype=np.int64)  # index of each separator layer
    x, strip, sep = 0, 0, 0
    while x < nx:
        w = min(width, nx - x)
        if nx - (x + w) == 1:                 # a lone last layer joins this strip
            w += 1
        lay[x:x + w] = strip
        x += w
        if x < nx:                            # at least two layers left: separator, strip
            sep_of[x] = sep
            sep += 1
            x += 1
        strip += 1
    xs = np.broadcast_to(np.arange(nx), dims).ravel()
    label = lay[xs].astype(np.int32)
    iface = np.nonzero(label < 0)[0].astype(np.int32)
    k = sep_of[xs[iface]]
    sides = np.stack([k, k + 1], axis=1).astype(np.int32)
    return label, iface, sides


def _widths(length: int, b):
    if isinstance(b, (int, np.integer)):
        full, rest = divmod(length, int(b))
        return [int(b)] * full + ([rest] if rest else [])
    w = [int(v) for v in b]
    assert sum(w) == length
    return w


def random_cut_widths(rng: np.random.Generator, length: int, wmin: int = 8, wmax: int = 24):
    """Random 1-D cut: while more than ``wmax`` nodes remain, draw a width
    uniformly from {wmin, ..., min(wmax, remaining - wmin)}; the rest is the last
    piece (so every piece lies in [wmin, wmax])."""
    widths = []
    rem = length
    while rem > wmax:
        w = int(rng.integers(wmin, min(wmax, rem - wmin) + 1))
        widths.append(w)
        rem -= w
    widths.append(rem)
    return widths


# --------------------------------------------------------------------------- #
# Workloads
# --------------------------------------------------------------------------- #
@dataclass
class Workload:
    name: str
    dims: tuple                      # grid shape, slowest axis first
    A: sp.csr_matrix                 # nodal matrix, float64, n x n
    b: np.ndarray                    # right-hand sides, float64 [nrhs, n]
    part: np.ndarray                 # subdomain label per node, int32 [n]
    Z: float                         # line impedance (ohm), one value for every cut wire
    tol: float                       # relative residual target
    precision: str                   # "fp64" | "fp32_refine" | "bf16_refine"
    edges: np.ndarray                # branch list, int64 [m, 2], canonical order
    g: np.ndarray                    # branch conductances, float64 [m]
    ground: np.ndarray               # ground conductance per node
    vccs: Optional[tuple] = None     # (k, c, gm): A[k, c] += gm
    probes: Optional[np.ndarray] = None
    block_widths: Optional[tuple] = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def nrhs(self) -> int:
        return self.b.shape[0]

    @property
    def n_sub(self) -> int:
        return int(self.part.max()) + 1


# Each entry: grid dims, block spec, conductance law, nrhs, tol, precision, extras.
CONFIGS = {
    1: dict(dims=(64, 64), block=(16, 16), law="uniform", nrhs=1, tol=1e-10,
            precision="fp64"),
    2: dict(dims=(2048, 2048), block=(8, 8), law="loguniform", nrhs=1, tol=1e-8,
            precision="fp64"),
    3: dict(dims=(128, 128, 128), block=(8, 8, 8), law="uniform", nrhs=1, tol=1e-8,
            precision="fp32_refine", vccs_frac=0.02, vccs_std=0.2),
    4: dict(dims=(1024, 1024), block="random", law="uniform", nrhs=64, tol=1e-8,
            precision="bf16_refine"),
    5: dict(dims=(512, 512), block=(16, 16), law="uniform", nrhs=1, tol=1e-8,
            precision="fp32_refine", probes=4096),
}


def make(cfg: int, seed: int = 0, dims: Optional[tuple] = None, nrhs: Optional[int] = None,
         block=None, n_probes: Optional[int] = None) -> Workload:
    """Build workload ``cfg`` (1..5).  ``dims``/``nrhs``/``block``/``n_probes``
    shrink it for tests while keeping its structure and value distributions."""
    spec = dict(CONFIGS[cfg])
    dims = tuple(dims) if dims is not None else spec["dims"]
    nrhs = int(nrhs) if nrhs is not None else spec["nrhs"]
    block = block if block is not None else spec["block"]
    rng = np.random.default_rng(seed)

    if len(dims) == 2:
        edges = grid2d_edges(*dims)
    else:
        edges = grid3d_edges(*dims)
    n = int(np.prod(dims))
    m = edges.shape[0]

    # 1. branch conductances, canonical edge order
    if spec["law"] == "uniform":
        g = rng.uniform(0.5, 2.0, size=m)
    else:
        g = 10.0 ** rng.uniform(-1.0, 1.0, size=m)
    ground = np.full(n, GROUND_S)

    # 2. current sources N(0, 1), one row per right-hand side
    b = rng.standard_normal((nrhs, n))

    # the deterministic partitions are needed before the controlled sources
    widths = None
    if block != "random":
        part = (block_partition_2d(*dims, *block) if len(dims) == 2
                else block_partition_3d(*dims, *block))
    else:
        part = None

    # 3. controlled sources on a fraction of the edges inside one subdomain
    vccs = None
    if spec.get("vccs_frac"):
        intra = np.nonzero(part[edges[:, 0]] == part[edges[:, 1]])[0]
        k_count = int(round(spec["vccs_frac"] * m))
        pick = np.sort(rng.choice(intra.size, size=k_count, replace=False))
        sel = edges[intra[pick]]
        flip = rng.integers(0, 2, size=k_count).astype(bool)
        k_node = np.where(flip, sel[:, 1], sel[:, 0])
        c_node = np.where(flip, sel[:, 0], sel[:, 1])
        gm = rng.normal(0.0, spec["vccs_std"], size=k_count)
        vccs = (k_node.astype(np.int64), c_node.astype(np.int64), gm)

    # 4. random cuts (x widths first, then y widths)
    if block == "random":
        wx = random_cut_widths(rng, dims[1])
        wy = random_cut_widths(rng, dims[0])
        part = block_partition_2d(dims[0], dims[1], wy, wx)
        widths = (tuple(wy), tuple(wx))

    # 5. probe nodes for the IR-drop loss
    probes = None
    if spec.get("probes"):
        k_probe = n_probes if n_probes is not None else min(spec["probes"], n)
        probes = np.sort(rng.choice(n, size=k_probe, replace=False)).astype(np.int64)

    A = nodal_matrix(n, edges, g, ground, vccs)
    Z = 1.0 / float(np.mean(g))
    name = f"cfg{cfg}:" + "x".join(str(d) for d in dims)
    return Workload(name=name, dims=dims, A=A, b=b, part=part, Z=Z, tol=spec["tol"],
                    precision=spec["precision"], edges=edges, g=g, ground=ground,
                    vccs=vccs, probes=probes, block_widths=widths,
                    meta=dict(cfg=cfg, seed=seed, block=block, law=spec["law"]))
