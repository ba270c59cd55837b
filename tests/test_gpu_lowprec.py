"""Parity of the low-precision sweep kernels with the oracle, iterate by iterate.

A refining handle (FP32 or BF16 inner sweeps inside FP64 refinement) is run
for exactly one outer step from x = 0, so its inner right-hand side is b
itself, and that inner solve is stopped after k sweeps (one check at sweep k,
max_sweeps = k).  The result is x = 0 + d^k, the k-th low-precision VTM iterate
of A d = b (Section VI, eqs. 11 and 14), which is compared element by element
with the oracle's FP64 x^k.  This checks every low-precision kernel at its own
precision: refinement with an FP64 residual would hide a kernel that skips work
as long as the iteration still contracts.

Tolerances, derived from the arithmetic (u = unit roundoff of the stored
operator, 2^-24 for FP32, 2^-8 for BF16).  One local solve forms
x_i = sum_j t_ij with terms t_ij = K^-1_ij rhs_j.  With independent roundings
(relative errors spread uniformly over [-u, u], standard deviation u / sqrt(3))
the error of x_i is close to Gaussian with standard deviation sigma_i below:

* BF16 (inverses and right-hand sides rounded to BF16, products accumulated
  in FP32 on the matrix cores, waves in FP32): each term carries two roundings,
  so sigma_i = sqrt(2/3) u rss_i, rss_i = sqrt(sum_j t_ij^2); the FP32
  accumulation adds n_s 2^-24, negligible beside u = 2^-8.
* FP32 (inverses, port operators, waves and accumulation in FP32): the n_s
  partial sums of the dot product are rounded too, each at most
  sum_j |t_ij|, so sigma_i <= u sqrt((2 + n_s) / 3) sum_j |t_ij|.

On these circuits rms(rss) <= 1.25 rms|x|, max(rss) <= max|x| and
max(sum_j |t_ij|) <= 8 max|x| (measured with dense inverses on the test grids:
0.88-1.18, 0.49-0.85 and 2.2-6.8).  Roundings of different sweeps are
independent and the waves carry earlier errors forward through contractions
(the line reflections, Section VIII), so after k sweeps the deviations add in
quadrature: a factor sqrt(k).  The maximum over <= 10^6 entries stays within
5.5 standard deviations (a Gaussian exceeds that with probability 4e-8 per
entry).  Hence, relative to max|x| (rms|x| for the root mean square):

  FP32 max: 5.5 sqrt(k) u sqrt((2 + n_s) / 3) * 8
  BF16 max: 5.5 sqrt(k) u sqrt(2/3)          (about 4.5 u sqrt(k))
  BF16 rms: sqrt(k) u sqrt(2/3) * 1.25      (about 1.0 u sqrt(k))

A structural mistake (a skipped 16-row tile, a port's h or twin misread, a
wrong coefficient) moves the affected entries by O(max|x|), orders of
magnitude above these bounds.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

U_FP32 = 2.0 ** -24
U_BF16 = 2.0 ** -8
SIGMAS = 5.5     # the maximum over <= 10^6 entries stays within this many standard deviations
C_ABS = 8.0      # bound on max(sum_j |t_ij|) / max|x| on these circuits (measured <= 6.8)
C_RSS_RMS = 1.25  # bound on rms(rss) / rms|x| (measured <= 1.18); max(rss) <= max|x|


def fp32_rtol(k, n_s):
    return SIGMAS * math.sqrt(k) * U_FP32 * math.sqrt((2.0 + n_s) / 3.0) * C_ABS


def bf16_rtol(k):
    return SIGMAS * math.sqrt(k) * U_BF16 * math.sqrt(2.0 / 3.0)


def bf16_rms_rtol(k):
    return math.sqrt(k) * U_BF16 * math.sqrt(2.0 / 3.0) * C_RSS_RMS


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


def inner_iterate(torch, make_solver, b, k):
    """d^k of the handle's low-precision inner solve of A d = b (see module doc)."""
    s = make_solver(check_every=k, max_sweeps=k, max_outer=1, adaptive_checks=False)
    x = torch.empty(b.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(vtm().VTMError) as ei:
        s.solve(to_dev(torch, b), 1e-300, x)
    rep = ei.value.report
    assert ei.value.name == "VTM_E_MAXITER" and rep.outer == 1 and rep.sweeps == k, (ei.value.name, rep)
    s.close()
    return x.cpu().numpy(), rep


def check(x, ref, rtol, rms_rtol=None, label=""):
    scale = np.abs(ref).max()
    err = np.abs(x - ref).max()
    print(f"{label}: max err / max|x| = {err / scale:.3e} (bound {rtol:.3e})", flush=True)
    assert err <= rtol * scale, f"{label}: max err {err:.3e} vs {rtol:.2e} * {scale:.3e}"
    if rms_rtol is not None:
        rms = np.sqrt(np.mean((x - ref) ** 2))
        rref = np.sqrt(np.mean(ref ** 2))
        print(f"{label}: rms err / rms|x| = {rms / rref:.3e} (bound {rms_rtol:.3e})", flush=True)
        assert rms <= rms_rtol * rref, f"{label}: rms err {rms:.3e} vs {rms_rtol:.2e} * {rref:.3e}"


# ----------------------------------------------------------------------------- FP32
@pytest.mark.parametrize("cfg,kw,form", [
    (2, dict(dims=(64, 64)), "port"),           # packed sweep, two sub-circuits per wavefront
    (2, dict(dims=(64, 64)), "port_dense"),     # q x q port operator
    (2, dict(dims=(64, 64)), "full"),           # full inverse, one right-hand side
    (1, dict(), "port"),                         # packed sweep, 16x16 blocks: eight wavefronts each
    (5, dict(dims=(128, 128)), "port"),
    (3, dict(dims=(16, 16, 16)), "port"),       # port-node operator K^-1[N,N], controlled sources
    (3, dict(dims=(16, 16, 16)), "full"),
    (4, dict(dims=(64, 64), nrhs=3), "port"),   # three right-hand sides: full sweeps of several columns
])
def test_fp32_iterates_match_oracle(torch, cfg, kw, form):
    w = workloads.make(cfg, **kw)
    ks = [1, 5, 9]
    ref = oracle_iterates(w.A, w.part, w.Z, w.b, ks)
    n_s = int(np.bincount(w.part).max())

    def make(**o):
        return vtm().Solver(w.A, w.part, w.Z, precision="fp32_refine", nrhs_max=w.nrhs, local_form=form, **o)

    for k in ks:
        x, _ = inner_iterate(torch, make, w.b, k)
        check(x, ref[k], fp32_rtol(k, n_s), label=f"fp32 {w.name} {form} k={k}")


# ----------------------------------------------------------------------------- BF16 (MFMA)
@pytest.mark.parametrize("dims,nrhs,form", [
    ((96, 96), 20, "port"),    # batched port-to-port sweep; 20 columns: a ragged last block
    ((96, 96), 20, "full"),    # full batched sweep every time
    ((90, 90), 17, "port"),    # node and column counts off the 64 x 64 renumbering tiles
    ((64, 64), 1, "port"),     # one right-hand side
])
def test_bf16_iterates_match_oracle(torch, dims, nrhs, form):
    w = workloads.make(4, dims=dims, nrhs=nrhs)
    ks = [1, 4, 9]
    ref = oracle_iterates(w.A, w.part, w.Z, w.b, ks)

    def make(**o):
        return vtm().Solver(w.A, w.part, w.Z, precision="bf16_refine", nrhs_max=nrhs, local_form=form, **o)

    for k in ks:
        x, rep = inner_iterate(torch, make, w.b, k)
        if form == "port" and k > 2:
            assert rep.pp_shape[0] > 0
        check(x, ref[k], bf16_rtol(k), bf16_rms_rtol(k), label=f"bf16 {w.name} nrhs={nrhs} {form} k={k}")


def test_bf16_h_at_store_iterates_match_oracle(torch):
    """A 1,024-port operator (two strips of a 1024 x 7 grid torn at one
    separator column) leaves no LDS room to stage h beside the incident waves:
    the batched BF16 port-to-port sweep then reads h at the store."""
    A, b, label, iface, sides, W = _strips((1024, 7), 3, nrhs=16, seed=3)
    torn = oracle.tear_at_vertices(A, label, iface, sides, W)
    sw = oracle.Sweeper(torn)
    f = torn.src @ b.T
    a = np.zeros((2, torn.n_lines, b.shape[0]))
    ref = {}
    for k in range(1, 10):
        u, a = sw.sweep(f, a)
        ref[k] = (torn.out @ u).T

    def make(**o):
        return vtm().Solver(A, label, 1.0 / W, iface=iface, sides=sides, precision="bf16_refine", nrhs_max=16,
                            **o)

    for k in (1, 4, 9):
        x, rep = inner_iterate(torch, make, b, k)
        if k > 2:
            assert rep.pp_shape[0] > 0
        check(x, ref[k], bf16_rtol(k), bf16_rms_rtol(k), label=f"bf16 1024-port separator k={k}")


def _strips(dims, width, nrhs=1, seed=0):
    rng = np.random.default_rng(seed)
    edges = workloads.grid2d_edges(*dims)
    g = 10.0 ** rng.uniform(-1, 1, edges.shape[0])
    n = int(np.prod(dims))
    A = workloads.nodal_matrix(n, edges, g, np.full(n, workloads.GROUND_S))
    b = rng.standard_normal((nrhs, n))
    label, iface, sides = workloads.separator_strips(dims, width)
    return A, b, label, iface, sides, float(np.mean(g))


# ----------------------------------------------------------------------------- full size, sampled
@pytest.mark.parametrize("cfg,centres,R,k,prec", [
    # 128^3 with controlled sources: FP32 port-node operators over 296 port nodes
    (3, [0, 8 * 256 + 8 * 16 + 8, 4095], 2, 3, "fp32_refine"),
    # 1024^2 uneven sub-circuits, 64 right-hand sides: BF16 tiles on the matrix cores
    (4, [0, "mid", -1], 3, 4, "bf16_refine"),
])
def test_full_size_sampled_low_precision_iterates(torch, cfg, centres, R, k, prec):
    """At full size, in the bench's launch configuration, the low-precision x^k on
    sampled sub-circuits against the oracle's x^k on the window of sub-circuits
    within R >= k - 1 hops (exact for k <= R + 1)."""
    from oracle_window import window_iterate
    w = workloads.make(cfg)
    print(f"{w.name}: n={w.n} subs={w.n_sub} nrhs={w.nrhs} k={k} {prec}", flush=True)

    def make(**o):
        return vtm().Solver(w.A, w.part, w.Z, precision=prec, nrhs_max=w.nrhs, **o)

    x, _ = inner_iterate(torch, make, w.b, k)
    n_s = int(np.bincount(w.part).max())
    for c in centres:
        c = w.n_sub // 2 if c == "mid" else c % w.n_sub
        nodes = np.nonzero(w.part == c)[0]
        ref = window_iterate(w, c, R, k)
        if prec == "fp32_refine":
            check(x[:, nodes], ref, fp32_rtol(k, n_s), label=f"{w.name} sub-circuit {c}")
        else:
            check(x[:, nodes], ref, bf16_rtol(k), bf16_rms_rtol(k), label=f"{w.name} sub-circuit {c}")


# ----------------------------------------------------------------------------- refinement schedule
def test_fp32_refinement_counts_match_oracle_schedule(torch):
    """The oracle's refinement (the same outer/inner schedule with FP64 inner
    sweeps, checks every 8 sweeps) against the FP32 handle: an FP32 inner solve
    tracks the FP64 one down to its 1e-5 target (FP32 resolves ~1e-7), so the
    outer count is the same and each inner solve ends at the same check or the
    next."""
    w = workloads.make(5, dims=(128, 128))
    ref = oracle.vtm_refine(oracle.tear_wires(w.A, w.part, w.Z), w.A, w.b, w.tol, 1e-5, check_every=8)
    assert ref.status == "ok"
    s = vtm().Solver(w.A, w.part, w.Z, precision="fp32_refine", check_every=8, adaptive_checks=False)
    x, rep = s.solve(to_dev(torch, w.b), w.tol)
    print(f"oracle outer {ref.outer} inner {ref.inner_sweeps}; gpu outer {rep.outer} sweeps {rep.sweeps}",
          flush=True)
    assert rep.outer == ref.outer
    assert abs(rep.sweeps - sum(ref.inner_sweeps)) <= 8 * ref.outer
    assert oracle.relative_residual(w.A, w.b, x.cpu().numpy()).max() <= w.tol
