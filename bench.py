#!/usr/bin/env python3
"""Benchmark of the VTM hot path on one MI355X.

Workload: 2048 x 2048 5-point resistor grid (4,194,304 unknowns), branch
conductances log-uniform in [0.1, 10] S, 0.01 S to ground per node, one N(0,1)
current-source right-hand side, torn into 256 x 256 sub-circuits of 8 x 8 nodes
(dense explicit inverse each), line impedance 1 / mean(g), FP64, solved to
relative residual 1e-8.  A step is one solve from zero waves to the tolerance
(setup is timed separately).  value = sweeps per second over the timed steps.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "VTM time-to-1e-8 residual and sweeps/s; mixed/batched vs plain FP64 speedup"
COUNTERS = os.path.join(ROOT, "profiles", "sweep_pps_fp64_2048sq_8x8_counters.json")
KERNEL_SRC = os.path.join(ROOT, "paper_0910_0663_amd", "csrc", "ports.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_relres(A, b, x):
    """||b - A x|| / ||b|| per column on the host in FP64 (b, x: [nrhs, n]) -- an
    independent check of the library's own stop rule."""
    b = np.atleast_2d(b)
    x = np.atleast_2d(x)
    r = b - (A @ x.T).T
    bn = np.linalg.norm(b, axis=1)
    return np.linalg.norm(r, axis=1) / np.where(bn > 0, bn, 1.0)


def sweep_bytes(n, n_sub, n_wires, inverse_bytes):
    """Algorithmic bytes of one sweep launch: every stored inverse once, b read and
    x written (16 B per node), per port the incident wave read and the outgoing
    wave written (16 B), its c/beta/gamma (24 B) and node/slot/twin indices
    (12 B), and 16 B of offsets per sub-circuit."""
    return inverse_bytes + 16 * n + 2 * n_wires * 52 + 16 * n_sub


def port_rows_sweep_bytes(A, part, n_sub, n_wires):
    """Algorithmic bytes of the first full sweep of a port-to-port run, which forms
    x on the port nodes only (numbered first in each sub-circuit): the inverse's
    rows of those nodes, b read on every node (the right-hand side is staged
    whole), x written on the port nodes, and the per-port and per-sub-circuit terms
    of sweep_bytes."""
    A = A.tocoo()
    cut = part[A.row] != part[A.col]
    k = np.bincount(part[np.unique(A.row[cut])], minlength=n_sub).astype(np.int64)
    ns = np.bincount(part, minlength=n_sub).astype(np.int64)
    return int(8 * np.dot(k, ns) + 8 * len(part) + 8 * k.sum() + 2 * n_wires * 52 + 16 * n_sub)


def kernel_hash():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(launches_bytes):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary,
    when it was taken on the current kernel source."""
    try:
        with open(COUNTERS) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("kernel_sha") != kernel_hash():
        return None
    return c.get("hbm_bytes_per_launch")


def machine():
    """The host the CPU baseline ran on: usable cores and CPU model."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"nproc": cores, "cpu_model": model}


def cpu_baseline(seconds, full_sweeps):
    """The oracle as it stands, on a 512 x 512 grid of the same kind (4,096 of the
    65,536 sub-circuits): sweeps timed after the (untimed) tear and factorisation,
    the rate scaled by 4,096 / 65,536 to the full workload.  Run twice: BLAS
    threads limited to one, then to every usable core (the oracle's sweep is a
    SuperLU triangular solve of the block-diagonal local systems and sparse
    products, which run on one core either way).  Time to tolerance is
    extrapolated: per-sweep time at full size times the full workload's sweep
    count.  Context: a sparse LU of the untorn sample (the direct work VTM
    avoids), with its solve."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from threadpoolctl import threadpool_limits
    import oracle
    import workloads
    w = workloads.make(2, dims=(512, 512))
    torn = oracle.tear_wires(w.A, w.part, w.Z)
    sw = oracle.Sweeper(torn)
    m = machine()
    runs = {}
    for label, threads in (("1_thread", 1), ("all_cores", m["nproc"])):
        with threadpool_limits(limits=threads):
            t = time.perf_counter()
            oracle.vtm_solve(torn, w.A, w.b, 0.0, max_sweeps=2, sweeper=sw)
            per = (time.perf_counter() - t) / 2
            k = max(3, int(0.5 * seconds / max(per, 1e-6)))
            t = time.perf_counter()
            r = oracle.vtm_solve(torn, w.A, w.b, 0.0, max_sweeps=k, sweeper=sw)
            dt = time.perf_counter() - t
        runs[label] = (r.sweeps, dt, threads)
    scale = w.n_sub / 65536
    sweeps1, dt1, _ = runs["1_thread"]
    sweepsN, dtN, nth = runs["all_cores"]
    rate1, rateN = sweeps1 / dt1 * scale, sweepsN / dtN * scale
    t = time.perf_counter()
    lu = spla.splu(sp.csc_matrix(w.A), permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    lu.solve(w.b.ravel())
    splu_s = time.perf_counter() - t
    best = max(rate1, rateN)
    return {"value": round(best, 4), "unit": "sweeps/s", "cores": nth if rateN >= rate1 else 1, "kind": "oracle",
            "sample": f"512x512 grid of the same kind ({w.n_sub} sub-circuits of 8x8): {sweeps1} sweeps in "
                      f"{dt1:.1f} s with 1 BLAS thread, {sweepsN} in {dtN:.1f} s with {nth}; rates scaled by "
                      f"{w.n_sub}/65536 to the full workload",
            "machine": m,
            "sweeps_per_s_1_thread": round(rate1, 4), "sweeps_per_s_all_cores": round(rateN, 4),
            "time_to_tol_s_extrapolated": round(full_sweeps / best, 1),
            "time_to_tol_note": f"extrapolated: {full_sweeps} sweeps (the full workload's count) at the "
                                f"full-size per-sweep time",
            "splu_sample_s": round(splu_s, 2),
            "splu_note": "sparse LU and solve of the untorn 512x512 sample (SuperLU, minimum-degree ordering "
                         "of A + A^T), the direct work VTM avoids; context only"}


def direct_reference(A, b, cols=None):
    """x* = A^-1 b for the accuracy figures, by a sparse LU of the untorn A
    (scipy's SuperLU; symmetric minimum-degree ordering when A is symmetric),
    for all right-hand sides or the given columns."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    A = sp.csc_matrix(A)
    sym = abs(A - A.T).max() == 0
    lu = (spla.splu(A, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))
          if sym else spla.splu(A))
    bb = np.atleast_2d(b) if cols is None else np.atleast_2d(b)[cols]
    return lu.solve(np.ascontiguousarray(bb.T)).T


def rel_error(x, xs):
    """max over columns of ||x - x*||_2 / ||x*||_2"""
    x, xs = np.atleast_2d(x), np.atleast_2d(xs)
    return float((np.linalg.norm(x - xs, axis=1) / np.linalg.norm(xs, axis=1)).max())


def hbm_resident_roofline(vtm, torch, workloads, sweeps=256):
    """The packed port-to-port sweep on a 4096 x 4096 grid of the bench kind
    (262,144 sub-circuits of 8 x 8): about 1.2 GB per sweep, 4.4 times the
    256 MiB Infinity Cache, so the fraction is an HBM one.  A fixed run of
    sweeps (every sweep after the first port-to-port; no check before the
    last), timed by HIP events around each run of port-to-port sweeps."""
    t = time.perf_counter()
    w = workloads.make(2, dims=(4096, 4096))
    gen_s = time.perf_counter() - t
    s = vtm.Solver(w.A, w.part, w.Z, check_every=sweeps, max_sweeps=sweeps, adaptive_checks=False, timing=2)
    b = torch.as_tensor(w.b, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    rep = None
    for _ in range(2):  # the first run warms up
        try:
            s.solve(b, 1e-300, x)
        except vtm.VTMError as e:
            rep = e.report
    nbytes = s.port_sweep_bytes
    us = rep.pp_kernel_ms / rep.pp_launches * 1e3
    gbs = nbytes / (us * 1e-6) / 1e9
    out = {"workload": f"4096x4096 grid, {s.n_sub} sub-circuits of 8x8, log-uniform g, FP64, {sweeps} sweeps",
           "bound": "hbm", "kernel": "k_sweep_pps<double,double>", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_launch": nbytes,
           "avg_launch_us": round(us, 2), "launches_timed": int(rep.pp_launches),
           "working_set_vs_infinity_cache": round(nbytes / float(256 << 20), 2)}
    s.close()
    log(f"4096^2 packed sweep: {us:.1f} us per sweep, {gbs:.0f} GB/s, frac {gbs / HBM_PEAK_GBS:.3f} "
        f"(workload {gen_s:.0f} s to generate)")
    return out


def refresh_timing(vtm, torch, w, s, b, x, reps=3):
    """vtm_refresh on the bench workload: every branch conductance scaled by
    U[0.8, 1.25] (the same pattern), timed from the host call to its return
    (host merge of the values, port coefficients, uploads, inverses, operators),
    then a solve; beside a fresh vtm_setup of the same values."""
    g = w.g * np.random.default_rng(1).uniform(0.8, 1.25, w.g.size)
    A2 = workloads_nodal(w, g)
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        s.refresh(A2)
        times.append(time.perf_counter() - t)
    _, rep = s.solve(b, w.tol, x)
    host_rel = float(host_relres(A2, w.b, x.cpu().numpy()).max())
    torch.cuda.synchronize()
    t = time.perf_counter()
    fresh = vtm.Solver(A2, w.part, w.Z, check_every=8)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t
    fresh.close()
    s.refresh(w.A)  # back to the bench values
    return {"refresh_s": round(min(times), 4), "setup_s_same_values": round(setup_s, 3),
            "solve_after_refresh_sweeps": rep.sweeps, "solve_after_refresh_relres": host_rel}


def workloads_nodal(w, g):
    import workloads
    return workloads.nodal_matrix(w.n, w.edges, g, w.ground, w.vccs)


def measured_read_peak(torch, gib=4, reps=5):
    """Streaming-read bandwidth of this GPU's HBM, measured here: a sum over a
    4 GiB buffer (one read of every byte, a negligible write), best of reps."""
    buf = torch.ones((gib << 30) // 8, dtype=torch.float64, device="cuda")
    buf.sum()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        buf.sum()
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del buf
    torch.cuda.empty_cache()
    return (gib << 30) / best / 1e9


def timed_solve(vtm, torch, w, precision, nrhs_max, reps=2):
    """Setup (untimed here), one warm solve, then the mean of `reps` solves."""
    s = vtm.Solver(w.A, w.part, w.Z, precision=precision, nrhs_max=nrhs_max)
    b = torch.as_tensor(w.b, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    s.solve(b, w.tol, x)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        _, rep = s.solve(b, w.tol, x)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) / reps * 1e3
    s.close()
    return ms, rep, x


def batched_pp_roofline(vtm, torch, w):
    """HBM roofline of the batched port-to-port sweep (BF16 and FP64 operator tiles,
    64 right-hand sides): algorithmic bytes per launch over the average launch time
    from HIP events around each run of port-to-port sweeps (timing mode 2).
    Bytes: the padded q_s x q_s operator of every sub-circuit once (q_s = cut wires
    at s, padded to a multiple of 32; 2 or 8 bytes an entry), and per port and
    right-hand side the incident wave, h and the outgoing wave (4 or 8 bytes each),
    plus a 4-byte twin index per port."""
    i, j = w.edges[:, 0], w.edges[:, 1]
    cut = w.part[i] != w.part[j]
    q = np.bincount(w.part[i[cut]], minlength=w.n_sub) + np.bincount(w.part[j[cut]], minlength=w.n_sub)
    qp = (q + 31) // 32 * 32
    ports = int(q.sum())
    b = torch.as_tensor(w.b, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    out = {}
    for prec, e_op, e_vec in (("bf16_refine", 2, 4), ("fp64", 8, 8)):
        s = vtm.Solver(w.A, w.part, w.Z, precision=prec, nrhs_max=w.nrhs, timing=2)
        s.solve(b, w.tol, x)
        _, rep = s.solve(b, w.tol, x)
        s.close()
        us = rep.pp_kernel_ms / max(rep.pp_launches, 1) * 1e3
        nbytes = int((qp.astype(np.int64) ** 2).sum() * e_op + ports * w.nrhs * 3 * e_vec + ports * 4)
        gbs = nbytes / (us * 1e-6) / 1e9
        out["bf16" if prec == "bf16_refine" else "fp64"] = {
            "bound": "hbm", "kernel": "k_sweep_mfma_pp", "achieved": round(gbs, 1), "peak": 8000.0,
            "unit": "GB/s", "frac": round(gbs / 8000.0, 4), "bytes_per_launch": nbytes,
            "avg_launch_us": round(us, 2), "launches_timed": int(rep.pp_launches),
            "shape": list(rep.pp_shape)}
    return out


def mixed_and_batched(vtm, torch, workloads):
    """The precision/batching forms against plain FP64 VTM on the same GPU, each
    solved to relative residual 1e-8 (recomputed on the host in FP64)."""
    res = {}
    w = workloads.make(4)
    t16, r16, x16 = timed_solve(vtm, torch, w, "bf16_refine", 64)
    t64, r64, x64 = timed_solve(vtm, torch, w, "fp64", 64)
    rel16 = float(host_relres(w.A, w.b, x16.cpu().numpy()).max())
    rel64 = float(host_relres(w.A, w.b, x64.cpu().numpy()).max())
    assert rel16 <= w.tol and rel64 <= w.tol, (rel16, rel64)
    diff = float(((x16 - x64).norm(dim=1) / x64.norm(dim=1)).max())
    cols = list(range(0, 64, 8))   # 8 of the 64 columns: a direct solve of all 64 takes ~40 s on the host
    xs = direct_reference(w.A, w.b, cols)
    err16 = rel_error(x16.cpu().numpy()[cols], xs)
    err64 = rel_error(x64.cpu().numpy()[cols], xs)
    res["batched_bf16_vs_fp64"] = {
        "workload": f"1024x1024 grid, {w.n_sub} uneven sub-circuits (8..24 nodes a side), 64 RHS N(0,1), tol 1e-8",
        "bf16_refine_ms": round(t16, 2), "fp64_batched_ms": round(t64, 2), "speedup": round(t64 / t16, 3),
        "bf16_sweeps": r16.sweeps, "bf16_outer": r16.outer, "fp64_sweeps": r64.sweeps,
        "bf16_relres": rel16, "fp64_relres": rel64, "bf16_vs_fp64_rel_error": diff,
        "bf16_error_vs_direct": err16, "fp64_error_vs_direct": err64,
        "error_note": "max over columns 0, 8, ..., 56 of ||x - x*|| / ||x*||, x* by sparse LU of A (SuperLU)",
        "batch_shape_bf16": list(r16.batch_shape), "batch_shape_fp64": list(r64.batch_shape)}
    # the same 64 right-hand sides as 64 single-column FP64 solves (port-to-port form)
    s1 = vtm.Solver(w.A, w.part, w.Z, precision="fp64", nrhs_max=1)
    bcols = [torch.as_tensor(w.b[r:r + 1], dtype=torch.float64, device="cuda") for r in range(w.nrhs)]
    xcols = [torch.empty_like(c) for c in bcols]
    s1.solve(bcols[0], w.tol, xcols[0])
    torch.cuda.synchronize()
    t = time.perf_counter()
    sweeps1 = 0
    for c, xc in zip(bcols, xcols):
        _, rep1 = s1.solve(c, w.tol, xc)
        sweeps1 += rep1.sweeps
    torch.cuda.synchronize()
    t1 = (time.perf_counter() - t) * 1e3
    s1.close()
    x1 = torch.cat(xcols).cpu().numpy()
    rel1 = float(host_relres(w.A, w.b, x1).max())
    assert rel1 <= w.tol, rel1
    res["batched_bf16_vs_fp64"].update({
        "fp64_single_rhs_x64_ms": round(t1, 1), "fp64_single_rhs_sweeps_total": sweeps1,
        "fp64_single_rhs_relres": rel1, "speedup_vs_single_rhs": round(t1 / t16, 2)})
    log(f"cfg4: bf16 {t16:.1f} ms ({r16.sweeps} sweeps, {r16.outer} outer) vs fp64 batched {t64:.1f} ms "
        f"({r64.sweeps} sweeps): x{t64 / t16:.2f}; vs 64 single-RHS fp64 solves {t1:.0f} ms: x{t1 / t16:.1f}")
    res["roofline_batched_pp"] = batched_pp_roofline(vtm, torch, w)
    w = workloads.make(3)
    t32, r32, x32 = timed_solve(vtm, torch, w, "fp32_refine", 1, reps=2)
    t64, r64, x64 = timed_solve(vtm, torch, w, "fp64", 1, reps=2)
    rel32 = float(host_relres(w.A, w.b, x32.cpu().numpy()).max())
    rel64 = float(host_relres(w.A, w.b, x64.cpu().numpy()).max())
    assert rel32 <= w.tol and rel64 <= w.tol, (rel32, rel64)
    sref = vtm.Solver(w.A, w.part, w.Z)
    xref, _ = sref.solve(torch.as_tensor(w.b, dtype=torch.float64, device="cuda"), 1e-12)
    sref.close()
    xr = xref.cpu().numpy()
    err32_3d = rel_error(x32.cpu().numpy(), xr)
    err64_3d = rel_error(x64.cpu().numpy(), xr)
    res["fp32_vs_fp64_3d"] = {
        "workload": f"128^3 7-point grid with {w.vccs[0].size} controlled sources (unsymmetric), "
                    f"{w.n_sub} sub-circuits of 8^3, 1 RHS, tol 1e-8; port-node operators K^-1[N,N] "
                    f"(296 port nodes carry 384 ports)",
        "fp32_refine_ms": round(t32, 2), "fp64_ms": round(t64, 2), "speedup": round(t64 / t32, 3),
        "fp32_sweeps": r32.sweeps, "fp32_outer": r32.outer, "fp64_sweeps": r64.sweeps,
        "fp32_relres": rel32, "fp64_relres": rel64,
        "fp32_error_vs_fp64_1e-12": err32_3d, "fp64_error_vs_fp64_1e-12": err64_3d,
        "error_note": "||x - x_ref|| / ||x_ref|| with x_ref the plain FP64 VTM solve to relative residual "
                      "1e-12 on the GPU (a sparse LU of this 3-D grid does not fit the host's time budget)"}
    log(f"cfg3: fp32 refine {t32:.1f} ms vs fp64 {t64:.1f} ms: x{t64 / t32:.2f}")
    del x32, x64
    w = workloads.make(5)
    t32, r32, x32 = timed_solve(vtm, torch, w, "fp32_refine", 1, reps=5)
    t64, r64, x64 = timed_solve(vtm, torch, w, "fp64", 1, reps=5)
    rel32 = float(host_relres(w.A, w.b, x32.cpu().numpy()).max())
    rel64 = float(host_relres(w.A, w.b, x64.cpu().numpy()).max())
    assert rel32 <= w.tol and rel64 <= w.tol, (rel32, rel64)
    xs5 = direct_reference(w.A, w.b)
    res["fp32_vs_fp64"] = {
        "workload": "512x512 grid, 1,024 sub-circuits of 16x16, 1 RHS, tol 1e-8",
        "fp32_refine_ms": round(t32, 3), "fp64_ms": round(t64, 3), "speedup": round(t64 / t32, 3),
        "fp32_sweeps": r32.sweeps, "fp32_outer": r32.outer, "fp64_sweeps": r64.sweeps,
        "fp32_relres": rel32, "fp64_relres": rel64,
        "fp32_error_vs_direct": rel_error(x32.cpu().numpy(), xs5),
        "fp64_error_vs_direct": rel_error(x64.cpu().numpy(), xs5),
        "error_note": "||x - x*|| / ||x*||, x* by sparse LU of A (SuperLU)"}
    log(f"cfg5: fp32 refine {t32:.2f} ms vs fp64 {t64:.2f} ms: x{t64 / t32:.2f}")
    res["gradient"] = gradient_path(vtm, torch, workloads)
    res["line_admittance_rules_2048sq"] = preconditioners(vtm, torch, workloads)
    res["vertex_tearing"] = vertex_tearing(vtm, torch, workloads)
    return res


def gradient_path(vtm, torch, workloads, reps=5):
    """The IR-drop loss L = sum of x^2 over 4,096 probe nodes of the 512x512 grid:
    forward solve, adjoint solve with g = dL/dx = 2 x at the probes, then
    dL/dg_e = -(lambda_i - lambda_j)(x_i - x_j) for every branch; FP32 sweeps
    with FP64 refinement to 1e-8, each stage timed on its own."""
    w = workloads.make(5)
    s = vtm.Solver(w.A, w.part, w.Z, precision="fp32_refine")
    b = torch.as_tensor(w.b, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    lam = torch.empty_like(b)
    ij = torch.as_tensor(w.edges, dtype=torch.int32, device="cuda")
    probes = torch.as_tensor(w.probes, dtype=torch.int64, device="cuda")
    t = {"forward": 0.0, "adjoint": 0.0, "grad": 0.0}
    for k in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.solve(b, w.tol, x)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = torch.zeros_like(x)
        g[0, probes] = 2.0 * x[0, probes]
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        s.solve_adjoint(g, w.tol, lam)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        dg = s.grad(x, lam, ij)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        if k:  # the first pass is a warm-up
            t["forward"] += (t1 - t0) / reps
            t["adjoint"] += (t3 - t2) / reps
            t["grad"] += (t4 - t3) / reps
    s.close()
    rel_f = float(host_relres(w.A, w.b, x.cpu().numpy()).max())
    rel_a = float(host_relres(w.A.T.tocsr(), g.cpu().numpy(), lam.cpu().numpy()).max())
    assert rel_f <= w.tol and rel_a <= w.tol and bool(torch.isfinite(dg).all()), (rel_f, rel_a)
    out = {"workload": f"512x512 grid, 1,024 sub-circuits of 16x16, loss over {w.probes.size} probes, "
                       f"{ij.shape[0]:,} branches; FP32 sweeps + FP64 refinement to 1e-8",
           "forward_ms": round(t["forward"] * 1e3, 3), "adjoint_ms": round(t["adjoint"] * 1e3, 3),
           "grad_ms": round(t["grad"] * 1e3, 3),
           "total_ms": round(sum(t.values()) * 1e3, 3), "forward_relres": rel_f, "adjoint_relres": rel_a}
    log(f"cfg5 gradient: forward {out['forward_ms']} ms, adjoint {out['adjoint_ms']} ms, "
        f"dL/dg {out['grad_ms']} ms")
    return out


def preconditioners(vtm, torch, workloads):
    """Section VIII's line admittances on the bench grid (2048x2048, FP64, 1e-8):
    the workload's own W = mean conductance, a scaled mean, and the weighted
    overlapped block W = alpha C (C = each twin's 2g); sweeps and solve time."""
    w = workloads.make(2)
    b = torch.as_tensor(w.b, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    out = []
    for rule, alpha in (("scaled_mean", 1.0), ("scaled_mean", 0.25), ("ob", 1.0), ("wob", 0.0625)):
        W = vtm.line_admittance(w.A, w.part, rule, alpha)
        s = vtm.Solver(w.A, w.part, 1.0 / W)
        s.solve(b, w.tol, x)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, rep = s.solve(b, w.tol, x)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3
        s.close()
        rel = float(host_relres(w.A, w.b, x.cpu().numpy()).max())
        assert rel <= w.tol, (rule, alpha, rel)
        out.append({"rule": rule, "alpha": alpha, "sweeps": rep.sweeps, "ms": round(ms, 2), "relres": rel})
        log(f"cfg2 W {rule} x{alpha}: {rep.sweeps} sweeps, {ms:.1f} ms")
    return out


def setup_times(vtm, torch, workloads, which="all"):
    """Setup (plan, uploads, blocked Gauss-Jordan inverses on the GPU, port operators)
    of the two workloads with the largest sub-circuits, each set up twice: "128",
    the 128^3 grid with controlled sources (4,096 inverses of 512 nodes); "30", the
    30^3 unit grid torn at one separator plane (two inverses of 14,400 nodes)."""
    cases = {}
    if which in ("all", "128"):
        w = workloads.make(3)
        cases["128^3, 4096 sub-circuits of 512 nodes, FP64"] = lambda: vtm.Solver(w.A, w.part, w.Z)
    if which in ("all", "30"):
        dims = (30, 30, 30)
        e = workloads.grid3d_edges(*dims)
        n = int(np.prod(dims))
        A = workloads.nodal_matrix(n, e, np.ones(e.shape[0]), np.full(n, workloads.GROUND_S))
        label, iface, sides = workloads.separator_strips(dims, 14)
        W = vtm.vertex_admittance(A, label, iface, sides, "diag", 1.0)
        cases["30^3 torn at one separator plane, 2 sub-circuits of 14,400 nodes, FP64"] = \
            lambda: vtm.Solver(A, label, None, iface=iface, sides=sides, W=W)
    out = {}
    for name, make in cases.items():
        ms = []
        for _ in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            s = make()
            torch.cuda.synchronize()
            ms.append(round((time.perf_counter() - t) * 1e3, 1))
            s.close()
        out[name] = {"setup_ms": ms}
        log(f"setup {name}: {ms} ms")
    return out


def vertex_tearing(vtm, torch, workloads):
    """Tearing at interfacial nodes (Section V) with the admittance rules of
    Section VIII as coupled lines, on unit resistor grids like Table I's Grid2d
    and Grid3d (0.01 S to ground everywhere), torn in two by one separator
    layer (Table II's setting) or cut into strips / slabs by several: sweeps
    and time to 1e-8, setup time, residual checked on the host."""
    out = {}
    for name, dims, width in (("grid2d_100x100_one_separator", (100, 100), 49),
                              ("grid2d_100x100_strips_of_18", (100, 100), 18),
                              ("grid3d_20x20x20_one_separator", (20, 20, 20), 9),
                              ("grid3d_30x30x30_one_separator", (30, 30, 30), 14),
                              ("grid3d_20x20x40_slabs_of_2", (20, 20, 40), 2)):
        e = workloads.grid2d_edges(*dims) if len(dims) == 2 else workloads.grid3d_edges(*dims)
        n = int(np.prod(dims))
        A = workloads.nodal_matrix(n, e, np.ones(e.shape[0]), np.full(n, workloads.GROUND_S))
        bh = np.random.default_rng(0).standard_normal((1, n))
        b = torch.as_tensor(bh, dtype=torch.float64, device="cuda")
        x = torch.empty_like(b)
        label, iface, sides = workloads.separator_strips(dims, width)
        rows = []
        for rule, alpha in (("identity", 1.0), ("diag", 1.0), ("ob", 1.0), ("wob", 0.3),
                            ("sca_depth", 1 if iface.size > 500 and label.max() == 1 else 2)):
            t = time.perf_counter()
            W = (vtm.vertex_sca(A, label, iface, sides, 0, alpha) if rule == "sca_depth"
                 else vtm.vertex_admittance(A, label, iface, sides, rule, alpha))
            w_ms = (time.perf_counter() - t) * 1e3
            torch.cuda.synchronize()
            t = time.perf_counter()
            s = vtm.Solver(A, label, None, iface=iface, sides=sides, W=W)
            torch.cuda.synchronize()
            setup_ms = (time.perf_counter() - t) * 1e3
            s.solve(b, 1e-8, x)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, rep = s.solve(b, 1e-8, x)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t) * 1e3
            s.close()
            rel = float(host_relres(A, bh, x.cpu().numpy()).max())
            assert rel <= 1e-8, (name, rule, rel)
            rows.append({"rule": rule, "alpha": alpha, "sweeps": rep.sweeps, "ms": round(ms, 3),
                         "setup_ms": round(setup_ms, 1), "w_host_ms": round(w_ms, 1), "relres": rel})
            log(f"{name} W {rule} x{alpha}: {rep.sweeps} sweeps, {ms:.2f} ms (setup {setup_ms:.0f} ms)")
        out[name] = {"n": n, "interfacial_nodes": int(iface.size), "sub_circuits": int(label.max()) + 1,
                     "rules": rows}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--check-every", type=int, default=8)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision / batched comparison")
    ap.add_argument("--no-hbm", action="store_true", help="skip the 4096x4096 HBM-resident sweep roofline")
    ap.add_argument("--hbm-only", action="store_true",
                    help="for profiling: only the 4096x4096 packed sweep run; prints its JSON")
    ap.add_argument("--calibrate", action="store_true",
                    help="with --mfma-counters or --hbm-only: end with a 1 GiB device copy (known bytes) to "
                         "calibrate FETCH_SIZE / WRITE_SIZE")
    ap.add_argument("--mfma-counters", action="store_true",
                    help="for MFMA counters: one BF16 and one FP64 batched solve of the 64-RHS workload")
    ap.add_argument("--setup-only", nargs="?", const="all", choices=["all", "128", "30"],
                    help="for profiling: only the setups of large sub-circuits (128: the 128^3 grid's 4,096 "
                         "inverses of 512 nodes; 30: the 30^3 grid torn at one separator plane, two inverses "
                         "of 14,400 nodes; all: both); prints their JSON")
    ap.add_argument("--vertex-only", action="store_true",
                    help="for profiling: only the tearing at interfacial nodes; prints its JSON")
    ap.add_argument("--batched-only", action="store_true",
                    help="for profiling: only the mixed-precision / batched comparison; prints its JSON")
    ap.add_argument("--counters", action="store_true",
                    help="for rocprofv3 --pmc: 16 sweeps of the workload, then a 1 GiB device copy "
                         "(known bytes) to calibrate the counters; prints no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the VTM path here is built and measured on a single "
              "MI355X (multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    import paper_0910_0663_amd as vtm

    assert torch.cuda.is_available(), "bench.py needs a HIP device"

    def calibration_copy():
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read, 1 GiB written")

    if args.mfma_counters:
        # the 64-RHS workload once in BF16 refinement and once in FP64 batched form (MFMA tiles)
        w4 = workloads.make(4)
        b4 = torch.as_tensor(w4.b, dtype=torch.float64, device="cuda")
        out = {}
        for prec in ("bf16_refine", "fp64"):
            s4 = vtm.Solver(w4.A, w4.part, w4.Z, precision=prec, nrhs_max=64)
            x4, rep4 = s4.solve(b4, w4.tol)
            torch.cuda.synchronize()
            out[prec] = {"sweeps": rep4.sweeps, "outer": rep4.outer, "solve_ms": round(rep4.solve_ms, 2),
                         "batch_shape": list(rep4.batch_shape), "port_operator_bytes": s4.port_operator_bytes,
                         "relres": float(host_relres(w4.A, w4.b, x4.cpu().numpy()).max())}
            s4.close()
        if args.calibrate:
            calibration_copy()
        print(json.dumps(out), flush=True)
        return
    if args.setup_only:
        out = setup_times(vtm, torch, workloads, args.setup_only)
        if args.calibrate:
            calibration_copy()
        print(json.dumps(out), flush=True)
        return
    if args.vertex_only:
        print(json.dumps(vertex_tearing(vtm, torch, workloads)), flush=True)
        return
    if args.batched_only:
        print(json.dumps(mixed_and_batched(vtm, torch, workloads)), flush=True)
        return
    if args.hbm_only:
        r = hbm_resident_roofline(vtm, torch, workloads)
        if args.calibrate:
            calibration_copy()
        print(json.dumps(r), flush=True)
        return
    t = time.perf_counter()
    w = workloads.make(2)
    log(f"workload {w.name}: n={w.n} sub-circuits={w.n_sub} ({time.perf_counter() - t:.1f} s to generate)")
    torch.cuda.synchronize()
    t = time.perf_counter()
    # timing 2: one HIP event pair per run of port-to-port sweeps (events around every
    # launch would slow the timed solve itself)
    s = vtm.Solver(w.A, w.part, w.Z, check_every=args.check_every, timing=2)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t
    log(f"setup {setup_s:.2f} s: wires={s.n_wires} inverse bytes={s.inverse_bytes}")
    b = torch.as_tensor(w.b, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    if args.counters:
        c = vtm.Solver(w.A, w.part, w.Z, check_every=16, max_sweeps=16)
        try:
            c.solve(b, w.tol, x)
        except vtm.VTMError as e:
            log(f"counter run: {e.name} after {e.report.sweeps} sweeps")
        calibration_copy()
        return
    for k in range(args.warmup):
        _, rep = s.solve(b, w.tol, x)
        log(f"warmup {k}: sweeps {rep.sweeps} relres {rep.relres_max:.3e} {rep.solve_ms:.1f} ms")
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps = []
    for k in range(args.steps):
        _, rep = s.solve(b, w.tol, x)
        reps.append(rep)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    for k, rep in enumerate(reps):
        log(f"step {k}: sweeps {rep.sweeps} relres {rep.relres_max:.3e} {rep.solve_ms:.1f} ms")
    sweeps = sum(r.sweeps for r in reps)
    launches = sum(r.sweep_launches for r in reps)
    kern_ms = sum(r.sweep_kernel_ms for r in reps)
    pp_launches = sum(r.pp_launches for r in reps)
    pp_ms = sum(r.pp_kernel_ms for r in reps)
    host_rel = float(host_relres(w.A, w.b, x.cpu().numpy()).max())
    log(f"host-checked relres {host_rel:.3e}; full sweeps {launches}, port-to-port sweeps {pp_launches}")
    assert host_rel <= w.tol, host_rel

    # full sweeps: per solve the first of the port-to-port run (port rows only) and
    # the rebuild of x at the end (every row); bytes_per_launch is their mean
    full_bytes = sweep_bytes(w.n, s.n_sub, s.n_wires, s.inverse_bytes)
    first_bytes = port_rows_sweep_bytes(w.A, w.part, s.n_sub, s.n_wires)
    n_first = len(reps) if pp_launches else 0
    mean_bytes = (n_first * first_bytes + (launches - n_first) * full_bytes) / launches
    full_s = kern_ms / launches / 1e3
    roof_full = {"bound": "hbm", "kernel": "k_sweep1<double,double>", "achieved": round(mean_bytes / full_s / 1e9, 1),
                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(mean_bytes / full_s / 1e9 / HBM_PEAK_GBS, 4),
                 "bytes_per_launch": int(round(mean_bytes)), "avg_launch_us": round(full_s * 1e6, 2),
                 "launches_timed": launches,
                 "note": f"{n_first} first sweeps forming the port rows ({first_bytes} B each) and "
                         f"{launches - n_first} forming every row ({full_bytes} B each)"}
    if pp_launches:
        per_launch = s.port_sweep_bytes
        avg_launch_s = pp_ms / pp_launches / 1e3
        kernel, n_timed = "k_sweep_pps<double,double>", pp_launches
    else:
        per_launch, avg_launch_s, kernel, n_timed = full_bytes, full_s, roof_full["kernel"], launches
    achieved = per_launch / avg_launch_s / 1e9
    traffic = measured_traffic(per_launch)
    read_peak = measured_read_peak(torch)
    roof_full["frac_of_measured_read"] = round(roof_full["achieved"] / read_peak, 4)
    out = {
        "metric": METRIC,
        "value": round(sweeps / elapsed, 2),
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "2048x2048 5-point resistor grid, log-uniform g in [0.1,10] S, 0.01 S ground, "
                        "65,536 sub-circuits of 8x8 (dense FP64 inverse each), Z = 1/mean(g), "
                        "1 RHS N(0,1), tol 1e-8, FP64; port-to-port sweeps on the packed symmetric "
                        "port-node operators; residual checks from port quantities, confirmed on A after "
                        "one full sweep",
            "port_operator_bytes": s.port_operator_bytes,
            "n": w.n,
            "sub_circuits": s.n_sub,
            "cut_wires": s.n_wires,
            "sweeps_per_solve": reps[-1].sweeps,
            "check_every": args.check_every,
            "time_to_tol_ms": round(elapsed / args.steps * 1e3, 3),
            "setup_s": round(setup_s, 3),
            "final_relres": host_rel,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch": per_launch,
            "avg_launch_us": round(avg_launch_s * 1e6, 2),
            "launches_timed": n_timed,
            "read_peak_measured": round(read_peak, 1),
            "frac_of_measured_read": round(achieved / read_peak, 4),
        },
        "roofline_full_sweep": roof_full,
    }
    log("refresh of the conductances ...")
    out["refresh"] = refresh_timing(vtm, torch, w, s, b, x)
    s.close()
    if not args.no_hbm:
        log("HBM-resident packed sweep (4096x4096) ...")
        out["roofline_hbm_resident"] = hbm_resident_roofline(vtm, torch, workloads)
    if not args.no_mixed:
        log("mixed-precision and batched forms vs plain FP64 ...")
        out["mixed_batched"] = mixed_and_batched(vtm, torch, workloads)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds, reps[-1].sweeps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
