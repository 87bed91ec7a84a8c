#!/usr/bin/env python3
"""Benchmark of the ParAC hot path on one MI355X.  Prints one JSON line.

A step is one pass of the whole hot path over one batch of synthetic input
that is already resident on the device: the randomized elimination (setup:
checks, relabelling, persistent elimination kernel, finalisation to the solve
layout) followed by PCG with the factor to a 1e-6 relative residual (true
residual recomputed in FP64).

Workloads (--workload):
  chung_lu_22  default: Chung-Lu power-law Laplacian, 2^22 vertices generated
               (largest component kept, 4,117,731 vertices), average degree
               16, exponent 2.1, weights (0,1], random order: FP64 factor and
               FP64 PCG timed; after the timed steps one solve with the
               preconditioner applied from the FP32 copy (SpMV / dots /
               residuals in FP64) is reported beside it
  grid3d_128   3D 7-point Laplacian 128^3 (2,097,152 vertices), weights
               log-uniform [1e-2, 1e2], random order, FP64 factor and FP64 PCG
  grid2d_64    2D 5-point Laplacian 64x64, weights U[1,2] (small case)
  chung_lu_24_x32  Chung-Lu 2^24, average degree 8, 32 right-hand sides:
               block PCG with the FP32 apply
  chung_lu_16, chung_lu_18, chung_lu_20
               smaller members of the 2^22 family (ordering and AC(k) studies)
  serve_200    200 SDDM systems (sizes log-uniform 1e3..1e6, mixed families)
               with Poisson arrivals, served with continuous batching (mixed
               precision) and, for comparison, one at a time in FP64

--order nnz replaces the random elimination order of a single-system
workload by the NNZ-sorted one (ascending row count, ties by a seeded hash;
the ordering the paper recommends for GPUs), --order mis by independent-set
rounds (low degree first); both are computed on the device by parac_order
before the timed steps (ordering is not part of the setup time).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "setup+solve s to 1e-6 rel. residual; factor nnz/s; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
# HBM traffic of a kernel measured with rocprofv3 counters (FETCH_SIZE,
# WRITE_SIZE), scaled by the same counters on a copy of known size; valid only
# for the kernel sources and the workload it was taken from
TRAFFIC_PROFILES = {
    "chung_lu_22": os.path.join(ROOT, "profiles", "hbm_traffic_chung_lu_22.md"),
    "grid3d_128": os.path.join(ROOT, "profiles", "hbm_traffic_grid3d_128.md"),
}
KERNEL_SOURCES = ["ready.hip", "eliminate.hip", "internal.hpp", "device.hpp", "api.hip"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2505_02977_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, kernels):
    """HBM bytes per launch of a kernel (e.g. "k_ready<double, true, 1>"), or
    the sum over the launches of a list of kernels, from the committed counter
    summary, if it was taken on this workload from the current kernel sources;
    else None."""
    import re
    if isinstance(kernels, str):
        kernels = [kernels]
    path = TRAFFIC_PROFILES.get(workload)
    if path is None or not os.path.exists(path):
        return None
    text = open(path).read()
    m1 = re.search(r"kernel-sources-sha256:\s*([0-9a-f]{64})", text)
    if not m1 or m1.group(1) != kernel_source_hash():
        return None
    total = 0
    for k in kernels:
        m2 = re.search(r"hbm-bytes-per-launch %s:\s*([0-9]+)" % re.escape(k), text)
        if not m2:
            return None
        total += int(m2.group(1))
    return total


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic bytes: what the method has to move, with 4-byte indices and
# 8-byte values (4-byte values in the FP32 apply).
def elim_bytes(E, n_fill, n_off, N):
    """One elimination: the upper adjacency read once (12 B per edge), every
    fill record written and read (16 B each way) with its counter increment
    (8 B read-modify-write), every factor entry written (12 B) with its
    counter decrement (8 B), and D, queue slot and column offset per pivot
    (24 B)."""
    return 12 * E + 40 * n_fill + 20 * n_off + 24 * N


def fwd_bytes(n_off, N, elem=8):
    """The forward sweep F y = P r: every off-diagonal entry once (4 B index
    + value), and per row r read and y written (vector terms 20 N in FP64,
    halved in FP32)."""
    return n_off * (4 + elem) + (20 * N if elem == 8 else 10 * N)


def bwd_bytes(n_off, N, elem=8):
    """The backward sweep F^T x = D^+ y: every entry once, and per row D^+,
    y read, x and z written (28 N in FP64, halved in FP32)."""
    return n_off * (4 + elem) + (28 * N if elem == 8 else 14 * N)


def pcg_iter_bytes(nnz_L, n_off, N, elem=8):
    """One PCG iteration: SpMV with L (12 B per stored entry), both sweeps,
    and the vector traffic of the recurrence: SpMV 20N, r^T z 8N, three
    axpys 72N (plus the sweeps' own vector terms)."""
    return 12 * nnz_L + fwd_bytes(n_off, N, elem) + bwd_bytes(n_off, N, elem) + 100 * N


def rl_entry(name, nbytes, ms, traffic=None):
    achieved = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    e = {"kernel": name, "achieved": round(achieved, 2), "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 5), "algorithmic_bytes": int(nbytes),
         "avg_ms": round(ms, 4)}
    if traffic is not None:
        e["traffic"] = traffic
    return e


def roofline(info, timing, elem, workload):
    """The dominant part of a step (by time) against the HBM peak: the
    elimination's one launch, or a sweep (its dependency-driven launch, plus
    the narrow-level launches when the factor has them), with the other parts
    of the hot path beside it."""
    N, n_off = info["n"], info["nnz_off"]
    T = "double" if elem == 8 else "float"
    # a sweep is the dependency-driven launch plus, when the factor has narrow
    # final levels, the one-workgroup launches that solve them
    kf = ["k_ready<%s, false, 1>" % T]
    kb = ["k_ready<%s, true, 1>" % T]
    if info.get("narrow_levels", 0) > 0:
        kf += ["k_narrow_prep<%s>" % T, "k_narrow<%s, false, 3>" % T]
        kb = ["k_narrow<%s, true, 3>" % T] + kb
    fwd = rl_entry("forward sweep F y = P r (%s: %d launches)" % (" + ".join(kf), len(kf)),
                   fwd_bytes(n_off, N, elem), timing["fwd_ms"], measured_traffic(workload, kf))
    bwd = rl_entry("backward sweep F^T x = D^+ y (%s: %d launches)" % (" + ".join(kb), len(kb)),
                   bwd_bytes(n_off, N, elem), timing["bwd_ms"], measured_traffic(workload, kb))
    elim = rl_entry("k_eliminate (one factorisation, one persistent launch)",
                    elim_bytes(info["n_input_edges"], info["n_fill"], n_off, N), timing["elim_ms"],
                    measured_traffic(workload, "k_eliminate"))
    per_step = {"fwd": timing["fwd_ms"] * timing["applies"],
                "bwd": timing["bwd_ms"] * timing["applies"], "elim": timing["elim_ms"]}
    dom = max(per_step, key=per_step.get)
    d = {"fwd": fwd, "bwd": bwd, "elim": elim}[dom]
    out = {"bound": "hbm", "achieved": d["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": d["frac"], "traffic": d.get("traffic"), "kernel": d["kernel"],
           "algorithmic_bytes": d["algorithmic_bytes"], "avg_ms": d["avg_ms"],
           "limited_by": ("dependency latency: the elimination DAG depth (%d levels) times the "
                          "per-level publish-to-detect latency, not bandwidth" % info["depth"]),
           "others": [e for k, e in (("fwd", fwd), ("bwd", bwd), ("elim", elim)) if k != dom]}
    return out


def block_roofline(info, timing, elem, nrhs, shape):
    """The block apply (both sweeps over nrhs columns in one launch per
    direction) against the HBM peak: the factor once per direction and the
    vector terms once per column are what the method has to move; the
    launch reads the factor once per sweep slot of shape["cols_per_sweep"]
    columns."""
    N, n_off = info["n"], info["nnz_off"]
    T = "double" if elem == 8 else "float"
    cps = shape["cols_per_sweep"]
    fac = 2 * n_off * (4 + elem)
    vec = fwd_bytes(0, N, elem) + bwd_bytes(0, N, elem)
    slots = (nrhs + cps - 1) // cps
    app = rl_entry("k_ready<%s, false|true, %d> (both sweeps of one %d-column block apply, %d "
                   "slots of %d columns)" % (T, cps, nrhs, slots, cps),
                   fac + nrhs * vec, timing["apply_ms"])
    app["launch_bytes_factor_per_slot"] = int(slots * fac + nrhs * vec)
    elim = rl_entry("k_eliminate (one factorisation, one persistent launch)",
                    elim_bytes(info["n_input_edges"], info["n_fill"], n_off, N), timing["elim_ms"])
    dom_apply = timing["apply_ms"] * timing["applies"] >= timing["elim_ms"]
    d, other = (app, elim) if dom_apply else (elim, app)
    return {"bound": "hbm", "achieved": d["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": d["frac"], "traffic": None, "kernel": d["kernel"],
            "algorithmic_bytes": d["algorithmic_bytes"], "avg_ms": d["avg_ms"],
            "limited_by": ("dependency latency: the elimination DAG depth (%d levels) times the "
                           "per-level publish-to-detect latency, not bandwidth" % info["depth"]),
            "others": [other]}


# --------------------------------------------------------------------------
# single system (optionally several right-hand sides)
# --------------------------------------------------------------------------
def run_system(args, W, desc, precision, nrhs, mixed_extra=False):
    import numpy as np
    import torch
    from paper_2505_02977_amd import parac
    dA = parac.DeviceCSR(W.A)
    b = torch.tensor(W.b, device="cuda")
    x = torch.empty_like(b)
    keep32 = precision == parac.PREC_MIXED or mixed_extra
    torch.cuda.synchronize()

    def step(timing):
        f = parac.parac_factor(dA, perm=W.perm, seed=W.seed, keep_fp32=keep32,
                               samples=args.samples)
        log("  factor: %.1f ms" % f.info()["ms_total"])
        sts = parac.parac_pcg(dA, f, b, x, rtol=args.rtol, precision=precision, timing=timing)
        info = f.info()
        return f, info, sts

    for k in range(args.warmup):
        log("warmup step %d" % k)
        f, _, _ = step(False)
        del f
    torch.cuda.synchronize()
    infos, stss = [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        f, info, sts = step(True)
        if k + 1 < args.steps:
            del f
        infos.append(info)
        stss.append(sts)
        log("step %d: setup %.1f ms solve %.1f ms it %d" % (k, info["ms_total"], sts[0]["ms_total"],
                                                           max(s["iterations"] for s in sts)))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    info, sts = infos[-1], stss[-1]
    ms_setup = float(np.mean([i["ms_total"] for i in infos]))
    ms_elim = float(np.mean([i["ms_eliminate"] for i in infos]))
    # one launch sequence per chunk of up to 64 columns (stats repeat per
    # column of a chunk): sum over the chunks
    chunks = list(range(0, nrhs, 64))
    ms_solve = float(np.mean([sum(s[c]["ms_total"] for c in chunks) for s in stss]))
    applies = float(np.mean([s[0]["applies"] for s in stss]))
    ms_apply = float(np.mean([sum(s[c]["ms_apply"] / max(s[c]["applies"], 1) for c in chunks)
                              for s in stss]))
    ms_fwd = float(np.mean([s[0]["ms_fwd"] / max(s[0]["applies"], 1) for s in stss]))
    N, n_off = info["n"], info["nnz_off"]
    elem = 4 if precision == parac.PREC_MIXED else 8
    timing = {"fwd_ms": ms_fwd, "bwd_ms": ms_apply - ms_fwd, "elim_ms": ms_elim, "applies": applies}
    X = x.cpu().numpy()
    Bh = W.b
    L = W.A.to_scipy()
    resid = L @ X - Bh
    rel = np.linalg.norm(resid.reshape(N, -1), axis=0) / np.linalg.norm(Bh.reshape(N, -1), axis=0)
    iters = max(s["iterations"] for s in sts)
    out = {
        "value": round((ms_setup + ms_solve) / 1e3, 6),
        "ms_per_step": round(ms_step, 3),
        "dtype": "f64" if precision == parac.PREC_FP64 else "f64 (apply f32)",
        "config": {"workload": desc, "n": N, "nnz_L": int(W.A.nnz), "rhs": nrhs,
                   "seed": int(W.seed), "order": args.order, "samples_per_entry": args.samples,
                   "parallelism": "one GPU"},
        "t_setup_s": round(ms_setup / 1e3, 6),
        "t_solve_s": round(ms_solve / 1e3, 6),
        "t_eliminate_s": round(ms_elim / 1e3, 6),
        "factor_nnz_per_s": round((N + n_off) / (ms_setup * 1e-3), 1),
        "nnz_G": N + n_off,
        "n_fill": info["n_fill"],
        "depth": info["depth"],
        "max_gather": info["max_gather"],
        "iterations": iters,
        "true_relres_max": float(rel.max()),
        "apply_ms": round(ms_apply, 4),
        "fwd_sweep_ms": round(ms_fwd, 4) if nrhs == 1 else None,
        "workers": info["workers"],
    }
    if nrhs == 1:
        pcg_b = pcg_iter_bytes(int(W.A.nnz), n_off, N, elem)
        out["pcg_iteration"] = rl_entry("PCG iteration (SpMV, both sweeps, dots, axpys)", pcg_b,
                                        ms_solve / max(iters, 1))
    if nrhs > 1:
        shape = parac.parac_block_shape_get(f, min(nrhs, 64), precision)
        timing["apply_ms"] = ms_apply
        rl = block_roofline(info, timing, elem, min(nrhs, 64), shape)
        out["block_shape"] = shape
    else:
        rl = roofline(info, timing, elem, args.workload if args.order == "random" else None)
    out["roofline"] = rl
    if mixed_extra:
        # the same factor, preconditioner applied from its FP32 copy (not timed
        # in the steps: one solve after them)
        xm = torch.empty_like(b)
        sm = parac.parac_pcg(dA, f, b, xm, rtol=args.rtol, precision=parac.PREC_MIXED,
                             timing=True)[0]
        Xm = xm.cpu().numpy()
        relm = np.linalg.norm(L @ Xm - Bh) / np.linalg.norm(Bh)
        xp, xmp = X - X.mean(), Xm - Xm.mean()
        out["mixed"] = {
            "t_solve_s": round(sm["ms_total"] / 1e3, 6),
            "value_s": round((ms_setup + sm["ms_total"]) / 1e3, 6),
            "iterations": sm["iterations"],
            "apply_ms": round(sm["ms_apply"] / max(sm["applies"], 1), 4),
            "true_relres": float(relm),
            "rel_err_vs_fp64_solution": float(np.linalg.norm(xmp - xp) / np.linalg.norm(xp)),
            "note": ("FP32 preconditioner apply, FP64 SpMV/dots/residuals, same factor; error "
                     "against this run's FP64 solution, which the parity tests tie to the oracle's "
                     "to 1e-8"),
        }
        log("mixed: solve %.1f ms, %d iterations, error vs FP64 %.2e" % (
            sm["ms_total"], sm["iterations"], out["mixed"]["rel_err_vs_fp64_solution"]))
    del f
    return out


# --------------------------------------------------------------------------
# serving stream
# --------------------------------------------------------------------------
def run_serve(args):
    """C4: the systems one at a time in FP64 first (their service times set
    the Poisson rate: 0.7 / mean service time), then served with continuous
    batching (FP32 apply) at that rate, then all at once (burst)."""
    import numpy as np
    import torch
    from paper_2505_02977_amd import inputs, parac
    count = args.serve_count
    log("generating %d systems" % count)
    reqs, ns = [], []
    for k in range(count):
        Wk = inputs.sddm_system(k)
        reqs.append(dict(A=Wk.A, b=Wk.b, perm=Wk.perm, seed=Wk.seed, rtol=args.rtol))
        ns.append(Wk.A.n)
        if k % 20 == 19:
            log("  %d systems, sum n %d" % (k + 1, sum(ns)))
    log("one at a time (FP64)")
    service = []
    for k, rq in enumerate(reqs):
        dA = parac.DeviceCSR(rq["A"])
        b = torch.tensor(rq["b"], device="cuda")
        x = torch.empty_like(b)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        f = parac.parac_factor(dA, perm=rq["perm"], seed=rq["seed"])
        parac.parac_pcg(dA, f, b, x, rtol=args.rtol)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - ts)
        del f
        if k % 20 == 19:
            log("  %d done, %.1f s of service" % (k + 1, sum(service)))
    service = np.array(service)
    rate = 0.7 / service.mean()
    arrivals = inputs.poisson_arrivals(count, rate)
    # the same arrivals replayed one at a time
    clock, lat1 = 0.0, []
    for a, dt in zip(arrivals, service):
        clock = max(clock, a) + dt
        lat1.append(clock - a)
    lat1 = np.array(lat1)

    def serve(arr, what):
        log("serving %s (FP32 apply, %d systems in flight, a stream each)" % (what, args.serve_slots))
        rs = [dict(rq, arrival_s=float(a)) for rq, a in zip(reqs, arr)]
        t0 = time.perf_counter()
        res, _ = parac.parac_serve(rs, precision=parac.PREC_MIXED, max_slots=args.serve_slots)
        wall = time.perf_counter() - t0
        lat = np.array([r["t_done"] - r["t_arrive"] for r in res])
        log("  %s: makespan %.2f s, p50 %.3f s, p99 %.3f s" % (
            what, wall, np.percentile(lat, 50), np.percentile(lat, 99)))
        return res, wall, lat

    res, wall, lat = serve(arrivals, "Poisson arrivals %.2f/s" % rate)
    resb, wallb, latb = serve(np.zeros(count), "a burst (all at t = 0)")
    ok = all(r["status"] == 0 for r in res + resb)
    worst = max(r["true_relres"] for r in res + resb)
    return {
        "value": round(wall, 6),
        "ms_per_step": round(wall * 1e3, 3),
        "dtype": "f64 (apply f32)",
        "config": {"workload": "serve_200: %d SDDM systems, n log-uniform 1e3..1e6 (sum %d), "
                               "2D/3D grids, Chung-Lu, random geometric; Poisson arrivals at 0.7 / "
                               "mean one-at-a-time FP64 service time = %.3f/s; continuous "
                               "serving, %d systems in flight on streams of their own, FP32 apply"
                               % (count, sum(ns), rate, args.serve_slots),
                   "systems": count, "sum_n": int(sum(ns)), "parallelism": "one GPU"},
        "all_converged": ok,
        "true_relres_max": float(worst),
        "arrival_rate_per_s": round(float(rate), 6),
        "p50_latency_s": round(float(np.percentile(lat, 50)), 6),
        "p99_latency_s": round(float(np.percentile(lat, 99)), 6),
        "burst": {"makespan_s": round(wallb, 6),
                  "p50_latency_s": round(float(np.percentile(latb, 50)), 6),
                  "p99_latency_s": round(float(np.percentile(latb, 99)), 6)},
        "one_at_a_time_fp64": {"service_s_total": round(float(service.sum()), 6),
                               "service_s_mean": round(float(service.mean()), 6),
                               "p50_latency_s": round(float(np.percentile(lat1, 50)), 6),
                               "p99_latency_s": round(float(np.percentile(lat1, 99)), 6),
                               "burst_makespan_s": round(float(service.sum()), 6)},
        "roofline": None,
    }


# --------------------------------------------------------------------------
def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def cpu_baseline(name, W, rtol):
    """The CPU oracle as it stands, pinned to one core of the host: the full
    workload for the grid cases, a bounded sample of the same family for the
    power-law ones (scaled by stored entries to the full size)."""
    import oracle
    oracle.build()
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[-1]
    os.sched_setaffinity(0, {core})  # this thread only: the oracle is single-threaded C
    try:
        if name in ("grid3d_128", "grid2d_64"):
            t0 = time.perf_counter()
            f = oracle.factor(W.A, perm=W.perm, seed=W.seed)
            t1 = time.perf_counter()
            x, st = oracle.pcg(W.A, f, W.b, rtol=rtol)
            t2 = time.perf_counter()
            value = t2 - t0
            sample = ("the full workload, one run: factor %.2f s + FP64 PCG %.2f s (%d iterations)"
                      % (t1 - t0, t2 - t1, st["iterations"]))
        else:
            from paper_2505_02977_amd import inputs
            ncol = 32 if name == "chung_lu_24_x32" else 1
            S = inputs.chung_lu_workload(18, dbar=16.0 if name == "chung_lu_22" else 8.0)
            prec = 0 if name == "chung_lu_22" else 1
            t0 = time.perf_counter()
            f = oracle.factor(S.A, perm=S.perm, seed=S.seed)
            t1 = time.perf_counter()
            x, st = oracle.pcg(S.A, f, S.b, rtol=rtol, precision=prec)
            t2 = time.perf_counter()
            scale = W.A.nnz / S.A.nnz
            value = ((t1 - t0) + ncol * (t2 - t1)) * scale
            sample = ("Chung-Lu 2^18 of the same family (n %d, nnz %d): factor %.2f s + %s PCG "
                      "%.2f s (%d iterations)%s, scaled by stored entries to the full workload "
                      "(x%.1f); the oracle's cost grows faster than nnz on power-law graphs, so "
                      "this understates it" % (S.A.n, S.A.nnz, t1 - t0,
                                               "FP64" if prec == 0 else "FP32-apply", t2 - t1,
                                               st["iterations"],
                                               " x %d columns" % ncol if ncol > 1 else "", scale))
    finally:
        os.sched_setaffinity(0, set(allowed))
    return dict(value=round(value, 3), unit="s", cores=1, kind="oracle", sample=sample,
                pinned_core=core, host_cpu=host_cpu(), host_cores=len(allowed))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chung_lu_22")
    ap.add_argument("--order", choices=["random", "nnz", "mis"], default="random")
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--precision", choices=["default", "fp64", "mixed"], default="default")
    ap.add_argument("--samples", type=int, default=1,
                    help="AC(k): k sampling slots per merged neighbour (1: the plain method)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-count", type=int, default=200)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a copy of 2^27 doubles five times (read 1 GiB, write 1 GiB per "
                         "launch): the reference for scaling HBM counters")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": x.numel() * 8,
                          "calibrate_copy_bytes_written": y.numel() * 8, "launches": 5}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the single-system factorisation does not shard "
              "(the design notes say how it would); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    # long solves report their progress (host convergence checks) on stderr
    os.environ.setdefault("PARAC_VERBOSE", "1")
    from paper_2505_02977_amd import inputs, parac
    inputs.PROGRESS = log  # the large generators report their stages
    name = args.workload
    W = None
    if name == "serve_200":
        out = run_serve(args)
        args.steps, args.warmup = 1, 0
    else:
        log("generating %s" % name)
        fp64 = args.precision == "fp64"
        mixed = args.precision == "mixed"
        if name == "grid3d_128":
            W = inputs.grid3d_workload(128)
            desc = ("grid3d_128: 3D 7-point Laplacian 128^3, weights log-uniform [1e-2,1e2], "
                    "%s order, FP64 factor + %s PCG to 1e-6")
            prec = parac.PREC_MIXED if mixed else parac.PREC_FP64
        elif name == "grid2d_64":
            W = inputs.grid2d_workload(64)
            desc = ("grid2d_64: 2D 5-point Laplacian 64x64, weights U[1,2], %s order, "
                    "FP64 factor + %s PCG to 1e-6")
            prec = parac.PREC_MIXED if mixed else parac.PREC_FP64
        elif name == "chung_lu_22":
            W = inputs.chung_lu_workload(22)
            desc = ("chung_lu_22: Chung-Lu Laplacian, 2^22 generated (largest component %d), "
                    "avg degree 16, exponent 2.1, weights (0,1], %%s order; FP64 factor + %%s PCG "
                    "to 1e-6" % W.A.n)
            prec = parac.PREC_MIXED if mixed else parac.PREC_FP64
        elif name in ("chung_lu_16", "chung_lu_18", "chung_lu_20"):
            lg = int(name.split("_")[-1])
            W = inputs.chung_lu_workload(lg)
            desc = ("%s: Chung-Lu Laplacian, 2^%d generated (largest component %d), "
                    "avg degree 16, exponent 2.1, weights (0,1], %%s order; FP64 factor + %%s PCG "
                    "to 1e-6 (a smaller member of the 2^22 family, for ordering and AC(k) "
                    "studies)" % (name, lg, W.A.n))
            prec = parac.PREC_MIXED if mixed else parac.PREC_FP64
        elif name == "chung_lu_24_x32":
            W = inputs.chung_lu_workload(24, dbar=8.0, nrhs=32)
            desc = ("chung_lu_24_x32: Chung-Lu Laplacian, 2^24 generated (largest component %d), "
                    "avg degree 8, exponent 2.1, weights (0,1], %%s order, 32 right-hand sides; "
                    "FP64 factor + %%s block PCG to 1e-6" % W.A.n)
            prec = parac.PREC_FP64 if fp64 else parac.PREC_MIXED
        else:
            raise SystemExit("unknown workload " + name)
        if args.order != "random":
            import dataclasses
            kind = parac.ORDER_NNZ if args.order == "nnz" else parac.ORDER_MIS
            perm, rounds = parac.parac_order(W.A, kind, W.seed)
            W = dataclasses.replace(W, perm=perm)
            log("order %s computed on the device (%d rounds)" % (args.order, rounds))
        pdesc = "FP64" if prec == parac.PREC_FP64 else "FP32-apply (FP64 SpMV/dots/residuals)"
        desc = desc % (args.order, pdesc)
        nrhs = 32 if name == "chung_lu_24_x32" else 1
        out = run_system(args, W, desc, prec, nrhs,
                         mixed_extra=(name == "chung_lu_22" and prec == parac.PREC_FP64))
    line = {
        "metric": METRIC,
        "value": out.pop("value"),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": out.pop("ms_per_step"),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": out.pop("dtype"),
        "data": "synthetic",
        "config": out.pop("config"),
    }
    line.update(out)
    if not args.no_cpu_baseline and W is not None:
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(name, W, args.rtol)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
