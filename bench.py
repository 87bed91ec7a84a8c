#!/usr/bin/env python3
"""Benchmark of the ParAC hot path on one MI355X.  Prints one JSON line.

A step is one pass of the whole hot path over one batch of synthetic input
that is already resident on the device: the randomized elimination (setup:
checks, relabelling, persistent elimination kernel, finalisation to the solve
layout) followed by PCG with the factor to a 1e-6 relative residual (true
residual recomputed in FP64).

Workloads (--workload):
  grid3d_128   default: 3D 7-point Laplacian 128^3 (2,097,152 vertices),
               weights log-uniform [1e-2, 1e2], random order, FP64 factor and
               FP64 PCG
  grid2d_64    2D 5-point Laplacian 64x64, weights U[1,2] (small case)
  chung_lu_22  Chung-Lu power-law Laplacian, 2^22 vertices generated (largest
               component kept), average degree 16, exponent 2.1, weights
               (0,1]: FP64 factor, preconditioner applied from its FP32 copy,
               SpMV / dots / residuals in FP64
  chung_lu_24_x32  Chung-Lu 2^24, average degree 8, 32 right-hand sides:
               block PCG with the FP32 apply
  serve_200    200 SDDM systems (sizes log-uniform 1e3..1e6, mixed families)
               with Poisson arrivals, served with continuous batching (mixed
               precision) and, for comparison, one at a time in FP64
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
# HBM traffic of the apply measured with rocprofv3 counters (FETCH_SIZE,
# WRITE_SIZE), scaled by the same counters on a copy of known size; valid only
# for the kernel sources it was taken from
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_ready_traffic_grid3d_128.md")
SWEEP_SOURCES = ["ready.hip", "internal.hpp", "device.hpp"]


def sweep_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in SWEEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2505_02977_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per apply from the committed counter summary, if it was taken
    on this workload from the current sweep sources; else None."""
    import re
    if workload != "grid3d_128" or not os.path.exists(TRAFFIC_PROFILE):
        return None
    text = open(TRAFFIC_PROFILE).read()
    m1 = re.search(r"sweep-sources-sha256:\s*([0-9a-f]{64})", text)
    m2 = re.search(r"hbm-bytes-per-apply:\s*([0-9]+)", text)
    if not (m1 and m2) or m1.group(1) != sweep_source_hash():
        return None
    return int(m2.group(1))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def elim_bytes(E, n_fill, n_off, N):
    """Algorithmic bytes of one elimination: the upper adjacency read once
    (4 B index + 8 B weight per edge), every fill record written and read
    (16 B each way) with its counter increment (8 B read-modify-write), every
    factor entry written (12 B) with its counter decrement (8 B), and D,
    queue slot and column offset per pivot (24 B)."""
    return 12 * E + 40 * n_fill + 20 * n_off + 24 * N


def apply_bytes(n_off, N, elem=8):
    """Algorithmic bytes of one preconditioner apply: each solve reads every
    off-diagonal entry once (4 B index + value) and gathers one vector value
    per entry; per row, the forward solve reads its entry offset (8 B), source
    index (4 B) and right-hand side (8 B) and writes y; the backward solve
    reads its offset, D^+ and y, writes x and z (8 B) and reads its source
    index."""
    return 2 * n_off * (4 + 2 * elem) + N * (8 + 4 + 8 + elem) + N * (8 + elem + elem + elem + 8 + 4)


def roofline(info, apply_ms, n_applies, ms_elim, elem, workload):
    """The dominant unit of a step (elimination or applies, by time) against
    the HBM peak."""
    N, n_off = info["n"], info["nnz_off"]
    eb = elim_bytes(info["n_input_edges"], info["n_fill"], n_off, N)
    ab = apply_bytes(n_off, N, elem)
    if ms_elim >= apply_ms * n_applies:
        unit, nbytes, ms = "k_eliminate (one factorisation, one persistent launch)", eb, ms_elim
    else:
        unit, nbytes, ms = ("preconditioner apply (k_ready forward and backward sweeps, one "
                            "launch each)"), ab, apply_ms
    achieved = nbytes / (ms * 1e-3) / 1e9
    traffic = measured_traffic(workload) if unit.startswith("preconditioner") else None
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic, "kernel": unit,
            "algorithmic_bytes": int(nbytes), "avg_ms": round(ms, 4)}


# --------------------------------------------------------------------------
# single system (optionally several right-hand sides)
# --------------------------------------------------------------------------
def run_system(args, W, desc, precision, nrhs):
    import numpy as np
    import torch
    from paper_2505_02977_amd import parac
    dA = parac.DeviceCSR(W.A)
    b = torch.tensor(W.b, device="cuda")
    x = torch.empty_like(b)
    keep32 = precision == parac.PREC_MIXED
    torch.cuda.synchronize()

    def step(timing):
        f = parac.parac_factor(dA, perm=W.perm, seed=W.seed, keep_fp32=keep32)
        log("  factor: %.1f ms" % f.info()["ms_total"])
        sts = parac.parac_pcg(dA, f, b, x, rtol=args.rtol, precision=precision, timing=timing)
        info = f.info()
        del f
        return info, sts

    for k in range(args.warmup):
        log("warmup step %d" % k)
        step(False)
    torch.cuda.synchronize()
    infos, stss = [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        info, sts = step(True)
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
    N, n_off = info["n"], info["nnz_off"]
    elem = 4 if precision == parac.PREC_MIXED else 8
    rl = roofline(info, ms_apply, applies, ms_elim, elem, args.workload)
    if nrhs > 1:
        rl["note"] = ("block apply: algorithmic bytes counted as for one column (factor read once), "
                      "the %d-column vector traffic comes on top" % nrhs)
    X = x.cpu().numpy()
    Bh = W.b
    resid = W.A.to_scipy() @ X - Bh
    rel = np.linalg.norm(resid.reshape(N, -1), axis=0) / np.linalg.norm(Bh.reshape(N, -1), axis=0)
    out = {
        "value": round((ms_setup + ms_solve) / 1e3, 6),
        "ms_per_step": round(ms_step, 3),
        "dtype": "f64" if precision == parac.PREC_FP64 else "f64 (apply f32)",
        "config": {"workload": desc, "n": N, "nnz_L": int(W.A.nnz), "rhs": nrhs,
                   "seed": int(W.seed), "parallelism": "one GPU"},
        "t_setup_s": round(ms_setup / 1e3, 6),
        "t_solve_s": round(ms_solve / 1e3, 6),
        "t_eliminate_s": round(ms_elim / 1e3, 6),
        "factor_nnz_per_s": round((N + n_off) / (ms_setup * 1e-3), 1),
        "nnz_G": N + n_off,
        "n_fill": info["n_fill"],
        "depth": info["depth"],
        "max_gather": info["max_gather"],
        "iterations": max(s["iterations"] for s in sts),
        "true_relres_max": float(rel.max()),
        "apply_ms": round(ms_apply, 4),
        "workers": info["workers"],
        "roofline": rl,
    }
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
        log("serving %s (continuous batching, FP32 apply, %d slots)" % (what, args.serve_slots))
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
                               "batching, %d slots, FP32 apply"
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
def cpu_baseline(name, W, rtol):
    """The CPU oracle as it stands, one core: the full workload for the grid
    cases, a bounded sample otherwise."""
    import oracle
    oracle.build()
    if name in ("grid3d_128", "grid2d_64"):
        t0 = time.perf_counter()
        f = oracle.factor(W.A, perm=W.perm, seed=W.seed)
        t1 = time.perf_counter()
        x, st = oracle.pcg(W.A, f, W.b, rtol=rtol)
        t2 = time.perf_counter()
        return dict(value=round(t2 - t0, 3), unit="s", cores=1, kind="oracle",
                    sample="the full workload, one run: factor %.2f s + PCG %.2f s (%d iterations)"
                    % (t1 - t0, t2 - t1, st["iterations"]))
    from paper_2505_02977_amd import inputs
    S = inputs.chung_lu_workload(16, dbar=16.0 if name == "chung_lu_22" else 8.0)
    t0 = time.perf_counter()
    f = oracle.factor(S.A, perm=S.perm, seed=S.seed)
    t1 = time.perf_counter()
    x, st = oracle.pcg(S.A, f, S.b, rtol=rtol, precision=1)
    t2 = time.perf_counter()
    scale = W.A.nnz / S.A.nnz
    return dict(value=round((t2 - t0) * scale, 3), unit="s", cores=1, kind="oracle",
                sample="Chung-Lu 2^16 of the same family (nnz %d), factor %.2f s + PCG %.2f s "
                       "(%d iterations, FP32 apply), scaled by nnz to the full workload (%.0fx); "
                       "one right-hand side" % (S.A.nnz, t1 - t0, t2 - t1, st["iterations"], scale))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grid3d_128")
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-count", type=int, default=200)
    ap.add_argument("--serve-slots", type=int, default=32)
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

    from paper_2505_02977_amd import inputs, parac
    inputs.PROGRESS = log  # the large generators report their stages
    name = args.workload
    W = None
    if name == "serve_200":
        out = run_serve(args)
        args.steps, args.warmup = 1, 0
    else:
        log("generating %s" % name)
        if name == "grid3d_128":
            W = inputs.grid3d_workload(128)
            desc = ("grid3d_128: 3D 7-point Laplacian 128^3, weights log-uniform [1e-2,1e2], "
                    "random order, FP64 factor + FP64 PCG to 1e-6")
            out = run_system(args, W, desc, parac.PREC_FP64, 1)
        elif name == "grid2d_64":
            W = inputs.grid2d_workload(64)
            desc = ("grid2d_64: 2D 5-point Laplacian 64x64, weights U[1,2], random order, "
                    "FP64 factor + FP64 PCG to 1e-6")
            out = run_system(args, W, desc, parac.PREC_FP64, 1)
        elif name == "chung_lu_22":
            W = inputs.chung_lu_workload(22)
            desc = ("chung_lu_22: Chung-Lu Laplacian, 2^22 generated (largest component %d), "
                    "avg degree 16, exponent 2.1, weights (0,1], random order; FP64 factor, "
                    "FP32 copy for the apply, FP64 SpMV/dots/residuals, to 1e-6" % W.A.n)
            out = run_system(args, W, desc, parac.PREC_MIXED, 1)
        elif name == "chung_lu_24_x32":
            W = inputs.chung_lu_workload(24, dbar=8.0, nrhs=32)
            desc = ("chung_lu_24_x32: Chung-Lu Laplacian, 2^24 generated (largest component %d), "
                    "avg degree 8, exponent 2.1, weights (0,1], 32 right-hand sides; FP64 factor, "
                    "block PCG with the FP32 apply" % W.A.n)
            out = run_system(args, W, desc, parac.PREC_MIXED, 32)
        else:
            raise SystemExit("unknown workload " + name)
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
