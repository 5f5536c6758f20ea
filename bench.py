#!/usr/bin/env python
"""Benchmark of the multigrid pressure solve on one MI355X.

Workload (default): the 512^3 drop-splash field with a Fourier-perturbed film
(density ratio 1000, divergence right-hand side, seed 2), coarsest grid 8^3,
V(2,2) cycles.  One step = one solve to relative residual 1e-10 from p = 0 with
the FP32-refined solver (FP32 V-cycles inside FP64 iterative refinement), the
hierarchy already resident (setup is timed separately and reported).  The same
number of plain FP64 multigrid solves is timed for the comparison the metric
asks for.

Prints ONE JSON line.  value = milliseconds per FP32-refined solve (lower is
better); extra keys carry the FP64 time, the speed ratio, achieved HBM GB/s per
V-cycle, cell-updates/s, the roofline of the dominant kernel and the CPU oracle
baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ["paper_1410_8568_amd/csrc/mg_kernels.h", "paper_1410_8568_amd/csrc/mg_core.hip"]   # kernels and their launch shapes
METRIC = "time to 1e-10 residual + HBM GB/s per V-cycle; FP32-refined vs FP64 MG"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_solves(S, b, p, steps, warmup, tol):
    import torch
    for _ in range(warmup):
        p.zero_()
        st = S.solve(b, p, tol=tol)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stats = []
    e0.record()
    t0 = time.perf_counter()
    for _ in range(steps):
        p.zero_()
        stats.append(S.solve(b, p, tol=tol))
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    return e0.elapsed_time(e1) / steps, wall / steps, stats


def profiled(build, b, p, tol):
    """One extra solve of the same workload with the library's profile mode on:
    every kernel launch bracketed by HIP events on the solve stream."""
    S, _ = build(profile=True)
    p.zero_()
    st = S.solve(b, p, tol=tol)
    S.close()
    return st


def cpu_baseline(P, n_coarsest, precision, tol):
    """The oracle timed on the host: the same solve (precision, tolerance, coarsest
    grid) of the same input to convergence, from p = 0; the time after the
    hierarchy setup is reported (the GPU step excludes setup too).  Returns the
    baseline record and the oracle's solution."""
    import oracle
    oracle.lib()
    t0 = time.perf_counter()
    r = oracle.solve(P.bx, P.by, P.bz, P.b, n_coarsest=n_coarsest, max_cycles=60, tol=tol, precision=precision)
    wall = time.perf_counter() - t0
    setup_s, rest_s = oracle.last_timing()
    rec = dict(value=rest_s * 1e3, unit="ms", cores=oracle.num_threads(), kind="oracle",
               sample=f"{precision} oracle on the same {P.n[0]}^3 input to relative residual {tol:g} "
                      f"({r['status']}, {r['cycles']} outer iterations, final {r['history'][-1]:.2e}), "
                      f"measured after {setup_s:.2f} s of hierarchy setup; {wall:.1f} s of CPU wall time in all")
    return rec, r


def oracle_reference(P, n_coarsest):
    """p*: the oracle's FP64 solve to relative residual 1e-13 (or stagnation)."""
    import oracle
    t0 = time.perf_counter()
    r = oracle.solve(P.bx, P.by, P.bz, P.b, n_coarsest=n_coarsest, max_cycles=60, tol=1e-13)
    return r, time.perf_counter() - t0


# Algorithmic HBM bytes per cell of the two projection kernels (FP64): the
# divergence reads the three face velocities and writes b; the correction reads
# p and the three lower-face coefficients and reads and writes the velocities.
PROJ_BYTES_PER_CELL = {"divergence": 32, "correct_velocity": 80}


def projection_bench(S, n, steps, warmup, tol, dev):
    """The projection step around the solve on the same coefficient field: MAC
    divergence of a random face velocity (interior N(0,1), walls 0, seed 37),
    the solve, and the velocity correction; dt = 1e-3, h = 1/n.  Each kernel is
    timed over 10 back-to-back launches with HIP events on the stream it runs on;
    the whole step (divergence + solve + correction, blocking) per step."""
    import numpy as np
    import torch
    from paper_1410_8568_amd import inputs, mg
    t = time.perf_counter()
    u0, v0, w0 = (torch.from_numpy(a).to(dev) for a in inputs.velocity_field((n, n, n), np.random.default_rng(37)))
    log(f"generated the {n}^3 velocity field in {time.perf_counter() - t:.1f} s")
    u, v, w = u0.clone(), v0.clone(), w0.clone()
    b = torch.empty((n, n, n), dtype=torch.float64, device=dev)
    p = torch.zeros_like(b)
    h, dt = 1.0 / n, 1e-3
    N = n ** 3

    def per_launch(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    step_ms, st = [], None
    for i in range(warmup + steps):
        u.copy_(u0)
        v.copy_(v0)
        w.copy_(w0)
        p.zero_()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        st = S.project(u, v, w, dt, h, p=p, b=b, tol=tol)
        e1.record()
        torch.cuda.synchronize()
        if i >= warmup:
            step_ms.append(e0.elapsed_time(e1))
    ms = {"divergence": per_launch(lambda: mg.divergence(u0, v0, w0, h / dt, b)),
          "correct_velocity": per_launch(lambda: S.correct_velocity(p, u, v, w, dt / h))}
    out = {"workload": f"projection step on the same field: random face velocity (seed 37), dt {dt:g}, h 1/{n}",
           "ms_per_step": sorted(step_ms)[len(step_ms) // 2], "outer": st["outer"],
           "final_rel_residual": st["rel_residual"]}
    for k, v_ms in ms.items():
        byt = PROJ_BYTES_PER_CELL[k] * N
        gbps = byt / (v_ms * 1e-3) / 1e9
        out[k] = {"avg_launch_ms": v_ms, "bytes_per_launch": byt, "achieved_gbps": gbps,
                  "frac": gbps / HBM_PEAK_GBPS}
    del u0, v0, w0, u, v, w
    return out


def levelset_bench(n, dev):
    """The face coefficients of the benchmark field built on the device from its
    level set (drop splash, Fourier-perturbed film, seed 2, eps = 1.5 h): 10
    back-to-back launches timed with HIP events on the launch stream; algorithmic
    bytes 8 (phi) + 24 (three faces) per cell."""
    import torch
    from paper_1410_8568_amd import inputs, mg
    phi = torch.from_numpy(inputs.drop_splash_levelset(n, seed=2, perturb=True)).to(dev)
    out = mg.faces_from_levelset(phi, 1000.0, 1.0, 1.5 / n)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        mg.faces_from_levelset(phi, 1000.0, 1.0, 1.5 / n, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    byt = 32 * n ** 3
    del phi, out
    return {"avg_launch_ms": ms, "bytes_per_launch": byt, "achieved_gbps": byt / (ms * 1e-3) / 1e9,
            "frac": byt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS}


def kernel_source_sha():
    """Hash of the kernel sources' code: comments and blank lines are left out, so
    a change of wording alone keeps the counter summary valid."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, f), encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = (re.sub(r"//.*", "", ln).rstrip() for ln in text.splitlines())
        h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()[:16]


def traffic_for(kernel, n):
    """HBM bytes per launch of `kernel` on the n^3 workload from the committed
    counter summary, or None if there is none for that workload or the kernel
    sources changed since it was taken."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except Exception:
        return None
    sha = kernel_source_sha()
    for e in t.get("entries", [t]):
        if e.get("source_sha") == sha and e.get("class") == kernel and e.get("n") == n:
            return e.get("bytes_per_launch")
    return None


def calibrate_copy(gib=1, reps=5):
    """A plain device copy of known size, for scaling the FETCH_SIZE/WRITE_SIZE counters."""
    import torch
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes_read": 4 * n, "calibrate_copy_bytes_written": 4 * n, "reps": reps}))


def _counter_rows(d):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        rows += list(csv.DictReader(open(f)))
    return rows


def write_traffic(fetch_dir, write_dir, cal_fetch_dir, cal_write_dir, n, gib=1):
    """profiles/traffic.json from four rocprofv3 --pmc runs: FETCH_SIZE and
    WRITE_SIZE over the bench, and over --calibrate-copy.  The counters (KiB per
    dispatch) are scaled by what they read for the plain copy of known size.  The
    kernel class is the FP32 fine-grid smoother: among the k_rb_sweep<float, ...>
    dispatches of the solves (from the first finest-level residual pass on; the
    setup's tuning runs come before), every dispatch whose fetch is at least 20% of the
    largest (the finest level; the next level moves 8x less, and the finest
    level's passes differ by up to 2.4x: a pass entering from zero reads no
    iterate, the last one also updates the FP64 iterate), fused-restriction,
    plain and update passes alike, as the bench's roofline averages over all.  The finest
    level's dispatches of each kernel are picked in each run by its own counter and
    paired by their order.  n: the grid size of
    the bench run the counters were taken on."""
    copy_bytes = gib * (1 << 30)

    def copy_kib(d):
        import statistics
        v = [float(r["Counter_Value"]) for r in _counter_rows(d) if "copyBuffer" in r["Kernel_Name"]]
        return statistics.median(v)

    fs = copy_bytes / (copy_kib(cal_fetch_dir) * 1024.0)
    ws = copy_bytes / (copy_kib(cal_write_dir) * 1024.0)

    def groups(d):
        # dispatches from the first solve on (the setup's smoother tuning comes before it)
        rows = sorted(_counter_rows(d), key=lambda r: int(r["Dispatch_Id"]))
        first = min(int(r["Dispatch_Id"]) for r in rows
                    if r["Kernel_Name"].startswith(("void mgk::k_resid_flat", "void mgk::k_resid_cells")))
        g = {}
        for r in rows:
            if int(r["Dispatch_Id"]) >= first and r["Kernel_Name"].startswith("void mgk::k_rb_sweep<float"):
                g.setdefault((r["Kernel_Name"].split("(")[0], r["Grid_Size"]), []).append(float(r["Counter_Value"]))
        return g

    def finest(g):
        # the finest level's dispatches of each kernel, in order (the two runs may tune
        # coarser levels differently, so the groups are filtered before pairing)
        top = max(max(v) for v in g.values())
        out = {}
        for (name, _), v in sorted(g.items()):
            out.setdefault(name, []).extend(x for x in v if x >= 0.2 * top)
        return out

    F, W = finest(groups(fetch_dir)), finest(groups(write_dir))
    fetch, write, kernels = [], [], set()
    for name, fv in F.items():
        wv = W.get(name, [])
        for f, w in zip(fv, wv):
            fetch.append(f * 1024.0 * fs)
            write.append(w * 1024.0 * ws)
            kernels.add(name.replace("void mgk::", ""))
    out = {"class": "smooth_fine", "n": n, "kernels": sorted(kernels), "dispatches": len(fetch),
           "fetch_bytes": sum(fetch) / len(fetch), "write_bytes": sum(write) / len(write),
           "bytes_per_launch": (sum(fetch) + sum(write)) / len(fetch), "fetch_scale": fs, "write_scale": ws,
           "source_sha": kernel_source_sha()}
    # one entry per grid size; entries of other sizes taken on the same kernel code stay
    try:
        old = json.load(open(TRAFFIC_FILE))
        entries = [e for e in old.get("entries", [old])
                   if e.get("n") != n and e.get("source_sha") == out["source_sha"]]
    except Exception:
        entries = []
    with open(TRAFFIC_FILE, "w") as f:
        json.dump({"entries": sorted(entries + [out], key=lambda e: e["n"])}, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


def summarize(d):
    """Markdown summary of rocprofv3 CSV output in directory d (kernel stats,
    per-dispatch durations by grid size, counters per dispatch)."""
    import csv
    import glob
    import statistics
    out = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)):
        rows = list(csv.DictReader(open(f)))
        out.append(f"### kernel stats ({os.path.basename(f)})\n")
        out.append("| kernel | calls | total ms | avg us | % |\n|---|---|---|---|---|")
        for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:20]:
            out.append(f"| {r['Name'][:90]} | {r['Calls']} | {float(r['TotalDurationNs'])/1e6:.3f} | "
                       f"{float(r['AverageNs'])/1e3:.2f} | {float(r['Percentage']):.1f} |")
        out.append("")
    for f in sorted(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)):
        rows = list(csv.DictReader(open(f)))
        groups = {}
        for r in rows:
            key = (r["Kernel_Name"][:90], r.get("Grid_Size", r.get("Grid_Size_X", "?")))
            groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        out.append(f"### dispatches by kernel and grid size ({os.path.basename(f)})\n")
        out.append("| kernel | grid | calls | avg us | median us |\n|---|---|---|---|---|")
        for (k, g), v in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:25]:
            out.append(f"| {k} | {g} | {len(v)} | {statistics.mean(v):.2f} | {statistics.median(v):.2f} |")
        out.append("")
    for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        rows = list(csv.DictReader(open(f)))
        groups = {}
        for r in rows:
            key = (r["Kernel_Name"][:90], r["Grid_Size"], r["Counter_Name"])
            groups.setdefault(key, []).append(float(r["Counter_Value"]))
        out.append(f"### counters per dispatch ({os.path.basename(f)})\n")
        out.append("| kernel | grid | counter | dispatches | avg KiB |\n|---|---|---|---|---|")
        for (k, g, c), v in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:25]:
            out.append(f"| {k} | {g} | {c} | {len(v)} | {statistics.mean(v):.1f} |")
        out.append("")
    print("\n".join(out))


def ratio_sweep(args):
    """Drop splash (Fourier-perturbed film, seed 2) at n^3 (default 256) for density
    ratios 1e1..1e5 with arithmetic and harmonic faces: FP64 V-cycle iteration,
    FP64 flexible CG and FP32-refined V-cycles, each solved from p = 0 to the
    tolerance (median of `steps` timed solves after `warmup`).  One JSON line per
    case, then a summary line."""
    import torch
    from paper_1410_8568_amd import inputs, mg
    n = args.n if args.n != 512 else 256
    rows = []
    for faces in ("arith", "harmonic"):
        for ratio in (1e1, 1e2, 1e3, 1e4, 1e5):
            P = inputs.drop_splash_problem(n, 0.1, (0.5, 0.5, 0.2, 0.08), ratio, 1.0, seed=2, perturb=True,
                                           faces=faces)
            bx, by, bz, b = mg.to_device(P)
            p = torch.zeros_like(b)
            row = {"n": n, "faces": faces, "ratio": ratio}
            for name, prec, kry in (("fp64_mg", "fp64", "none"), ("fp64_fcg", "fp64", "fcg"),
                                    ("fp32_refined_mg", "fp32_refined", "none")):
                S = mg.Solver(bx, by, bz, precision=prec, n_coarsest=args.n_coarsest, graph=bool(args.graph),
                              krylov=kry)
                ms, _, st = timed_solves(S, b, p, args.steps, args.warmup, args.tol)
                S.close()
                last = st[-1]
                row[name] = {"ms": ms, "cycles": last["cycles"], "gamma": last["gamma"],
                             "rel_residual": last["rel_residual"], "rc": last["rc"]}
            rows.append(row)
            log(json.dumps(row))
            del bx, by, bz, b, p
            torch.cuda.empty_cache()
    print(json.dumps({"sweep": "density ratio", "tol": args.tol, "n_coarsest": args.n_coarsest, "rows": rows}),
          flush=True)


VARIANT_SET = [
    ("default", {}),
    ("sor_1.1", {"omega": 1.1}),
    ("sor_1.2", {"omega": 1.2}),
    ("sor_1.3", {"omega": 1.3}),
    ("restrict64", {"restrict64": True}),
    ("coarse_gmres16_1e-2", {"coarse_gmres": 16, "coarse_gmres_tol": 1e-2, "coarse_gmres_maxit": 500}),
    ("coarse_gmres16_1e-6", {"coarse_gmres": 16, "coarse_gmres_tol": 1e-6, "coarse_gmres_maxit": 2000}),
    ("sor_1.2+restrict64", {"omega": 1.2, "restrict64": True}),
]


def variant_bench(args):
    """The paper-faithful cycle variants on the benchmark's drop-splash field:
    cycles, gamma and time to the tolerance for the FP64 and FP32-refined
    solvers (every variant runs the fused smoother passes; the 64-point
    restriction adds a separate residual pass and its gather).  One JSON line
    per variant, then a summary line."""
    import torch
    from paper_1410_8568_amd import inputs, mg
    P = inputs.config2(args.n)
    bx, by, bz, b = mg.to_device(P)
    p = torch.zeros_like(b)
    rows = []
    for name, kw in VARIANT_SET:
        row = {"variant": name, "options": kw}
        for prec in ("fp64", "fp32_refined"):
            S = mg.Solver(bx, by, bz, precision=prec, n_coarsest=args.n_coarsest, graph=bool(args.graph), **kw)
            ms, _, st = timed_solves(S, b, p, args.steps, args.warmup, args.tol)
            S.close()
            last = st[-1]
            row[prec] = {"ms": ms, "cycles": last["cycles"], "outer": last["outer"], "gamma": last["gamma"],
                         "rel_residual": last["rel_residual"]}
        rows.append(row)
        log(json.dumps(row))
    print(json.dumps({"variants": f"drop splash {args.n}^3, ratio 1000, coarsest {args.n_coarsest}^3",
                      "tol": args.tol, "rows": rows}), flush=True)


def batch_bench(args):
    """64 uneven problems (sizes 32..128^3, 1-8 drops, ratio 10..1000): all submitted
    at once to the continuous-batching server vs solved one after another."""
    import torch
    from paper_1410_8568_amd import inputs, mg
    t = time.perf_counter()
    probs = inputs.batch_problems(args.batch_count)
    log(f"generated {len(probs)} batch problems in {time.perf_counter() - t:.1f} s")
    dev = [mg.to_device(P) for P in probs]
    cells = sum(P.cells for P in probs)
    prec = "fp32_refined"
    # warm the tuner cache for every size class
    for n in sorted({P.n for P in probs}):
        P = next(Q for Q in probs if Q.n == n)
        mg.Solver(*mg.to_device(P)[:3], precision=prec).close()
    torch.cuda.synchronize()
    t = time.perf_counter()
    seq_cycles = 0
    for (bx, by, bz, b) in dev:
        S = mg.Solver(bx, by, bz, precision=prec)
        p = torch.zeros_like(b)
        st = S.solve(b, p, tol=args.tol)
        seq_cycles += st["cycles"] * b.numel()
        S.close()
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t
    o = mg.options(precision=prec)
    arena = sum(mg.server_request_bytes(P.n, o) for P in probs) + (1 << 20)
    srv = mg.Server(arena, precision=prec, max_slots=args.slots)
    outs = [torch.zeros_like(b) for (_, _, _, b) in dev]
    torch.cuda.synchronize()
    t = time.perf_counter()
    tickets = [srv.submit(bx, by, bz, b, p, tol=args.tol) for (bx, by, bz, b), p in zip(dev, outs)]
    res = [srv.wait(tk) for tk in tickets]
    srv_s = time.perf_counter() - t
    info = srv.stats()
    srv.close()
    bad = [r["rc"] for r in res if r["rc"] != 0]
    lat = sorted(r["finish_ms"] - r["submit_ms"] for r in res)
    out = {
        "metric": "batched uneven solves: solves/s (FP32-refined, tol %g)" % args.tol,
        "value": len(probs) / srv_s, "unit": "solves/s", "higher_is_better": True,
        "n_gpus": 1, "data": "synthetic",
        "config": {"workload": f"{len(probs)} problems n~U{{32,64,96,128}}, 1-8 drops, film 0.05-0.2, "
                               f"ratio U{{10,100,1000}}, seeds 3 / 3000+i", "cells": cells,
                   "slots": args.slots},
        "server_s": srv_s, "sequential_s": seq_s, "speedup_vs_sequential": seq_s / srv_s,
        "cell_updates_per_s": seq_cycles / srv_s, "failed": len(bad),
        "latency_ms_p50": lat[len(lat) // 2], "latency_ms_max": lat[-1],
        "server_batching": info,
    }
    print(json.dumps(out), flush=True)


def serve_bench(args):
    """Open-loop Poisson arrivals of solves with n ~ U{64,128,192,256} and batch-like
    geometry; p50/p99 latency (submit to finish) and achieved solves/s per rate.

    Each request's face coefficients are built on the device from its scene's level
    set (mg_faces_from_levelset: indicator, eq. 8, face means) on a producer
    stream at arrival, and the request is submitted on that stream (the server
    starts on it after the face build); --faces host submits faces built on the
    host beforehand instead."""
    import numpy as np
    import torch
    from paper_1410_8568_amd import inputs, mg
    prec = "fp32_refined"
    rates = [float(r) for r in args.rates.split(",")]
    # a pool of distinct scenes per size class (requests reuse the pool's scenes):
    # the level set, density ratio and rhs on the device
    pool = {}
    t = time.perf_counter()
    for i, d in enumerate(inputs.request_stream(4 * args.pool, 1.0)):
        desc = d[1]
        if len(pool.setdefault(desc["n"], [])) < args.pool:
            P = inputs.problem_from_desc(desc)
            dv = mg.to_device(P)
            phi = torch.from_numpy(inputs.scene_levelset(desc)).cuda()
            pool[desc["n"]].append(dict(faces=dv[:3], b=dv[3], phi=phi, ratio=desc["ratio"]))
    log(f"generated request pool {[(n, len(v)) for n, v in sorted(pool.items())]} in {time.perf_counter() - t:.1f} s")
    for n, v in pool.items():
        mg.Solver(*v[0]["faces"], precision=prec).close()   # warm the tuner cache
    arena = int(args.arena_gb * (1 << 30))
    prod = torch.cuda.Stream()
    lines = []
    for rate in rates:
        stream = inputs.request_stream(args.requests, rate, seed=4)
        srv = mg.Server(arena, precision=prec, max_slots=args.slots)
        tickets = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, (ta, d) in enumerate(stream):
            while time.perf_counter() - t0 < ta:
                time.sleep(0.0001)
            e = pool[d["n"]][i % len(pool[d["n"]])]
            n = d["n"]
            with torch.cuda.stream(prod):
                p = torch.zeros_like(e["b"])
                if args.faces == "device":
                    faces = mg.faces_from_levelset(e["phi"], e["ratio"], 1.0, 1.5 / n, stream=prod)
                else:
                    faces = e["faces"]
                tickets.append((i, srv.submit(*faces, e["b"], p, tol=args.tol, stream=prod)))
        res = [srv.wait(tk, timeout_s=600) for _, tk in tickets]
        span = time.perf_counter() - t0
        info = srv.stats()
        srv.close()
        lat = np.array([r["finish_ms"] - r["submit_ms"] for r in res])
        line = {"rate_per_s": rate, "requests": len(res), "solves_per_s": len(res) / span,
                "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
                "failed": int(sum(r["rc"] != 0 for r in res)), "max_batch": info["max_batch"],
                "problems_per_replay": info["problem_iterations"] / max(1, info["replays"])}
        log(json.dumps(line))
        lines.append(line)
    out = {"metric": "serving: p50/p99 latency and solves/s under Poisson arrivals (FP32-refined)",
           "value": lines[-1]["solves_per_s"], "unit": "solves/s", "higher_is_better": True, "n_gpus": 1,
           "data": "synthetic",
           "config": {"workload": f"n~U{{64,128,192,256}}, batch-like geometry, {args.requests} requests per rate, "
                                  f"pool of {args.pool} scenes per size, faces built on the {args.faces}",
                      "arena_gb": args.arena_gb, "slots": args.slots},
           "rates": lines}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--n-coarsest", type=int, default=8)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tight-tol", type=float, default=1e-11,
                    help="also time both solvers to this tolerance (0: skip): the one at which the FP32-refined "
                         "result is within 1e-8 of the FP64 oracle's p* with margin")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--inner-m", type=int, default=0, help="FP32 V-cycles per outer iteration (0: library default)")
    ap.add_argument("--graph", type=int, default=1, help="replay each outer iteration as a HIP graph (1) or launch eagerly (0)")
    ap.add_argument("--projection", type=int, default=1,
                    help="also time the projection step around the solve (divergence, solve, correction)")
    ap.add_argument("--krylov", type=int, default=1,
                    help="also time the FP64 Krylov solve (flexible CG preconditioned by one V-cycle)")
    ap.add_argument("--sor-omega", type=float, default=1.2,
                    help="also time the FP32-refined solve with this SOR factor (1: skip)")
    ap.add_argument("--sweep", action="store_true",
                    help="density-ratio sweep (1e1..1e5, arithmetic and harmonic faces) of the three solvers")
    ap.add_argument("--variants", action="store_true",
                    help="cycles, gamma and time of the paper-faithful cycle variants (SOR, 64-point restriction, "
                         "coarse GMRES)")
    ap.add_argument("--calibrate-copy", action="store_true", help="run a 1 GiB device copy (counter scale)")
    ap.add_argument("--summarize", metavar="DIR", help="print a markdown summary of rocprofv3 CSV output")
    ap.add_argument("--traffic", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "CAL_FETCH_DIR", "CAL_WRITE_DIR"),
                    help="write profiles/traffic.json from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs")
    ap.add_argument("--batch", action="store_true", help="batched uneven solves through the server")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--serve", action="store_true", help="Poisson-arrival serving sweep")
    ap.add_argument("--rates", default="50,100,200,300,400,500")
    ap.add_argument("--requests", type=int, default=1000)
    ap.add_argument("--pool", type=int, default=2)
    ap.add_argument("--arena-gb", type=float, default=24.0)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--faces", choices=["device", "host"], default="device",
                    help="serving: build each request's faces on the device from its level set, or on the host")
    args = ap.parse_args()
    if args.traffic:
        write_traffic(*args.traffic, n=args.n)
        return
    if args.summarize:
        summarize(args.summarize)
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.variants:
        if args.gpus != 1:
            print("bench.py: one GPU only", file=sys.stderr)
            sys.exit(2)
        import torch
        torch.cuda.set_device(0)
        variant_bench(args)
        return
    if args.sweep:
        if args.gpus != 1:
            print("bench.py: one GPU only", file=sys.stderr)
            sys.exit(2)
        import torch
        torch.cuda.set_device(0)
        ratio_sweep(args)
        return
    if args.batch or args.serve:
        if args.gpus != 1:
            print("bench.py: one GPU only", file=sys.stderr)
            sys.exit(2)
        import torch
        torch.cuda.set_device(0)
        batch_bench(args) if args.batch else serve_bench(args)
        return
    if args.gpus != 1:
        print(f"bench.py: this solver runs on one GPU; --gpus {args.gpus} is not supported "
              f"(independent problems shard across GPUs without communication; one large solve "
              f"would need a halo-exchange domain decomposition, which is not built)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1410_8568_amd import inputs, mg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t = time.perf_counter()
    P = inputs.config2(args.n)
    log(f"generated {args.n}^3 drop-splash input in {time.perf_counter() - t:.1f} s")
    bx, by, bz, b = mg.to_device(P, dev)
    torch.cuda.synchronize()
    N = args.n ** 3

    def build(precision, profile=False, krylov="none", omega=1.0):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kw = {"inner_m": args.inner_m} if args.inner_m else {}
        S = mg.Solver(bx, by, bz, precision=precision, n_coarsest=args.n_coarsest, profile=profile,
                      graph=args.graph and not profile, krylov=krylov, omega=omega, **kw)
        torch.cuda.synchronize()
        return S, (time.perf_counter() - t0) * 1e3

    p = torch.zeros_like(b)
    S32, setup32 = build("fp32_refined")
    log(f"fp32_refined setup {setup32:.1f} ms")
    ms32, wall32, st32 = timed_solves(S32, b, p, args.steps, args.warmup, args.tol)
    last32 = st32[-1]
    p32 = p.clone()
    host32 = p32.cpu().numpy()
    log(f"fp32_refined: {ms32:.2f} ms/solve, outer {last32['outer']}, rho {last32['rel_residual']:.2e}")
    tight, tight_host = {}, {}
    if args.tight_tol > 0:
        # the tolerance at which the error against the FP64 oracle's p* is well inside 1e-8
        mst, _, stt = timed_solves(S32, b, p, max(2, args.steps // 4), 1, args.tight_tol)
        tight["fp32_refined_ms"] = mst
        tight["fp32_refined_cycles"] = stt[-1]["cycles"]
        tight_host["fp32_refined_tol_%g" % args.tight_tol] = p.cpu().numpy()
    S32.close()
    prof32 = profiled(lambda profile: build("fp32_refined", profile), b, p, args.tol)

    res = {}
    host64 = None
    if not args.no_fp64:
        S64, setup64 = build("fp64")
        ms64, wall64, st64 = timed_solves(S64, b, p, args.steps, args.warmup, args.tol)
        last64 = st64[-1]
        log(f"fp64: {ms64:.2f} ms/solve, cycles {last64['cycles']}, rho {last64['rel_residual']:.2e}")
        p64 = p.clone()
        host64 = p64.cpu().numpy()
        if args.tight_tol > 0:
            mst, _, stt = timed_solves(S64, b, p, max(2, args.steps // 4), 1, args.tight_tol)
            tight["fp64_ms"] = mst
            tight["fp64_cycles"] = stt[-1]["cycles"]
            tight["speedup_fp32_refined_vs_fp64"] = mst / tight["fp32_refined_ms"]
            tight_host["fp64_tol_%g" % args.tight_tol] = p.cpu().numpy()
            a32 = tight_host["fp32_refined_tol_%g" % args.tight_tol]
            a64 = tight_host["fp64_tol_%g" % args.tight_tol]
            tight["rel_l2_fp32_refined_vs_fp64"] = float(np.linalg.norm(a32 - a64) / np.linalg.norm(a64))
        S64.close()
        prof64 = profiled(lambda profile: build("fp64", profile), b, p, args.tol)
        rel = (torch.linalg.vector_norm(p32 - p64) / torch.linalg.vector_norm(p64)).item()
        res.update(fp64_ms_per_solve=ms64, fp64_setup_ms=setup64, fp64_cycles=last64["cycles"],
                   fp64_final_rel_residual=last64["rel_residual"], fp64_gamma=last64["gamma"],
                   speedup_fp32_refined_vs_fp64=ms64 / ms32,
                   rel_l2_fp32_refined_vs_fp64=rel)
        cyc64 = last64["cycles"]
        bytes64 = sum(prof64["kernel_bytes"].values())
        res["fp64_gbps_per_vcycle"] = bytes64 / cyc64 / 1e6 / (ms64 / cyc64)
        res["fp64_cell_updates_per_s"] = N * cyc64 / (ms64 * 1e-3)
    if args.sor_omega != 1.0:
        # the same FP32-refined solve with over-relaxed smoothing (the paper's red-black SOR)
        SS, _ = build("fp32_refined", omega=args.sor_omega)
        mss, _, sts = timed_solves(SS, b, p, args.steps, args.warmup, args.tol)
        SS.close()
        lasts = sts[-1]
        res["fp32_refined_sor"] = {"omega": args.sor_omega, "ms_per_solve": mss, "cycles": lasts["cycles"],
                                   "outer": lasts["outer"], "final_rel_residual": lasts["rel_residual"]}
        if "fp64_ms_per_solve" in res:
            res["fp32_refined_sor"]["speedup_vs_fp64_mg"] = res["fp64_ms_per_solve"] / mss
        log(f"fp32_refined omega {args.sor_omega}: {mss:.2f} ms/solve, cycles {lasts['cycles']}")
    if args.krylov:
        # FP64 flexible CG preconditioned by one V-cycle per iteration
        SK, setupk = build("fp64", krylov="fcg")
        msk, wallk, stk = timed_solves(SK, b, p, args.steps, args.warmup, args.tol)
        lastk = stk[-1]
        SK.close()
        profk = profiled(lambda profile: build("fp64", profile, krylov="fcg"), b, p, args.tol)
        kk = profk["kernel_ms"]["krylov"]
        res["fp64_fcg"] = {"ms_per_solve": msk, "iterations": lastk["cycles"],
                           "final_rel_residual": lastk["rel_residual"], "gamma": lastk["gamma"],
                           "krylov_passes_gbps": profk["kernel_bytes"]["krylov"] / (kk * 1e-3) / 1e9 if kk else None,
                           "krylov_passes_ms": kk,
                           "vcycle_ms": sum(v for k, v in profk["kernel_ms"].items() if k != "krylov")}
        if "fp64_ms_per_solve" in res:
            res["fp64_fcg"]["speedup_vs_fp64_mg"] = res["fp64_ms_per_solve"] / msk
        log(f"fp64 fcg: {msk:.2f} ms/solve, iterations {lastk['cycles']}, rho {lastk['rel_residual']:.2e}")

    if args.projection:
        Sp, _ = build("fp32_refined")
        res["projection_step"] = projection_bench(Sp, args.n, args.steps, args.warmup, args.tol, dev)
        Sp.close()
        log(f"projection step: {json.dumps(res['projection_step'])}")

    if args.projection:
        res["levelset_faces"] = levelset_bench(args.n, dev)
        log(f"faces from the level set: {json.dumps(res['levelset_faces'])}")

    # dominant kernel of the timed (FP32-refined) step, from the profiled solve
    kms = prof32["kernel_ms"]
    dom = max((k for k in kms if k != "smooth"), key=lambda k: kms[k])
    dom_launch = prof32["kernel_launches"][dom]
    dom_avg_ms = kms[dom] / dom_launch
    dom_bytes = prof32["kernel_bytes"][dom] / dom_launch
    achieved = dom_bytes / (dom_avg_ms * 1e-3) / 1e9
    cyc32 = last32["cycles"]
    bytes32 = sum(prof32["kernel_bytes"].values())

    out = {
        "metric": METRIC,
        "value": ms32,
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32-inner/f64-outer",
        "data": "synthetic",
        "config": {"workload": f"drop splash {args.n}^3, Fourier-perturbed film, density ratio 1000, "
                               f"divergence rhs seed 2, V(2,2), coarsest {args.n_coarsest}^3, tol {args.tol:g}",
                   "cells": N, "parallelism": "single GPU"},
        "setup_ms": setup32,
        "wall_ms_per_step": wall32,
        "fp32_refined_outer": last32["outer"],
        "fp32_refined_cycles": cyc32,
        "final_rel_residual": last32["rel_residual"],
        "gamma": last32["gamma"],
        "gbps_per_vcycle": bytes32 / cyc32 / 1e6 / (ms32 / cyc32),
        "cell_updates_per_s": N * cyc32 / (ms32 * 1e-3),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic_for(dom, args.n),
                     "avg_launch_ms": dom_avg_ms, "bytes_per_launch": dom_bytes},
        "kernel_ms_fp32_refined": prof32["kernel_ms"],
    }
    if tight:
        tight["tol"] = args.tight_tol
        out["at_tight_tol"] = tight
    out.update(res)
    if not args.no_cpu_baseline:
        # the oracle on the host: the baseline (the same FP32-refined solve, measured to
        # convergence) and p* (FP64 to 1e-13); every GPU result's error against them
        import numpy as np

        def rel(a, b):
            return float(np.linalg.norm(a - b) / np.linalg.norm(b))

        try:
            out["cpu_baseline"], r32 = cpu_baseline(P, args.n_coarsest, "fp32_refined", args.tol)
            log(f"cpu baseline: {out['cpu_baseline']['value']:.0f} ms on {out['cpu_baseline']['cores']} threads")
            rstar, star_s = oracle_reference(P, args.n_coarsest)
            log(f"oracle p*: {rstar['cycles']} cycles to {rstar['history'][-1]:.2e} in {star_s:.1f} s")
            err = {"p_star_rel_residual": float(rstar["history"][-1]), "p_star_cycles": rstar["cycles"],
                   "fp32_refined_vs_oracle_fp32_refined": rel(host32, r32["p"]),
                   "fp32_refined_vs_p_star": rel(host32, rstar["p"])}
            if host64 is not None:
                err["fp64_vs_p_star"] = rel(host64, rstar["p"])
            for key, hp in tight_host.items():
                err[key + "_vs_p_star"] = rel(hp, rstar["p"])
            out["oracle_error"] = err
        except Exception as e:  # the baseline is a report, never the product path
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
