"""Benchmark of the two-site DMRG H_eff . psi hot path on one MI355X.

Workload: N = 40 orbitals, 40 electrons, S_z = 0, bond dimension D = 4096,
middle bond (sites 20, 21 one-based), seeded synthetic Hamiltonian and
random isometries (see synth.py).  Setup (renormalized operators, task
table) is untimed.  One step = one Davidson step (one H_eff . psi product
plus the FP64 subspace update) for each product precision; K timed steps
follow W warm-up steps.  value = algorithmic TFLOP/s of the product inside
the FP64 Davidson steps; the FP32 and bf16-split results are reported
alongside.  A convergence leg (--converge, on by default) then runs
Davidson at the same size from the same start vector in every precision:
FP64 to the tolerance, the reduced precisions to the tolerance or their
noise floor, each reduced-precision Ritz vector scored by one FP64 product
(the energy error against FP64 that the mixed-precision bar is about) and
refined by FP64 steps to the FP64 tolerance.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}
KERNEL_SRC = [os.path.join(ROOT, "paper_2501_18263_amd", "csrc", f) for f in ("heff_kernels.hip", "heff_host.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_chain_dma_f64_n40_d4096.json")


def kernel_source_hash():
    """sha256 over the kernel source and the host code that orders its work."""
    import hashlib
    h = hashlib.sha256()
    for p in KERNEL_SRC:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_name(head, v, vst):
    """Product kernel that runs variant v in precision `head` under the
    library's automatic choice: FP64 takes the LDS-ring kernel for the 128-
    and 256-wide variants, and for the narrower ones when a wider variant
    has work; FP32 the register-staged kernel; the bf16 split its own."""
    nt = [2, 4, 8, 16][v]
    if head == "fp64":
        ring = v >= 2 or vst[2][0] > 0 or vst[3][0] > 0
        return "%s<double, %d>" % ("chain_dma" if ring else "chain_mfma", nt)
    if head == "bf16x3":
        return "chain_b3<%d>" % nt
    return "chain_mfma<float, %d>" % nt


def measured_traffic(variant):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, scaled by the copy-kernel
    calibration; None when the summary is missing, covers another variant
    or was taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash() or t.get("variant") != variant:
        return None
    return t.get("hbm_bytes_per_launch")


def _counter_rows(folder, counter, name_part):
    """Counter values per dispatch of kernels whose name contains name_part,
    from the rocprofv3 --output-format csv counter files under folder."""
    import csv
    import glob
    vals = []
    for path in sorted(glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)):
        with open(path) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") == counter and name_part in row.get("Kernel_Name", ""):
                    vals.append((int(row.get("Dispatch_Id", 0)), float(row["Counter_Value"]),
                                 int(row.get("Grid_Size", 0))))
    vals.sort()
    return vals


def write_traffic_record(args):
    """Write profiles/<name>.json and .md from four rocprofv3 counter runs
    (FETCH_SIZE and WRITE_SIZE of the product, FETCH_SIZE and WRITE_SIZE of
    the 1 GiB copy calibration) found under args.traffic_record, stamped with
    the hash of the current kernel sources: the record is written only from
    a measurement, never edited by hand."""
    import numpy as np
    d = args.traffic_record
    kern = args.traffic_kernel
    # the product launches: the dispatches with the grid of the run's last
    # one whose fetch is at least half the largest (the block build launches
    # the same kernel first, on small blocks, some with the same grid)
    fr = _counter_rows(os.path.join(d, "fetch"), "FETCH_SIZE", kern)
    wr = _counter_rows(os.path.join(d, "write"), "WRITE_SIZE", kern)
    if not (fr and wr):
        raise SystemExit("missing counter rows for %s" % kern)
    g_last = fr[-1][2]
    fmax = max(v for _, v, g in fr if g == g_last)
    prod_ids = [i for i, v, g in fr if g == g_last and v >= 0.5 * fmax]
    fetch = [v for i, v, g in fr if i in prod_ids]
    # WRITE_SIZE comes from a second run with the same dispatch sequence
    wids = [i for i, _, g in wr if g == g_last]
    write = [v for i, v, g in wr if g == g_last and i in wids[-len(prod_ids):]]
    grid = [g_last]
    cf = [v for _, v, _ in _counter_rows(os.path.join(d, "cfetch"), "FETCH_SIZE", "copyBuffer")]
    cw = [v for _, v, _ in _counter_rows(os.path.join(d, "cwrite"), "WRITE_SIZE", "copyBuffer")]
    if not (fetch and write and cf and cw):
        raise SystemExit("missing counter rows: fetch %d write %d copy %d/%d" % (len(fetch), len(write), len(cf), len(cw)))
    cfk, cwk = float(np.median(cf)), float(np.median(cw))
    fs, ws = 1048576.0 / cfk, 1048576.0 / cwk
    fk, wk = float(np.mean(fetch)), float(np.mean(write))
    hbm = 1024.0 * (fk * fs + wk * ws)
    rec = {"kernel": "%s (variant %d), product launch, grid %d threads" % (kern, args.traffic_variant, grid[0]),
           "variant": args.traffic_variant, "workload": args.traffic_workload,
           "kernel_source_sha256": kernel_source_hash(),
           "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk,
           "copy_fetch_kib_per_GiB": cfk, "copy_write_kib_per_GiB": cwk,
           "fetch_scale": fs, "write_scale": ws, "hbm_bytes_per_launch": hbm,
           "dispatches": {"fetch": fetch, "write": write},
           "commands": args.traffic_commands.split(";;") if args.traffic_commands else [],
           "kernel_source_files": [os.path.relpath(x, ROOT) for x in KERNEL_SRC]}
    base = os.path.join(ROOT, "profiles", args.traffic_name)
    with open(base + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    lines = ["# HBM traffic of %s, %s" % (kern, args.traffic_workload), "",
             "Written by `bench.py --traffic-record` from the counter runs below; sha256 of",
             "the kernel sources `%s`." % rec["kernel_source_sha256"], "", "Commands:", ""]
    lines += ["    " + c for c in rec["commands"]]
    lines += ["", "| quantity | value |", "|---|---|",
              "| FETCH_SIZE per launch (KiB) | %.4e (dispatches: %s) |" % (fk, ", ".join("%.4e" % v for v in fetch)),
              "| WRITE_SIZE per launch (KiB) | %.4e (dispatches: %s) |" % (wk, ", ".join("%.4e" % v for v in write)),
              "| FETCH_SIZE of a 1 GiB device copy (KiB) | %.6g -> scale %.4f |" % (cfk, fs),
              "| WRITE_SIZE of a 1 GiB device copy (KiB) | %.6g -> scale %.4f |" % (cwk, ws),
              "| HBM bytes per launch (scaled) | %.4e |" % hbm, ""]
    with open(base + ".md", "w") as f:
        f.write("\n".join(lines))
    print(json.dumps({"written": base + ".json", "hbm_bytes_per_launch": hbm}))


def copy_calibration(gib=1.0, reps=5):
    """Plain device-to-device copies of a known size (the calibration run of
    the HBM byte counters)."""
    import torch
    n = int(gib * (1 << 30)) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "reps": reps,
                      "GB_per_s": 8 * n / dt / 1e9}), flush=True)


CB_CONFIG = (24, 1024, 2)  # N, D, seed of the CPU baseline sample (the N=24, D=1024 configuration)


def _apply_chunk(i):
    """One worker's share of the oracle product: every W-th term, starting
    at term i (the terms and psi come from the forked parent)."""
    from oracle import block
    g = _CB_STATE
    t0 = time.perf_counter()
    block.FLOPS[0] = 0.0
    y = block.apply(g["p"], g["terms"][i::g["w"]], g["psi"])
    return y, time.perf_counter() - t0, block.FLOPS[0]


_CB_STATE = {}


def cpu_baseline_worker(args):
    """CPU-only process of the baseline (never touches the GPU): build the
    oracle's operators and term list for the sample, report readiness, wait
    for the parent's go (so the timed product does not share the host with
    the GPU measurements), then time one oracle product spread over a pool
    of single-threaded worker processes (terms dealt round-robin, partial
    outputs summed)."""
    import multiprocessing as mp

    import numpy as np

    from oracle import block
    from paper_2501_18263_amd import synth

    n, d, seed = CB_CONFIG
    t0 = time.perf_counter()
    p = synth.make_problem(n, d, seed)
    terms = block.heff_terms(p)
    psi = synth.random_psi(p)
    t_build = time.perf_counter() - t0
    w = args.cb_workers
    _CB_STATE.update(p=p, terms=terms, psi=psi, w=w)
    pool = mp.get_context("fork").Pool(w)
    pool.map(abs, range(w))  # workers up before the timed product
    print("ready", flush=True)
    sys.stdin.readline()
    t0 = time.perf_counter()
    parts = pool.map(_apply_chunk, range(w))
    y = np.sum([q[0] for q in parts], axis=0)
    dt = time.perf_counter() - t0
    pool.close()
    pool.join()
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    try:
        blas = np.show_config(mode="dicts")["Build Dependencies"]["blas"]
        blas = "%s %s" % (blas.get("name", "?"), blas.get("version", ""))
    except Exception:
        blas = "unknown"
    print(json.dumps({"seconds": dt, "workers": w, "build_s": t_build, "psi_dim": int(psi.size),
                      "terms": len(terms), "oracle_flops": float(sum(q[2] for q in parts)),
                      "worker_seconds": [q[1] for q in parts], "checksum": float(y @ psi),
                      "cpu_model": model, "blas": blas,
                      "host_cpus": len(os.sched_getaffinity(0))}), flush=True)


def cpu_baseline_start():
    """Start the baseline's CPU process before anything touches the GPU;
    its build overlaps the GPU measurements."""
    import subprocess
    w = max(1, min(16, len(os.sched_getaffinity(0))))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-baseline-worker",
                             "--cb-workers", str(w)], stdin=subprocess.PIPE, stdout=subprocess.PIPE,
                            text=True, env=env)


def cpu_baseline_finish(proc, flops_alg):
    """Let the baseline process time its product (after the GPU work) and
    turn it into the oracle's rate in algorithmic flops of the sample."""
    line = proc.stdout.readline().strip()
    if line != "ready":
        proc.kill()
        raise RuntimeError("CPU baseline process failed: %r" % line)
    proc.stdin.write("go\n")
    proc.stdin.flush()
    r = json.loads(proc.stdout.readline())
    proc.wait(timeout=60)
    n, d, seed = CB_CONFIG
    single = flops_alg / sum(r["worker_seconds"])
    return {"value": flops_alg / r["seconds"] / 1e12, "unit": "TFLOP/s", "cores": r["workers"], "kind": "oracle",
            "sample": "one O-BLOCK product (FP64 NumPy) at N=%d D=%d seed %d (%d-dim psi, %d terms), terms dealt "
                      "over %d single-threaded worker processes, %.1f s; rate = the library's algorithmic flops "
                      "of that product (%.3e) / wall time" % (n, d, seed, r["psi_dim"], r["terms"], r["workers"],
                                                              r["seconds"], flops_alg),
            "single_thread_tflops": single / 1e12, "cpu_model": r["cpu_model"], "blas": r["blas"],
            "host_cpus": r["host_cpus"], "oracle_build_s": r["build_s"], "oracle_executed_flops": r["oracle_flops"]}


def autotune_batch(bt, trials=3):
    """Project autotuner of the batched launch: time a few persistent grid
    sizes per kernel variant (work-groups = multiples of the 256 CUs) and keep
    the fastest; returns (grid, {grid: ms})."""
    import torch
    st = bt.stats()
    cands = [256, 512, 1024, 2048]
    table = {}
    best = None
    for gsz in cands:
        grid = [max(1, min(gsz, w)) for w in st["work_items"]]
        bt.set_grid(grid)
        bt.apply(use_graph=True)
        torch.cuda.synchronize()
        ts = []
        for _ in range(trials):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            bt.apply(use_graph=True)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = sorted(ts)[len(ts) // 2]
        table[gsz] = ms
        if best is None or ms < best[1]:
            best = (grid, ms)
    bt.set_grid(best[0])
    return best[0], table


def bench_batched(args):
    """Batched workload: 64 uneven two-site problems in one persistent,
    graph-captured FP32 launch per kernel variant vs 64 single launches."""
    import torch

    from paper_2501_18263_amd import heff, synth

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    specs = synth.batch_specs(args.batch)
    ctx = heff.Context(0)
    t0 = time.perf_counter()
    probs = [synth.make_problem(n, d, sd) for n, d, sd in specs]
    blocks = [heff.Blocks(ctx, p, precs=(heff.FP64, heff.FP32)) for p in probs]
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    bt = heff.Batch(ctx, blocks)
    for i, p in enumerate(probs):
        bt.views(i)[0].copy_(torch.tensor(synth.random_psi(p), dtype=torch.float32, device="cuda"))
    grid, table = autotune_batch(bt)
    F = bt.stats()["flops"]
    log("batch: %d problems, build %.1fs, F_alg %.3e, grid %s, tune %s" % (len(specs), t_build, F, grid, table))
    for _ in range(args.warmup):
        bt.apply(use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bt.apply(use_graph=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # the same products as 64 single-problem launches
    outs = [torch.empty_like(bt.views(i)[0]) for i in range(len(blocks))]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for i, B in enumerate(blocks):
            B.apply(bt.views(i)[0], outs[i], heff.FP32)
    torch.cuda.synchronize()
    dt_seq = (time.perf_counter() - t0) / args.steps
    out = {
        "metric": "batched H_eff·ψ TFLOP/s (64 uneven problems, FP32)", "value": F / dt / 1e12,
        "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "64 two-site problems, N~U{12..28}, D~U{128,256,512,1024}, FP32",
                   "flops_per_step": F, "build_s": t_build, "grid": grid, "autotune_ms": table},
        "roofline": {"bound": "mfma", "achieved": F / dt / 1e12, "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                     "frac": F / dt / 1e12 / PEAK_TFLOPS["fp32"], "traffic": None},
        "sequential_ms": dt_seq * 1e3, "speedup_vs_sequential": dt_seq / dt,
    }
    print(json.dumps(out), flush=True)


def _run_davidson(B, x0, prec, tol, max_steps, stall, log, tag):
    """Davidson from x0 with products in `prec` until ||r|| <= tol |theta|,
    `max_steps`, or (stall > 0) the reduced-precision noise floor: once
    ||r|| <= 1e-4 |theta|, `stall` steps in a row without a new smallest
    residual below 0.8 of the best.
    Returns the run's record and its Ritz vector (FP64, device)."""
    import torch

    from paper_2501_18263_amd import heff
    dav = heff.Davidson(B, x0, m_max=24, tol=tol)
    hist = []
    best, since = float("inf"), 0
    stop = "max_steps"
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max_steps):
        th, rn = dav.step(prec)
        hist.append((time.perf_counter() - t0, th, rn))
        if len(hist) % 25 == 0:
            log("%s: step %d, theta %.10f, resid %.2e" % (tag, len(hist), th, rn))
        if dav.converged:
            stop = "tolerance"
            break
        if rn < 0.8 * best:
            best, since = rn, 0
        elif rn <= 1e-4 * abs(th):
            since += 1
            if stall and since >= stall:
                stop = "stalled"
                break
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    u = torch.empty_like(x0)
    dav.ritz(u)
    dav.close()
    th, rn = hist[-1][1], hist[-1][2]
    log("%s: %d steps, %.1f s, theta %.12f, resid %.2e (%s)" % (tag, len(hist), secs, th, rn, stop))
    return {"steps": len(hist), "seconds": secs, "theta": th, "resid": rn, "stop": stop}, hist, u


def _fp64_score(B, u):
    """FP64 Rayleigh quotient of u and the FP64 residual norm ||Hu - E u|| / ||u||."""
    import torch

    from paper_2501_18263_amd import heff
    hu = torch.empty_like(u)
    B.apply(u, hu, heff.FP64)
    uu = float(u @ u)
    e = float(u @ hu) / uu
    r = float(torch.linalg.vector_norm(hu - e * u)) / uu ** 0.5
    return e, r


def convergence_leg(B, x0, precs, args, log):
    """The mixed-precision accuracy bar at the benchmark's own size: FP64
    Davidson to ||r|| <= conv_tol |theta|; FP32 and bf16-split Davidson from
    the same start vector until the same tolerance or their noise floor;
    every mixed-precision Ritz vector scored with one FP64 product (the
    Rayleigh quotient is second order in the vector's error), then refined
    by FP64 Davidson steps from that vector to the FP64 tolerance.  Reports
    raw and FP64-corrected energy differences to the FP64 result, the FP64
    residual of each mixed-precision vector, and times: to each run's stop,
    to within 1e-6 Ha of the converged FP64 energy (FP64 run: first step
    whose Ritz value is within 1e-6 Ha of the final one; Ritz values fall
    monotonically), and mixed + FP64 refinement to the FP64 tolerance."""
    from paper_2501_18263_amd import heff
    names = {"fp64": heff.FP64, "fp32": heff.FP32, "bf16x3": heff.BF16X3}
    out = {"tol": args.conv_tol, "max_steps": args.converge, "stall_steps": args.conv_stall,
           "start": "the benchmark's random start vector (seed + 200)"}
    r64, h64, u64 = _run_davidson(B, x0, heff.FP64, args.conv_tol, args.converge, 0, log, "fp64 converge")
    e64, res64 = _fp64_score(B, u64)
    r64["energy_fp64_rayleigh"] = e64
    r64["resid_fp64"] = res64
    r64["converged"] = r64["stop"] == "tolerance"
    # FP64 time to come within 1e-6 Ha of its final energy
    t_1e6 = next((t for t, th, _ in h64 if th - e64 <= 1e-6), h64[-1][0])
    r64["seconds_to_1e-6"] = t_1e6
    r64["resid_history"] = [h[2] for h in h64[::5]]
    out["fp64"] = r64
    for name in precs:
        if name == "fp64":
            continue
        r, h, u = _run_davidson(B, x0, names[name], args.conv_tol, args.converge, args.conv_stall, log,
                                "%s converge" % name)
        e, res = _fp64_score(B, u)
        r["energy_fp64_rayleigh"] = e
        r["resid_fp64"] = res
        r["dE_raw"] = r["theta"] - e64
        r["dE_fp64_corrected"] = e - e64
        r["within_1e-6"] = abs(e - e64) <= 1e-6
        r["speedup_to_1e-6"] = t_1e6 / r["seconds"]
        r["resid_history"] = [x[2] for x in h[::5]]
        rr, _, ur = _run_davidson(B, u, heff.FP64, args.conv_tol, args.refine_steps, 0, log,
                                  "%s -> fp64 refine" % name)
        er, _ = _fp64_score(B, ur)
        r["refine_fp64"] = {"steps": rr["steps"], "seconds": rr["seconds"], "stop": rr["stop"],
                            "resid": rr["resid"], "dE": er - e64}
        r["speedup_at_fp64_tol"] = r64["seconds"] / (r["seconds"] + rr["seconds"])
        log("%s: dE raw %.3e  FP64-corrected %.3e  FP64 resid %.2e  refine %d steps" % (
            name, r["dE_raw"], r["dE_fp64_corrected"], res, rr["steps"]))
        out[name] = r
    return out


def bench_backward(args):
    """Differentiation workload (N=16, D=256): time of the reverse-mode
    backward of E = <psi|H_eff|psi> (dE/dpsi and both operand-arena
    gradients) in FP64 and FP32, and of the orbital-rotation gradient for all
    N(N-1)/2 orbital pairs (one block build and one product per pair)."""
    import numpy as np
    import torch

    from paper_2501_18263_amd import heff, synth
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    p = synth.make_problem(16, 256, 5)
    ctx = heff.Context(0)
    B = heff.Blocks(ctx, p, precs=(heff.FP64, heff.FP32))
    x = torch.tensor(synth.random_psi(p), device="cuda")
    out = {}
    for name, pr, xx in (("fp64", heff.FP64, x), ("fp32", heff.FP32, x.float())):
        B.energy_backward(xx, prec=pr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            B.energy_backward(xx, prec=pr)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        out[name] = {"backward_ms": 1e3 * dt}
        log("%s backward: %.3f ms" % (name, 1e3 * dt))
    d64 = B.energy_backward(x)
    d32 = B.energy_backward(x.float(), prec=heff.FP32)
    rel = [float(torch.linalg.vector_norm(a.double() - b.double()) / torch.linalg.vector_norm(a.double()))
           for a, b in zip(d64, d32)]
    out["fp32_vs_fp64_rel"] = {"dpsi": rel[0], "dL": rel[1], "dR": rel[2]}
    pairs = [(a, b) for a in range(16) for b in range(a + 1, 16)]
    t0 = time.perf_counter()
    g = heff.kappa_gradient(ctx, p, x, pairs)
    out["kappa_gradient"] = {"pairs": len(pairs), "seconds": time.perf_counter() - t0,
                             "norm": float(np.linalg.norm(g))}
    log("kappa gradient: %d pairs in %.2f s" % (len(pairs), out["kappa_gradient"]["seconds"]))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.apply(x, torch.empty_like(x))
    torch.cuda.synchronize()
    out["product_ms"] = 1e3 * (time.perf_counter() - t0) / args.steps
    for name in ("fp64", "fp32"):
        out[name]["products_equivalent"] = out[name]["backward_ms"] / out["product_ms"]
    res = {"metric": "backward of <psi|H_eff|psi> (N=16, D=256)", "value": out["fp64"]["backward_ms"],
           "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": out["fp64"]["backward_ms"],
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", "config": {"workload": "two-site energy backward, N=16 D=256 seed 5",
                                           "psi_dim": int(B.n_elem)},
           "details": out}
    print(json.dumps(res), flush=True)



def bench_shards(args):
    """One GPU's share of an output-block-sharded FP64 product (the design
    for several GPUs, of which one GPU can show each rank's kernel time):
    for every rank of --shards P, the product restricted to that rank's
    output blocks, timed around a device-wide synchronization; the slowest
    rank bounds the
    product on P GPUs (before the all-gather of psi')."""
    import torch

    from paper_2501_18263_amd import heff, synth
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    p = synth.make_problem(args.n_orb, args.d, args.seed, beta=args.beta)
    ctx = heff.Context(0)
    B = heff.Blocks(ctx, p)
    x = torch.tensor(synth.random_psi(p), device="cuda")
    y = torch.empty_like(x)
    F = B.stats()["flops"]

    def timed():
        B.apply(x, y)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):   # device-wide sync: the product runs on the library's streams
            t0 = time.perf_counter()
            B.apply(x, y)
            torch.cuda.synchronize()
            ts.append(1e3 * (time.perf_counter() - t0))
        return sorted(ts)[len(ts) // 2]
    full_ms = timed()
    ranks = []
    for r in range(args.shards):
        fl = B.shard(r, args.shards)
        ms = timed()
        ranks.append({"rank": r, "flops": fl, "ms": ms, "tflops": fl / ms / 1e9})
        log("rank %d/%d: %.3f ms  %.2f TFLOP/s" % (r, args.shards, ms, fl / ms / 1e9))
    B.shard(0, 1)
    worst = max(q["ms"] for q in ranks)
    out = {"metric": "FP64 product, slowest rank of %d output-block shards, N=%d D=%d" % (args.shards, args.n_orb, args.d),
           "value": worst, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": worst,
           "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "one GPU per rank of a %d-way output-block shard, N=%d D=%d beta=%g" % (
               args.shards, args.n_orb, args.d, args.beta), "flops_per_product": F},
           "full_product_ms": full_ms, "speedup_bound": full_ms / worst,
           "flop_imbalance": max(q["flops"] for q in ranks) / (F / args.shards), "ranks": ranks}
    print(json.dumps(out), flush=True)

def bench_sweep(args):
    """The phases around Diag_H at the benchmark's size (Sec. IV.A names
    SVD, Ren_l and StVec): one left-to-right sweep step (truncation to D,
    the left block grown by site k with the truncated isometry, the task
    table of the next pair, its start vector) and the mode-optimization
    micro-iteration of the pair (angle search over S_1/2, one SVD per
    trial), each timed around a device-wide synchronization; the SVD alone
    is timed separately.  The two-site vector is the benchmark's random
    start vector (the timings do not depend on its values)."""
    import torch

    from paper_2501_18263_amd import heff, synth
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    p = synth.make_problem(args.n_orb, args.d, args.seed, beta=args.beta)
    ctx = heff.Context(0)
    t0 = time.perf_counter()
    B = heff.Blocks(ctx, p, keep_env=True)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    x = torch.tensor(synth.random_psi(p), device="cuda")
    y = torch.empty_like(x)
    B.apply(x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.apply(x, y)
    torch.cuda.synchronize()
    t_prod = time.perf_counter() - t0
    out = {}
    svd_s = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr = B.truncate(x, args.d)
        svd_s.append(time.perf_counter() - t0)
    out["svd_s"] = sorted(svd_s)[len(svd_s) // 2]
    log("SVD (truncation to %d): %.3f s" % (args.d, out["svd_s"]))
    step_s = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B2, start, info = B.sweep_right(x, args.d)
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - t0)
        n2, st2 = B2.n_elem, B2.stats()
        B2.close()
    out["sweep_step_s"] = sorted(step_s)[len(step_s) // 2]
    out["ren_l_tables_stvec_s"] = out["sweep_step_s"] - out["svd_s"]
    out["next_pair"] = {"psi_dim": n2, "tasks": st2["n_tasks"], "flops_per_product": st2["flops"],
                        "discarded_weight": info["discarded"]}
    log("sweep step: %.3f s (SVD %.3f, Ren_l + tables + StVec %.3f)" % (
        out["sweep_step_s"], out["svd_s"], out["ren_l_tables_stvec_s"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th, xr, sb, sa, ne = B.optimize_pair(x)
    torch.cuda.synchronize()
    out["mode_micro_iteration"] = {"seconds": time.perf_counter() - t0, "trials": ne, "theta": th,
                                   "S_half_before": sb, "S_half_after": sa}
    log("mode micro-iteration: %.3f s, %d trials, S_1/2 %.6f -> %.6f" % (out["mode_micro_iteration"]["seconds"], ne, sb, sa))
    res = {"metric": "sweep step and mode micro-iteration around Diag_H, N=%d D=%d" % (args.n_orb, args.d),
           "value": out["sweep_step_s"], "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
           "ms_per_step": 1e3 * out["sweep_step_s"], "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "one sweep step and one mode micro-iteration, N=%d D=%d beta=%g" % (
               args.n_orb, args.d, args.beta), "build_s": t_build, "product_s": t_prod},
           "details": out}
    print(json.dumps(res), flush=True)


def bench_su2(args):
    """SU(2) spin-adapted product (Sec. II.C, Eq. Hamilton_act_su2) on the
    benchmark multiplet problem (75 sectors and 2692 multiplets per block,
    10645 states with the magnetic quantum number resolved; 1500 terms; 26
    electrons in a singlet): build time, then per precision the median of
    `steps` HIP-event-timed products after `warmup` untimed ones, with the
    algorithmic flops of the task table."""
    import torch

    from paper_2501_18263_amd import heff, synth_su2
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    p = synth_su2.bench_problem(3)
    ctx = heff.Context(0)
    precs = [heff.FP64, heff.FP32, heff.BF16X3]
    t0 = time.perf_counter()
    H = heff.Su2(ctx, p, precs=precs)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    st = H.stats()
    log("SU(2) build %.2f s: %d blocks, %d reduced amplitudes (%.3e resolved), %d tasks, %.3e flops" % (
        t_build, len(H.blocks), H.n_elem, st["n_resolved"], st["n_tasks"], st["flops"]))
    x64 = torch.tensor(synth_su2.random_psi(p, seed=5), device="cuda")
    by = {}
    for prec in precs:
        x = x64 if prec == heff.FP64 else x64.float()
        y = torch.empty_like(x)
        for _ in range(args.warmup):
            H.apply(x, y, prec)
        torch.cuda.synchronize()
        ctx.timing(True)
        times = []
        for _ in range(args.steps):
            H.apply(x, y, prec)
            ms, n = ctx.timing_read()
            times.append(max(ms))
        ctx.timing(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            H.apply(x, y, prec)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        t = sorted(times)[len(times) // 2] / 1e3
        by[heff.PREC_NAMES[prec]] = {"product_s": wall, "longest_variant_launch_s": t,
                                     "tflops": st["flops"] / wall / 1e12}
        log("%s: %.2f ms per product (wall), %.2f TFLOP/s" % (heff.PREC_NAMES[prec], 1e3 * wall,
                                                                 st["flops"] / wall / 1e12))
    v = by["fp64"]["tflops"]
    res = {"metric": "SU(2) spin-adapted H_eff.psi TFLOP/s, D_SU(2)=2692 multiplets per block",
           "value": v, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * by["fp64"]["product_s"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "SU(2) two-site product: 75 sectors, 2692 multiplets (10645 states) per block, "
                                  "1500 terms, 26 electrons, singlet",
                      "build_s": t_build, "tasks": st["n_tasks"], "flops_per_product": st["flops"],
                      "reduced_amplitudes": H.n_elem, "resolved_amplitudes": st["n_resolved"]},
           "roofline_fp64": {"bound": "mfma", "achieved": v, "peak": 78.6, "unit": "TFLOP/s", "frac": v / 78.6},
           "by_precision": by}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-orb", type=int, default=40)
    ap.add_argument("--d", type=int, default=4096)
    ap.add_argument("--beta", type=float, default=0.5)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--precs", default="fp64,fp32,bf16x3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["single", "batched", "backward", "shards", "sweep", "su2"], default="single")
    ap.add_argument("--shards", type=int, default=8)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--converge", type=int, default=500,
                    help="steps cap of the convergence leg (each precision's Davidson from the start "
                         "vector, energy errors against FP64); 0 skips it")
    ap.add_argument("--conv-tol", type=float, default=1e-8, help="Davidson tolerance ||r|| <= tol |theta|")
    ap.add_argument("--refine-steps", type=int, default=80,
                    help="steps cap of the FP64 refinement from each reduced-precision Ritz vector")
    ap.add_argument("--conv-stall", type=int, default=12,
                    help="a reduced-precision run stops, once ||r|| <= 1e-4 |theta|, after this many "
                         "steps without a new smallest residual below 0.8 of the best")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain device copies of 1 GiB (HBM counter calibration)")
    ap.add_argument("--cpu-baseline-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cb-workers", type=int, default=1, help=argparse.SUPPRESS)
    ap.add_argument("--traffic-record", default=None,
                    help="folder with fetch/ write/ cfetch/ cwrite/ rocprofv3 counter runs: write the "
                         "profiles/ traffic record from them and exit (no GPU)")
    ap.add_argument("--traffic-kernel", default="chain_dma<double, 8>")
    ap.add_argument("--traffic-variant", type=int, default=2)
    ap.add_argument("--traffic-name", default="traffic_chain_dma_f64_n40_d4096")
    ap.add_argument("--traffic-workload", default="two-site H_eff.psi, N=40, D=4096, beta=0.5, seed 3, FP64")
    ap.add_argument("--traffic-commands", default="", help="';;'-separated commands of the counter runs")
    args = ap.parse_args()
    if args.cpu_baseline_worker:
        cpu_baseline_worker(args)
        return
    if args.traffic_record:
        write_traffic_record(args)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the two-site product runs on one GPU only (a multi-GPU split would shard "
              "the task table by output blocks); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched":
        # This workload (64 problems built and run in one process) ended in a
        # host segmentation fault after the kernels moved to two work-groups
        # per CU and tree-dispatched stage instances; its cause is not found,
        # so it stays switched off.  The batched parity test (a few problems,
        # graph replays) passes with these kernels.
        print("bench.py: the batched workload is switched off (a host segmentation fault with the "
              "current kernels is not yet explained)", file=sys.stderr)
        sys.exit(3)
    if args.workload == "backward":
        bench_backward(args)
        return
    if args.workload == "shards":
        bench_shards(args)
        return
    if args.workload == "sweep":
        bench_sweep(args)
        return
    if args.workload == "su2":
        bench_su2(args)
        return

    cb_proc = None if args.no_cpu_baseline else cpu_baseline_start()  # before the GPU is touched

    import numpy as np  # noqa: F401
    import torch

    from paper_2501_18263_amd import heff, synth

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    names = {"fp64": heff.FP64, "fp32": heff.FP32, "bf16x3": heff.BF16X3}
    precs = [x for x in args.precs.split(",") if x]
    t0 = time.perf_counter()
    p = synth.make_problem(args.n_orb, args.d, args.seed, beta=args.beta)
    psi0 = synth.random_psi(p)
    log("generated N=%d D=%d psi=%d in %.1fs" % (args.n_orb, args.d, synth.psi_size(p), time.perf_counter() - t0))
    ctx = heff.Context(0)
    t0 = time.perf_counter()
    B = heff.Blocks(ctx, p, precs=tuple(names[x] for x in precs))
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    st = B.stats()
    vst = B.variant_stats()
    ist = B.issued_stats()
    F = st["flops"]
    log("build %.1fs  tasks %d  F_alg %.3e  bytes %s" % (t_build, st["n_tasks"], F, st["bytes"]))
    for v in range(len(vst)):
        if vst[v][1]:
            log("variant %d: work-groups %d  F_alg %.3e  F_mfma %.3e (issue eff %.3f)  steps %d (longest group %d)" % (
                v, vst[v][1], vst[v][0], ist[v][0], vst[v][0] / max(ist[v][0], 1.0), ist[v][1], ist[v][2]))
    x0 = torch.tensor(psi0, device="cuda")

    res = {}
    e_fp64 = None
    for name in precs:
        pr = names[name]
        # product alone: events on the product's stream around each call
        dt_ = torch.float64 if pr == heff.FP64 else torch.float32
        xs = x0.to(dt_)
        ys = torch.empty_like(xs)
        B.apply(xs, ys, pr)
        torch.cuda.synchronize()
        ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        for i in range(args.steps):
            ev0[i].record()
            B.apply(xs, ys, pr)
            ev1[i].record()
        torch.cuda.synchronize()
        prod_ms = sorted(a.elapsed_time(b) for a, b in zip(ev0, ev1))
        prod_med = prod_ms[len(prod_ms) // 2]
        log("%s product: median %.3f ms  %.2f TFLOP/s" % (name, prod_med, F / prod_med / 1e9))
        dav = heff.Davidson(B, x0, m_max=24, tol=1e-10)
        for _ in range(args.warmup):
            dav.step(pr)
        torch.cuda.synchronize()
        ctx.timing(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            th, rn = dav.step(pr)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms, nl = ctx.timing_read()
        ctx.timing(False)
        # energy of the final Ritz vector with an FP64 product (Rayleigh quotient)
        u = torch.empty_like(x0)
        dav.ritz(u)
        hu = torch.empty_like(x0)
        B.apply(u, hu, heff.FP64)
        e_corr = float(u @ hu) / float(u @ u)
        r = {"ms_per_step": 1e3 * dt / args.steps, "tflops": F * args.steps / dt / 1e12,
             "product_ms_median": prod_med, "product_tflops": F / prod_med / 1e9,
             "theta": th, "resid": rn, "energy_fp64_rayleigh": e_corr,
             "kernel_ms": ms, "kernel_launches": nl}
        if name == "fp64":
            e_fp64 = th
        res[name] = r
        dav.close()
        log("%s: %.2f ms/step  %.2f TFLOP/s  theta %.10f  resid %.2e" % (name, r["ms_per_step"], r["tflops"], th, rn))
    # accuracy of the reduced-precision products at this size: relative
    # error of H psi against FP64 and the error of the energy functional
    # <psi|H|psi>/<psi|psi> they give, on the start vector
    if "fp64" in precs:
        y64 = torch.empty_like(x0)
        B.apply(x0, y64, heff.FP64)
        e64 = float(x0 @ y64) / float(x0 @ x0)
        for name in precs:
            if name == "fp64":
                continue
            pr = names[name]
            x32 = x0.float()
            y32 = torch.empty_like(x32)
            B.apply(x32, y32, pr)
            yd = y32.double()
            res[name]["product_rel_error"] = float(torch.linalg.vector_norm(yd - y64) / torch.linalg.vector_norm(y64))
            res[name]["energy_functional_error"] = float(x0 @ yd) / float(x0 @ x0) - e64
    if args.converge > 0 and "fp64" in precs:
        conv = convergence_leg(B, x0, precs, args, log)
        for name in precs:
            res[name]["convergence"] = conv[name]
            if name != "fp64":
                c = conv[name]
                res[name]["dE_raw"] = c["dE_raw"]
                res[name]["dE_fp64_corrected"] = c["dE_fp64_corrected"]
                res[name]["speedup_product_vs_fp64"] = res["fp64"]["product_ms_median"] / res[name]["product_ms_median"]
                res[name]["speedup_to_1e-6_vs_fp64"] = c["speedup_to_1e-6"]
                res[name]["speedup_at_fp64_tol_vs_fp64"] = c["speedup_at_fp64_tol"]
    head = "fp64" if "fp64" in res else precs[0]
    hr = res[head]
    # roofline of the dominant kernel (the variant with the largest time)
    ms, nl = hr["kernel_ms"], hr["kernel_launches"]
    v = max(range(len(ms)), key=lambda i: ms[i])
    avg_s = ms[v] / 1e3 / max(nl[v], 1)
    achieved = vst[v][0] / avg_s / 1e12
    roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[head], "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS[head],
            "traffic": measured_traffic(v) if head == "fp64" else None,
            "kernel": "%s variant %d (output width and task middle dimension <= %d)" % (
                kernel_name(head, v, vst), v, [32, 64, 128, 256][v]),
            "flops_per_launch": vst[v][0], "avg_launch_ms": avg_s * 1e3,
            "mfma_flops_per_launch": ist[v][0], "mfma_issue_efficiency": vst[v][0] / max(ist[v][0], 1.0),
            "pipeline_steps_per_launch": ist[v][1], "pipeline_steps_longest_group": ist[v][2]}
    out = {
        "metric": "H_eff·ψ TFLOP/s and Davidson step time, FP64 vs mixed, N=40 D=4096",
        "value": hr["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": hr["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3-f32acc"}[head], "data": "synthetic",
        "config": {"workload": "two-site DMRG H_eff·psi + Davidson, N=%d D=%d" % (args.n_orb, args.d),
                   "n_orb": args.n_orb, "electrons": p.n_up + p.n_dn, "bond_dim": args.d, "beta": args.beta,
                   "psi_dim": int(B.n_elem), "tasks": st["n_tasks"], "flops_per_product": F,
                   "build_s": t_build},
        "roofline": roof,
        "by_precision": res,
    }
    if cb_proc is not None:
        n, d, seed = CB_CONFIG
        Bc = heff.Blocks(ctx, synth.make_problem(n, d, seed))
        f_c = Bc.stats()["flops"]
        Bc.close()
        out["cpu_baseline"] = cpu_baseline_finish(cb_proc, f_c)
        log("cpu baseline: %s" % out["cpu_baseline"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
