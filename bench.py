#!/usr/bin/env python
"""Benchmark: FEAST iterations/s and time-to-1e-10 residual on one MI355X.

Workload (default, --workload c2): a batch of 64 independent pencils, n ~ U{256..2048} (seeded),
each with a prescribed spectrum (8-32 eigenvalues inside |z| < 0.8, the rest in 1.5 < |z| < 5),
B = I + 0.1 random Hermitian, the unit circle with q = 16 trapezoid nodes, m0 in {16, 32},
R-FEAST.  One step = the whole batch from resident inputs: one graph launch assembles and factors
every node of every pencil, then all pencils iterate in lockstep until every candidate has
relative residual <= 1e-10 (count repeated).  ms_per_step is the batch's time-to-1e-10; value is
whole-job FEAST iterations per second.  The headline mode is FP32 LU + FP64 correction (the
shifted-residual form of the filter); plain FP64 is timed beside it, and both also one pencil at a
time.  The single-pencil n = 4096 (R-FEAST) and n = 8192 (Bi-FEAST) workloads are reported as extra
keys.  The roofline object is the trailing-update kernel, timed per launch with HIP events in a run
of the same batch whose factorisation is launched directly (the same kernels) instead of as a
graph.

    python bench.py [--steps K] [--warmup W] [--mode fp32|fp64|fp16] [--workload c2|c1|c3|...] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FEAST iterations/s & time-to-1e-10 residual: mixed-prec batched vs FP64"
PEAK = {"fp64": 78.6, "fp32": 157.3, "fp16": 2500.0}   # dense MFMA TFLOP/s (MI355X published)
HBM_PEAK = 8000.0                              # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_workload(name):
    import pencils
    with open(os.path.join(ROOT, "tests", "golden", f"spectrum_{name}.json")) as f:
        g = json.load(f)
    builder = {"c1": pencils.c1, "c3": pencils.c3}[name]
    P = builder(radius=g["radius"])
    ref = np.array([complex(a, b) for a, b in g["nearest"]])[: g["m"]]
    cfg = int(name[1])
    U0 = pencils.start_block(cfg, P.n, P.m0)
    return P, U0, ref, g


# sources whose change voids a PMC traffic record, per record
TRAFFIC_SOURCES = {"panel_step_kernel": ["lu.hip"], "lu_update": ["gemm.hip", "lu.hip"]}


def sources_hash(names):
    import hashlib
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_1404_2891_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, mode):
    """HBM bytes per launch of `kernel` on `workload` from the committed PMC record
    (profiles/pmc_traffic.json, written by --pmc-summary), or None when there is no record for that
    workload and mode or the sources behind it have changed since."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "pmc_traffic.json")))[f"{kernel}@{workload}"]
        digest = sources_hash(TRAFFIC_SOURCES[kernel])
    except (OSError, KeyError, ValueError):
        return None
    if digest != rec.get("sources_sha256_16") or mode != rec.get("mode"):
        return None
    return rec.get("bytes_per_launch", rec["bytes_per_dispatch"])


def batch_update_bytes(ns, q, elem):
    """Algorithmic bytes and launch count of the trailing updates of a batch factored as one set:
    launch s covers step s of every member that has it."""
    total, launches = 0.0, 0
    for n in ns:
        b, l = update_bytes(n, q, elem)
        total += b
        launches = max(launches, l)
    return total, launches


def pmc_summary(fetch_csv, write_csv, workload, mode, note):
    """Per-dispatch HBM traffic of the trailing update from two rocprofv3 --pmc runs of
    `bench.py --workload W --counters` (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), each scaled
    by what the same counter reads for the elementwise multiply of 64 Mi floats the run starts with
    (256 MiB read, 256 MiB written); recorded in profiles/pmc_traffic.json with a hash of the
    sources."""
    import csv
    # the update's kernel instances (both tile shapes of the FP16 kernels)
    kname = {"fp32": "cgemm_f16_kernel<true", "fp16": "cgemm_f16_kernel<false"}.get(
        mode, "cgemm_kernel<double, 2, 2, 2, 2, true, true, true, 1>")
    out = {}
    for key, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = list(csv.DictReader(open(path)))
        cal = [float(r["Counter_Value"]) for r in rows if "MulFunctor" in r["Kernel_Name"]]
        upd = [float(r["Counter_Value"]) for r in rows if kname in r["Kernel_Name"]]
        if not cal or not upd:
            raise SystemExit(f"{path}: calibration or update dispatches missing")
        factor = 256.0 * 1024 / cal[0]          # KiB the counter should read for 256 MiB
        out[key] = (sum(upd) / len(upd), factor, len(upd))
    elem = 16 if mode == "fp64" else 8
    if workload == "c2":
        ns, _ = __import__("pencils").c2_sizes(64)
        alg, launches = batch_update_bytes(ns, 16, elem)
    else:
        n, q = {"c1": (4096, 24), "c3": (8192, 32)}[workload]
        alg, launches = update_bytes(n, q, elem)
    per = 1024.0 * (out["fetch"][0] * out["fetch"][1] + out["write"][0] * out["write"][1])
    # the counter run's dispatches each cover one part of the nodes (the parts factored side by
    # side); per launch of the whole-node factorisation = the run's total over its launch count
    total = per * out["fetch"][2]
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        rec = {}
    rec[f"lu_update@{workload}"] = dict(
        workload=note, kernel=kname, mode=mode, dispatches=out["fetch"][2],
        fetch_kib_per_dispatch=out["fetch"][0], write_kib_per_dispatch=out["write"][0],
        calibration="torch elementwise multiply of 64 Mi floats: 256 MiB read, 256 MiB written",
        fetch_factor=out["fetch"][1], write_factor=out["write"][1], bytes_per_dispatch=per,
        bytes_per_factorisation=total, launches=launches, bytes_per_launch=total / launches,
        algorithmic_bytes_per_launch=alg / launches, ratio=total / alg,
        sources_sha256_16=sources_hash(TRAFFIC_SOURCES["lu_update"]))
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec[f"lu_update@{workload}"], indent=1))


def update_bytes(n, q, elem, nb=64, group=4):
    """Algorithmic bytes of the trailing-update launches of one factorisation and their count.

    Step s (i = s mod group, w = min(nb, n - j0), nr = n - j0 - w) updates nr rows by nc columns with
    K = i nb + w (nc = min(nb, nr) inside a group, nr at its last step): it reads L21 (nr x K) and
    U12 (K x nc) and reads and writes the block (nr x nc), for every node."""
    total, launches = 0.0, 0
    for step, j0 in enumerate(range(0, n, nb)):
        i = step % group
        w = min(nb, n - j0)
        nr = n - j0 - w
        if nr <= 0:
            break
        K = i * nb + w
        nc = min(nb, nr) if i < group - 1 else nr
        total += elem * q * (nr * K + K * nc + 2.0 * nr * nc)
        launches += 1
    return total, launches


def panel_bytes(n, q, elem, nb=64, reg_rows=None):
    """Algorithmic bytes of the panel column steps of one factorisation and their launch count.

    Launch j (0..w) of the panel at j0 reads and writes the columns >= j - 1 of rows >= j0 + j - 1
    (the active part), for every node: 2 elem q (n - j0 - j') (w - j') bytes with j' = max(j - 1, 0).
    Panels of at most reg_rows rows run as one register-panel launch reading and writing the whole
    panel once."""
    if reg_rows is None:
        reg_rows = 64
    total, launches = 0.0, 0
    for j0 in range(0, n, nb):
        w = min(nb, n - j0)
        rows = n - j0
        if rows <= reg_rows:
            total += 2.0 * elem * q * rows * w
            launches += 1
            continue
        for j in range(w + 1):
            jp = max(j - 1, 0)
            total += 2.0 * elem * q * (rows - jp) * (w - jp)
            launches += 1
    return total, launches


def match_err(got, ref):
    from scipy.optimize import linear_sum_assignment
    if len(got) != len(ref):
        return float("inf")
    C = np.abs(got[:, None] - ref[None, :]) / np.abs(ref)[None, :]
    r, c = linear_sum_assignment(C)
    return float(C[r, c].max())


def run_steps(fm, torch, A, B, U0, P, mode, steps, warmup, ws, timing, variant="R", pivoting="tournament",
              conj_nodes="none"):
    kw = dict(center=P.center, radius=P.radius, aspect=1.0, q=P.q, m0=P.m0, precision=mode, workspace=ws,
              variant=variant, pivoting=pivoting, conj_nodes=conj_nodes)
    results = []
    for _ in range(warmup):
        with fm.Feast(A, B, timing=False, **kw) as F:
            F.iterate(U0)
    torch.cuda.synchronize()
    phases = None
    t0 = time.perf_counter()
    for _ in range(steps):
        F = fm.Feast(A, B, timing=False, **kw)
        results.append(F.iterate(U0))
        F.close()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the phase breakdown from as many runs again with the library's HIP events (outside the timed
    # region: with events the nodes are factored in one sequence, not in two halves side by side)
    for _ in range(steps if timing else 0):
        with fm.Feast(A, B, timing=True, **kw) as F:
            F.iterate(U0)
            ph = F.timing()
        if phases is None:
            phases = {k: dict(v) for k, v in ph.items()}
        else:
            for k, v in ph.items():
                for f in ("ms", "flops", "launches"):
                    phases[k][f] += v[f]
    torch.cuda.synchronize()
    return wall, results, phases


def cpu_baseline(P, U0, iters, sample_nodes=4, variant="R"):
    """The oracle (NumPy/SciPy, FP64) timed on the same workload: the whole R-FEAST run (q node
    factorisations, iterations to 1e-10) for pencils up to n = 4096 (about 13 s on 16 threads), else
    a bounded sample (a few of the q node factorisations and solves plus one Rayleigh-Ritz step,
    scaled to q nodes and the iteration count of the solve)."""
    import scipy.linalg
    from oracle import feast as ofeast
    from oracle import quadrature as oq
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("internal_api") == "openblas"] or [1])
    except Exception:
        cores = os.cpu_count()
    if variant == "R" and P.n <= 4096:
        t0 = time.perf_counter()
        r = ofeast.rfeast(P.A, P.B, P.center, P.radius, 1.0, P.q, U0)
        t = time.perf_counter() - t0
        return dict(value=r.iters / t, unit="FEAST iterations/s", cores=int(cores), kind="oracle",
                    time_to_1e10_s=t,
                    sample=f"the whole workload: one oracle R-FEAST run (n={P.n}, q={P.q}, m0={P.m0}: {P.q} node "
                           f"LUs, {r.iters} iterations to 1e-10, m = {r.m}, converged {bool(r.converged)})",
                    iterations=int(r.iters))
    z, s = oq.nodes_and_weights(P.center, P.radius, 1.0, "trapezoid", P.q)
    t0 = time.perf_counter()
    lus = [scipy.linalg.lu_factor(ofeast.node_matrix(P.A, P.B, zk)) for zk in z[:sample_nodes]]
    t_lu = (time.perf_counter() - t0) / sample_nodes
    t0 = time.perf_counter()
    BU = P.B @ U0
    t_bu = time.perf_counter() - t0
    t0 = time.perf_counter()
    Y = [scipy.linalg.lu_solve(lu, BU) for lu in lus]
    t_solve = (time.perf_counter() - t0) / sample_nodes
    Q = sum(sk * yk for sk, yk in zip(s[:sample_nodes], Y))
    t0 = time.perf_counter()
    Qo = ofeast.orthonormalize(Q)
    Ah = Qo.conj().T @ (P.A @ Qo)
    Bh = Qo.conj().T @ (P.B @ Qo)
    lam, W = scipy.linalg.eig(Ah, Bh)
    X = Qo @ W
    ofeast.residuals(P.A, P.B, lam, X)
    t_rr = time.perf_counter() - t0
    total = P.q * t_lu + iters * (t_bu + P.q * t_solve + t_rr)
    return dict(value=iters / total, unit="FEAST iterations/s", cores=int(cores), kind="oracle",
                time_to_1e10_s=total,
                sample=f"{sample_nodes} of {P.q} node LUs and solves, one B U and one Rayleigh-Ritz step "
                       f"(n={P.n}, m0={P.m0}), scaled to {P.q} nodes and {iters} iterations",
                measured_s=dict(lu_per_node=t_lu, solve_per_node=t_solve, bu=t_bu, rayleigh_ritz=t_rr))


def load_batch(count=64, device=None):
    """The batched workload: count pencils with n ~ U{256..2048}, prescribed spectra (m ~ U{8..32}
    inside |z| < 0.8), B = I + 0.1 (H + H^H)/(2 sqrt n), unit circle, q = 16, m0 in {16, 32}.
    The random draws are made on the host; with device set, the products that build A and B run
    there (A, B are then device tensors)."""
    import pencils
    ns, ms = pencils.c2_sizes(count)
    out = []
    for j in range(count):
        out.append(pencils.c2_pencil(j, ns[j], ms[j], device=device))
        if device is None and j % 8 == 7:
            log(f"  {j + 1} of {count} pencils built")
    return out


def tune_tiles(fm, q, modes, dev):
    """The trailing update's tile shape per row bucket, measured for the update kernel of each mode in
    use (FP32: the split FP16 kernel; FP64: the FP64 kernel) and set in the library before timing
    (outside the timed region)."""
    out = {}
    for mode in sorted({m for m in modes if m in ("fp32", "fp64")}):
        t = fm.binding.autotune_tiles(mode, q, device=dev)
        out[mode] = [dict(rows_up_to=r, shape=shape, tflops={k: round(v, 1) for k, v in tf.items()})
                     for r, shape, tf in t]
        log(f"tile tuning {mode}, q={q}: " + ", ".join(f"<={r}: {shape}" for r, shape, _ in t))
    return out


def tune_panels(fm, q, modes, dev):
    """Panel crossover for each storage precision in use (outside the timed region)."""
    out = {}
    for mode in sorted({("fp64" if m == "fp64" else "fp32") for m in modes}):
        rows, table = fm.autotune(mode, q, device=dev)
        out[mode] = dict(single_rows=rows, table=[[int(r), round(a, 4), round(b, 4)] for r, a, b in table])
        log(f"panel tuning {mode}, q={q}: sweeping panel up to {rows} rows")
    return out


def batch_cpu_baseline(P, U0h, stride=4):
    """The oracle (NumPy/SciPy FP64 R-FEAST: 16 LUs per pencil, then iterations to 1e-10) run in
    full on a stratified sample of the batch (every stride-th pencil in order of n), its time scaled
    by stride to the whole batch; iterations/s = the sample's iterations over its time."""
    from oracle import feast as ofeast
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("internal_api") == "openblas"] or [1])
    except Exception:
        cores = os.cpu_count()
    order = sorted(range(len(P)), key=lambda j: P[j].n)
    sample = order[stride // 2::stride]
    t0 = time.perf_counter()
    iters, ok = 0, 0
    for j in sample:
        p = P[j]
        A = p.A.cpu().numpy() if hasattr(p.A, "cpu") else p.A
        B = p.B.cpu().numpy() if hasattr(p.B, "cpu") else p.B
        r = ofeast.rfeast(A, B, p.center, p.radius, 1.0, p.q, U0h[j])
        iters += r.iters
        ok += int(r.converged and r.m == p.m)
    t = time.perf_counter() - t0
    return dict(value=iters / t, unit="FEAST iterations/s", cores=int(cores), kind="oracle",
                time_to_1e10_s=t * len(P) / len(sample),
                sample=f"{len(sample)} of {len(P)} pencils (every {stride}th in order of n, n = "
                       f"{min(P[j].n for j in sample)}..{max(P[j].n for j in sample)}), full oracle R-FEAST runs "
                       f"(16 LUs + iterations to 1e-10); time scaled by {stride} to the batch",
                sample_s=t, sample_iterations=iters, sample_converged=ok)


def update_kernel(mode):
    """The trailing-update kernel of a mode: the matrix-core precision whose published peak bounds it,
    its name, and the FP16 products per real product (the FP32 mode splits every operand into high
    and low FP16 parts and takes three products, so its attainable algorithmic rate is a third of
    the FP16 peak)."""
    if mode == "fp64":
        return "fp64", "cgemm_kernel<double> (trailing update, kind 1, FP64 matrix cores)", 1
    if mode == "fp16":
        return "fp16", "cgemm_f16_kernel<false> (trailing update, FP16 matrix cores)", 1
    return "fp16", "cgemm_f16_kernel<true> (trailing update, FP16 matrix cores, split operands)", 3


def update_roof_fields(achieved, mode):
    key, name, products = update_kernel(mode)
    d = dict(bound="mfma", achieved=achieved, peak=PEAK[key], unit="TFLOP/s", frac=achieved / PEAK[key],
             kernel=name)
    if products > 1:
        d["fp16_products_per_real_product"] = products
        d["frac_of_split_attainable"] = achieved * products / PEAK[key]
    return d


def update_roofline(ph, prec, ns, mode):
    """Per-launch figures of the trailing-update kernel of a batch from the library's HIP-event phase
    timing: flops per launch (8 nr nc K over every member and node the launch covers) / average
    duration; algorithmic bytes per launch (batch_update_bytes) and the measured traffic (PMC
    record)."""
    u = ph["lu_update"]
    launches = max(1, u["launches"])
    avg_ms = u["ms"] / launches
    achieved = u["flops"] / launches / (avg_ms * 1e-3) / 1e12
    alg, _ = batch_update_bytes(ns, 16, 16 if mode == "fp64" else 8)
    return dict(**update_roof_fields(achieved, mode),
                traffic=measured_traffic("lu_update", "c2", mode),
                traffic_unit="bytes per launch (PMC FETCH_SIZE + WRITE_SIZE, calibrated)",
                kernel_phase="lu_update",
                avg_launch_ms=avg_ms, launches=u["launches"], flops_per_launch=u["flops"] / launches,
                algorithmic_bytes_per_launch=alg / launches)


def bench_batch(args, fm, torch, dev):
    """The batched workload (default): 64 pencils, one graph launch factors every node of every pencil,
    then all pencils iterate in lockstep to 1e-10.  Mixed precision (FP32 LU + FP64 correction) is the
    headline, plain FP64 beside it, both also one pencil at a time."""
    from oracle import brute
    t0 = time.perf_counter()
    P = load_batch(args.count, dev)
    torch.cuda.synchronize()
    log(f"batch of {len(P)} pencils generated in {time.perf_counter() - t0:.1f} s; "
        f"n in [{min(p.n for p in P)}, {max(p.n for p in P)}], sum n^3 = {sum(p.n ** 3 for p in P):.3e}")
    mats = [(p.A, p.B) for p in P]
    U0h = [pencils_start(p, j) for j, p in enumerate(P)]
    U0s = [fm.to_device(u, dev) for u in U0h]
    refs = [brute.eigenvalues_inside(p.lam, 0j, 1.0) for p in P]
    m0s = [p.m0 for p in P]
    lu_flops = sum(16 * (8.0 / 3.0) * p.n ** 3 for p in P)
    torch.cuda.synchronize()

    def batched(mode, timing=False):
        t = time.perf_counter()
        b = fm.FeastBatch(mats, (0j, 1.0, 1.0), m0=m0s, q=16, precision=mode, pivoting=args.pivoting, timing=timing)
        t_setup = time.perf_counter() - t
        res, rcs = b.iterate(U0s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        fms = b.factor_ms()
        ph = b.timing() if timing else None
        b.close()
        return wall, t_setup, fms, res, ph

    def one_at_a_time(mode):
        t = time.perf_counter()
        res = []
        for (A, B), U0, m0 in zip(mats, U0s, m0s):
            with fm.Feast(A, B, 0j, 1.0, 1.0, 16, m0, precision=mode, pivoting=args.pivoting) as F:
                res.append(F.iterate(U0))
        torch.cuda.synchronize()
        return time.perf_counter() - t, res

    def errs(res):
        return max(match_err(r.lam, ref) for r, ref in zip(res, refs))

    modes = [args.mode] + ([] if args.no_compare else [m for m in ("fp64", "fp32") if m != args.mode])
    tuning = tune_panels(fm, 16, modes, dev) if args.tune else None
    tiles = tune_tiles(fm, 16, modes, dev)
    out = {}
    for mode in modes:
        for _ in range(args.warmup):
            batched(mode)
        steps = args.steps if mode == args.mode else max(1, min(args.steps, 2))
        runs = [batched(mode) for _ in range(steps)]
        k = int(np.argsort([r[0] for r in runs])[len(runs) // 2])   # the median run
        wall, t_setup, fms, res, _ = runs[k]
        iters = sum(r.iterations for r in res)
        seq_wall, seq_res = one_at_a_time(mode) if not args.no_sequential else (float("nan"), res)
        out[mode] = dict(ms_per_step=1e3 * wall, iters_per_s=iters / wall, total_iterations=iters,
                         setup_ms=1e3 * t_setup, factor_graph_ms=fms,
                         iters_per_s_after_setup=iters / (wall - t_setup),
                         iteration_ms=1e3 * (wall - t_setup),
                         converged=all(r.converged for r in res),
                         found_all=all(len(r.lam) == len(ref) for r, ref in zip(res, refs)),
                         eig_err_vs_oracle=errs(res), max_resid=float(max(r.resid.max() for r in res)),
                         one_at_a_time_ms=1e3 * seq_wall, one_at_a_time_err=errs(seq_res),
                         batched_speedup=seq_wall / wall, steps=steps)
        out[mode]["factor_tflops"] = lu_flops / (fms * 1e-3) / 1e12
        log(f"{mode}: batch {out[mode]['ms_per_step']:.1f} ms (setup {out[mode]['setup_ms']:.1f} ms, graph "
            f"{fms:.1f} ms = {out[mode]['factor_tflops']:.1f} TF/s; iterations {out[mode]['iteration_ms']:.1f} ms), "
            f"one at a time {out[mode]['one_at_a_time_ms']:.1f} ms, {iters} iterations, "
            f"err {out[mode]['eig_err_vs_oracle']:.1e}")
    head = out[args.mode]
    prec = args.mode
    # the dominant kernel: per-launch times from a run of the same batch with HIP events around every
    # factorisation launch (the sequence launched directly instead of as a graph: same kernels)
    _, _, t_fms, t_res, ph = batched(args.mode, timing=True)
    phases = {k: dict(ms=v["ms"], launches=v["launches"],
                      tflops=(v["flops"] / (v["ms"] * 1e-3) / 1e12) if v["ms"] > 0 and v["flops"] > 0 else None)
              for k, v in ph.items()}
    for k, v in phases.items():
        log(f"   {k:16s} {v['ms']:9.2f} ms  {v['launches']:6d} launches  {v['tflops']} TF/s")
    roofline = update_roofline(ph, "fp16" if prec == "fp16" else prec, [p.n for p in P], prec)
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample of the batch ...")
        cpu = batch_cpu_baseline(P, U0h)
        log(f"oracle: {cpu['value']:.2f} it/s, batch estimate {cpu['time_to_1e10_s']:.1f} s ({cpu['sample']})")
    extras = {}
    if not args.no_extras:
        for name in ("c1", "c3"):
            extras[name] = single_pencil_summary(args, fm, torch, dev, name)
    mode_names = {"fp32": "FP32 LU (trailing updates on FP16 matrix cores, split operands) + FP64 shifted-residual correction", "fp64": "FP64",
                  "fp16": "FP16-update LU + FP64 shifted-residual correction"}
    line = {
        "metric": METRIC,
        "value": head["iters_per_s"],
        "unit": "FEAST iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32+f64", "fp16": "f16+f32+f64", "fp64": "f64"}[args.mode],
        "data": "synthetic",
        "config": {"workload": f"{len(P)} pencils, n ~ U{{256..2048}}, prescribed spectra (8-32 eigenvalues in "
                               f"|z| < 0.8), B = I + 0.1 random Hermitian, unit circle, q=16 trapezoid nodes, "
                               f"m0 in {{16, 32}}, R-FEAST, tol 1e-10",
                   "mode": mode_names[args.mode],
                   "step": "batch setup (one graph launch: assembly + 16 LUs of every pencil) + lockstep "
                           "iterations of all pencils to 1e-10",
                   "pivoting": args.pivoting},
        "time_to_1e10_s": head["ms_per_step"] / 1e3,
        "iters_per_s_after_setup": head["iters_per_s_after_setup"],
        "eig_err_vs_oracle": head["eig_err_vs_oracle"],
        "batched_speedup_vs_one_at_a_time": head["batched_speedup"],
        "speedup_vs_fp64": (out["fp64"]["ms_per_step"] / head["ms_per_step"]) if "fp64" in out else None,
        "speedup_vs_fp64_after_setup": (head["iters_per_s_after_setup"] / out["fp64"]["iters_per_s_after_setup"])
                                       if "fp64" in out else None,
        "modes": out,
        "timed_run_phases": phases,
        "roofline": roofline,
        "panel_tuning": tuning,
        "tile_tuning": tiles,
        "cpu_baseline": cpu,
        "extra_workloads": extras or None,
    }
    print(json.dumps(line), flush=True)


def single_pencil_summary(args, fm, torch, dev, name):
    """One solve per mode of a single-pencil workload (n = 4096 R-FEAST or n = 8192 Bi-FEAST), after
    one warm-up, for the extra keys of the default bench line."""
    P, U0h, ref, g = load_workload(name)
    variant = "Bi" if name == "c3" else "R"
    A, B, U0 = fm.to_device(P.A, dev), fm.to_device(P.B, dev), fm.to_device(U0h, dev)
    nbytes = max(fm.workspace_size(P.n, P.m0, fm.binding.make_contour(P.center, P.radius, 1.0, P.q),
                                   fm.binding.make_options(m, variant, pivoting=args.pivoting), True)
                 for m in ("fp32", "fp64"))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    res = dict(workload=f"n={P.n}, circle c={P.center}, R*={P.radius:.6g} (m={g['m']}), q={P.q}, m0={P.m0}, "
                        f"{variant}-FEAST, tol 1e-10")
    for mode in ("fp32", "fp64", "fp16"):
        wall, results, phases = run_steps(fm, torch, A, B, U0, P, mode, 1, 1 if mode == "fp32" else 0, ws,
                                          timing=True, variant=variant, pivoting=args.pivoting)
        r = results[0]
        setup_ms = sum(phases[k]["ms"] for k in ("lu_update", "lu_panel", "lu_other"))
        res[mode] = dict(time_to_1e10_ms=1e3 * wall, iterations=r.iterations, converged=r.converged,
                         m=len(r.lam), eig_err_vs_oracle=match_err(r.lam, ref),
                         factor_device_ms=setup_ms, escalated_to_fp32=bool(r.escalated),
                         iters_per_s=r.iterations / wall)
        log(f"{name} {mode}: {1e3 * wall:.1f} ms, {r.iterations} iterations, m={len(r.lam)}, "
            f"err {res[mode]['eig_err_vs_oracle']:.1e}, factorisation {setup_ms:.1f} ms"
            + (" (escalated)" if r.escalated else ""))
    res["speedup_fp32_vs_fp64"] = res["fp64"]["time_to_1e10_ms"] / res["fp32"]["time_to_1e10_ms"]
    res["speedup_fp16_vs_fp64"] = res["fp64"]["time_to_1e10_ms"] / res["fp16"]["time_to_1e10_ms"]
    del A, B, U0, ws
    torch.cuda.empty_cache()
    return res


def bench_conj(args, fm, torch, dev):
    """A real pencil on the unit circle: the nodes with Im z >= 0 are factored and their conjugates
    reuse them (13 of 24 trapezoid nodes), timed beside the same solve with all 24 factorisations."""
    import pencils
    from oracle import brute
    t0 = time.perf_counter()
    P = pencils.real_workload()
    log(f"real pencil n={P.n} generated in {time.perf_counter() - t0:.1f} s, m={P.m}")
    ref = brute.eigenvalues_inside(P.lam, 0j, 1.0)
    A, B = fm.to_device(P.A, dev), fm.to_device(P.B, dev)
    U0 = fm.to_device(pencils.start_block(5, P.n, P.m0), dev)
    C = fm.binding.make_contour(P.center, P.radius, 1.0, P.q)
    o = fm.binding.make_options(args.mode, "R", pivoting=args.pivoting)
    ws = torch.empty(fm.workspace_size(P.n, P.m0, C, o, True), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    out = {}
    for conj in ("real", "none"):
        steps = args.steps if conj == "real" else max(1, min(args.steps, 2))
        wall, results, phases = run_steps(fm, torch, A, B, U0, P, args.mode, steps, args.warmup, ws, timing=True,
                                          pivoting=args.pivoting, conj_nodes=conj)
        factor_ms = sum(phases[k]["ms"] for k in ("lu_update", "lu_panel", "lu_other")) / steps
        out[conj] = dict(ms_per_step=1e3 * wall / steps, iters_per_s=sum(r.iterations for r in results) / wall,
                         iterations=results[0].iterations, converged=all(r.converged for r in results),
                         m=len(results[0].lam), eig_err_vs_oracle=max(match_err(r.lam, ref) for r in results),
                         factor_ms=factor_ms, solve_ms=phases["solve"]["ms"] / steps,
                         refine_ms=phases["refine"]["ms"] / steps,
                         phases={k: dict(ms=v["ms"] / steps, launches=v["launches"] // steps,
                                         tflops=(v["flops"] / (v["ms"] * 1e-3) / 1e12) if v["ms"] > 0 else None)
                                 for k, v in phases.items()})
        log(f"conj_nodes={conj}: {out[conj]['ms_per_step']:.1f} ms/solve (factor {factor_ms:.1f} ms, solve "
            f"{out[conj]['solve_ms']:.1f} ms), {out[conj]['iterations']} iterations, m={out[conj]['m']}, "
            f"err {out[conj]['eig_err_vs_oracle']:.1e}")
    head = out["real"]
    upd = head["phases"]["lu_update"]
    elem = 16 if args.mode == "fp64" else 8
    q_factored = P.q // 2 + 1
    nbytes, launches = update_bytes(P.n, q_factored, elem)
    roofline = dict(**update_roof_fields(upd["tflops"], args.mode), traffic=None, kernel_phase="lu_update", avg_launch_ms=upd["ms"] / max(1, upd["launches"]),
                    launches=upd["launches"], algorithmic_bytes_per_launch=nbytes / max(1, launches))
    line = {
        "metric": METRIC,
        "value": head["iters_per_s"],
        "unit": "FEAST iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if args.mode == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"real generalized pencil n={P.n} (20 conjugate pairs and 8 real eigenvalues in "
                               f"|z| < 0.8), unit circle, q={P.q} trapezoid nodes of which {q_factored} factored, "
                               f"m0={P.m0}, R-FEAST, tol 1e-10",
                   "mode": "FP32 LU (trailing updates on FP16 matrix cores, split operands) + FP64 shifted-residual correction" if args.mode == "fp32" else "FP64",
                   "step": "setup (assembly + factored nodes) + iterations to 1e-10",
                   "conj_nodes": "real", "pivoting": args.pivoting},
        "time_to_1e10_s": head["ms_per_step"] / 1e3,
        "iterations": head["iterations"],
        "eig_err_vs_oracle": head["eig_err_vs_oracle"],
        "shared_conjugate_nodes": out["real"],
        "all_nodes": out["none"],
        "speedup_vs_all_nodes": out["none"]["ms_per_step"] / head["ms_per_step"],
        "factor_speedup_vs_all_nodes": out["none"]["factor_ms"] / head["factor_ms"],
        "roofline": roofline,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def bench_domains(args, fm, torch, dev):
    """Multi-domain run: one n = 2048 pencil (eigenvector basis of condition <= 1e2), m eigenvalues
    (--domain-eigs) in the square [-1, 1]^2 spread over an 8 x 8 grid of cells; count estimates for
    the 64 cells (one probe batch, 16 probes), a partition into tiles of about --domain-target
    eigenvalues, one batch over the tiles.  Timed beside one domain covering the square."""
    import pencils
    n, m_in, grid, region, target = 2048, args.domain_eigs, (8, 8), (-1.0, 1.0, -1.0, 1.0), args.domain_target
    rng = np.random.default_rng([pencils.base_seed(6), 0])
    lam = pencils.grid_spectrum(rng, n, m_in, region, grid)
    A, _ = pencils.prescribed_pencil(rng, n, lam, cond_max=1e2)
    ref = lam[(lam.real > -1) & (lam.real < 1) & (lam.imag > -1) & (lam.imag < 1)]
    Ad = fm.to_device(A, dev)
    probes = fm.to_device(pencils.rademacher_complex(np.random.default_rng([pencils.base_seed(6), 1]), (n, 16)), dev)
    U1 = fm.to_device(pencils.start_block(6, n, fm.m0_from_estimate(m_in)), dev)
    torch.cuda.synchronize()

    def tiled():
        t = time.perf_counter()
        rects, est, res, rcs = fm.multi_domain(Ad, None, region, probes, grid=grid, target=target, q=16,
                                               precision=args.mode, max_iter=60)
        torch.cuda.synchronize()
        return time.perf_counter() - t, rects, est, res, rcs

    def single():
        t = time.perf_counter()
        with fm.Feast(Ad, None, q=32, m0=U1.shape[1], rule="gauss-legendre", precision=args.mode, max_iter=60,
                      pieces=fm.rectangle(*region)) as F:
            r = F.iterate(U1)
        torch.cuda.synchronize()
        return time.perf_counter() - t, r

    for _ in range(args.warmup):
        tiled()
    runs = [tiled() for _ in range(args.steps)]
    wall = float(np.median([r[0] for r in runs]))
    _, rects, est, res, rcs = runs[0]
    found = np.concatenate([r.lam for r in res])
    counts = [len(r.lam) for r in res]
    iters = sum(r.iterations for r in res)
    err = match_err(found, ref) if len(found) == len(ref) else float("inf")
    log(f"tiled: {1e3 * wall:.1f} ms, {len(rects)} tiles, counts {counts}, {iters} tile iterations, "
        f"found {len(found)} of {len(ref)}, err {err:.1e}")
    s_wall, s_res = single()
    s_err = match_err(s_res.lam, ref) if len(s_res.lam) == len(ref) else float("inf")
    log(f"one domain (m0={U1.shape[1]}, q=32): {1e3 * s_wall:.1f} ms, {s_res.iterations} iterations, "
        f"found {len(s_res.lam)}, err {s_err:.1e}")
    line = {
        "metric": METRIC,
        "value": iters / wall,
        "unit": "FEAST iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if args.mode == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"one pencil n={n}, B=I, {m_in} eigenvalues in the square [-1,1]^2 (8 x 8 cells, "
                               f"away from cell edges), the rest in 2 < |z| < 5; probe batch over the 64 cells "
                               f"(8 Gauss-Legendre nodes, 16 probes, cond(V) <= 1e2), tiles of about {target} eigenvalues, "
                               f"q=16 per tile, R-FEAST, tol 1e-10",
                   "mode": "FP32 LU (trailing updates on FP16 matrix cores, split operands) + FP64 shifted-residual correction" if args.mode == "fp32" else "FP64",
                   "step": "count estimates + partition + one batch over the tiles (setup and iterations)"},
        "time_to_1e10_s": wall,
        "tiles": len(rects),
        "tile_counts": counts,
        "tile_estimates": [float(v) for v in est],
        "balance_max_over_mean": float(max(counts) / np.mean(counts)),
        "eigenvalues_found": int(len(found)), "eigenvalues_inside": int(len(ref)),
        "eig_err_vs_oracle": err,
        "one_domain": {"ms": 1e3 * s_wall, "iterations": int(s_res.iterations), "m0": int(U1.shape[1]),
                       "found": int(len(s_res.lam)), "eig_err_vs_oracle": s_err},
        "speedup_vs_one_domain": s_wall / wall,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


M0_CAP = 128   # subspace capacity of the estimator's solves (restarts double m0 up to it)


def m0_solve(fm, torch, dev, P, V, m0_rule, cap):
    """binding.sized_solve over the held-out pencils, timed end to end; returns (wall s, results,
    m0s, restarts, GFLOP)."""
    import pencils
    n = P[0].n
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, m0s, restarts, work = fm.binding.sized_solve(
        [(p.A, None) for p in P], [(p.center, p.radius, 1.0) for p in P],
        lambda i, m0: fm.to_device(pencils.start_block(4, n, m0), dev), m0_rule=m0_rule, cap=cap, probes=V)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, res, m0s, restarts, sum(work.values()) / 1e9


def m0_labels_and_features(fm, torch, dev, ids, V, chunk=512):
    """Training data of the estimator: for each pencil its probe features (the 16-node filter of its
    FEAST context) and its label, the eigenvalue count the plain FP64 method (R-FEAST, q = 16,
    m0 = 64) finds inside the contour; pencils generated on the device chunk by chunk."""
    import pencils
    feats, labels, construct, ok = [], [], [], 0
    for i0 in range(0, len(ids), chunk):
        part = [pencils.c4_pencil(j, 512, basis=bb, device=dev) for j, bb in ids[i0:i0 + chunk]]
        b = fm.FeastBatch([(p.A, None) for p in part], [(p.center, p.radius, 1.0) for p in part], m0=64, q=16,
                          precision="fp64")
        feats += list(b.probe_features(V))
        res, rcs = b.iterate([fm.to_device(pencils.start_block(4, 512, 64), dev) for _ in part])
        b.close()
        for p, r in zip(part, res):
            labels.append(len(r.lam))
            construct.append(p.m)
            ok += int(r.converged)
        del part
        torch.cuda.empty_cache()
        if (i0 // chunk) % 8 == 7:
            log(f"  labels of {len(labels)} pencils")
    return np.array(feats), np.array(labels, dtype=np.float64), np.array(construct), ok


def bench_m0(args, fm, torch, dev):
    """Learned subspace size.  Training: 20,000 pencils (n = 512, B = I, random circles, 0-48
    eigenvalues inside) labelled by the plain FP64 FEAST run's count, with features from 8
    Rademacher probes through the 16-node filter; the perceptron (FP16 operands) trained by the
    library's kernels.  Held out: 2,048 pencils solved in FP32 with the rank check, each strategy
    end to end (factorisation, probes, network, iterations, restarts on the same factorisations):
    m0 from the estimator, a fixed m0 = 64, and 1.5 x the mean probe trace."""
    import pencils
    from oracle import mlp as omlp
    n, ntr, nev = 512, args.count_train, args.count_eval
    V = fm.to_device(pencils.probe_block(4, 0, n), dev)
    t0 = time.perf_counter()
    Xtr, ytr, ctr, conv = m0_labels_and_features(fm, torch, dev, pencils.c4_split("train", ntr), V)
    t_label = time.perf_counter() - t0
    log(f"{ntr} training pencils: features and FP64 FEAST labels in {t_label:.1f} s ({conv} converged; "
        f"labels equal to the construction count for {int(np.sum(ytr == ctr))})")
    ev = [pencils.c4_pencil(j, n, basis=b, device=dev) for j, b in pencils.c4_split("eval", nev)]
    torch.cuda.synchronize()
    d = Xtr.shape[1]
    net = fm.MLP(omlp.flatten(omlp.init_params(np.random.default_rng(7), d)), n_in=d, half=True, max_batch=512,
                 device=dev)
    Xd = torch.from_numpy(Xtr.astype(np.float32)).to(dev)
    yd = torch.from_numpy(ytr.astype(np.float32)).to(dev)
    net.fit_standardization(Xd)
    rng = np.random.default_rng(8)
    t0 = time.perf_counter()
    steps = 0
    for epoch in range(args.epochs):
        perm = torch.from_numpy(rng.permutation(ntr)).to(dev)
        Xp, yp = Xd[perm].contiguous(), yd[perm].contiguous()
        for b in range(0, ntr - 127, 128):
            net.train_step(Xp[b:b + 128], yp[b:b + 128], lr=1e-3)
            steps += 1
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"training: {steps} Adam steps in {t_train:.1f} s")
    y_ev = np.array([p.m for p in ev], dtype=np.float64)
    est = {}

    def estimator(feats, i0):
        x = torch.from_numpy(feats.astype(np.float32)).to(dev)
        m_hat = net.forward(x).cpu().numpy().astype(np.float64)
        est.update({i0 + k: v for k, v in enumerate(m_hat)})
        return [fm.m0_from_estimate(v) for v in m_hat]

    def probe_mean(feats, i0):
        t = feats[:, 0:2 * V.shape[1]:2].mean(axis=1)
        return [max(8, int(np.ceil(1.5 * max(x, 0.0) / 8.0)) * 8) for x in t]

    strategies = [("estimator", estimator, M0_CAP), ("fixed_64", None, 64), ("probe_mean_x1.5", probe_mean, M0_CAP)]
    out = {}
    for name, rule, cap in strategies:
        m0_solve(fm, torch, dev, ev[:256], V, rule, cap)      # warm-up
        wall, res, m0s, restarts, gflop = m0_solve(fm, torch, dev, ev, V, rule, cap)
        ok = sum(1 for p, r in zip(ev, res) if r.converged and len(r.lam) == p.m)
        out[name] = dict(ms_per_pencil=1e3 * wall / nev, mean_m0=float(np.mean(m0s)), restarts=restarts,
                         iterations=int(sum(r.iterations for r in res)), gflop_per_pencil=gflop / nev, correct=ok)
        log(f"{name}: {out[name]}")
    m_hat = np.array([est[i] for i in range(nev)])
    line = {
        "metric": "learned m0: FEAST work and time per held-out pencil (estimator vs fixed m0 = 64 and the "
                  "probe-mean rule)",
        "value": out["fixed_64"]["gflop_per_pencil"] / out["estimator"]["gflop_per_pencil"],
        "unit": "x (GFLOP per pencil, fixed m0 = 64 / estimator m0)",
        "n_gpus": 1, "higher_is_better": True, "data": "synthetic", "dtype": "f16 MLP + f32 LU + f64 correction",
        "config": {"workload": f"{ntr} training / {nev} held-out pencils, n={n}, B=I, random circles, "
                               f"m ~ U{{0..48}}; labels: FP64 R-FEAST counts (q=16, m0=64); features: 8 Rademacher "
                               f"probes through the solve's own 16-node filter + (c, R); MLP {d}-256-256-1 FP16, "
                               f"{args.epochs} epochs; held-out FEAST q=16 FP32 + FP64 shifted-residual correction "
                               f"with the rank check, restarts on the same factorisations"},
        "label_s": t_label, "train_s": t_train,
        "labels_equal_construction": int(np.sum(ytr == ctr)), "label_runs_converged": conv,
        "heldout_mean_abs_err": float(np.mean(np.abs(m_hat - y_ev))),
        "heldout_rmse": float(np.sqrt(np.mean((m_hat - y_ev) ** 2))),
        "speedup_time_vs_fixed_64": out["fixed_64"]["ms_per_pencil"] / out["estimator"]["ms_per_pencil"],
        "gain_gflop_vs_probe_mean": out["probe_mean_x1.5"]["gflop_per_pencil"] / out["estimator"]["gflop_per_pencil"],
        "strategies": out,
    }
    print(json.dumps(line), flush=True)


def pencils_start(p, j):
    import pencils
    return pencils.start_block(2, p.n, p.m0, salt=10**6 + j)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", default="fp32", choices=["fp32", "fp64", "fp16"])
    ap.add_argument("--workload", default="c2", choices=["c1", "c3", "c2", "c4", "real4096", "domains"],
                    help="real4096: a real pencil whose conjugate nodes share factorisations; domains: "
                         "load-balanced tiles of a region in one batch")
    ap.add_argument("--count-train", type=int, default=20000, help="training pencils of the learned-m0 workload")
    ap.add_argument("--count-eval", type=int, default=2048, help="held-out pencils of the learned-m0 workload")
    ap.add_argument("--epochs", type=int, default=150)
    ap.add_argument("--count", type=int, default=64, help="pencils of the batched workload (c2)")
    ap.add_argument("--domain-eigs", type=int, default=512, help="eigenvalues in the region (domains workload)")
    ap.add_argument("--domain-target", type=int, default=48, help="eigenvalues per tile (domains workload)")
    ap.add_argument("--variant", default=None, choices=["R", "Bi", "L"],
                    help="R-FEAST (default for the n=4096 workload), Bi-FEAST (default for n=8192) or the "
                         "left-projector variant")
    ap.add_argument("--tune", action="store_true", help="measure the panel-kernel crossover before timing")
    ap.add_argument("--counters", action="store_true",
                    help="run only a calibration kernel (elementwise multiply, 256 MiB in and out) and one "
                         "factorisation of the workload, for hardware-counter runs")
    ap.add_argument("--pivoting", default="tournament", choices=["tournament", "partial"])
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="record the update's traffic from two rocprofv3 --pmc runs of --counters (no GPU)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batched workload: skip the one-pencil-at-a-time comparison (kernel profiles)")
    ap.add_argument("--no-extras", action="store_true",
                    help="batched workload: skip the single-pencil n=4096 and n=8192 extra keys")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one MI355X: the library is a single-GPU build (several GPUs would each "
              "own a share of the contour nodes and sum their filter blocks); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.pmc_summary:
        notes = {"c1": "n=4096 complex-symmetric pencil, q=24, factorisation (setup only)",
                 "c2": "64 pencils n ~ U{256..2048}, q=16, one factorisation graph (setup only)",
                 "c3": "n=8192 complex-symmetric pencil, q=32, factorisation (setup only)"}
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.workload, args.mode, notes[args.workload])
        return

    import torch
    import paper_1404_2891_amd as fm
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = "cuda:0"
    if args.counters:
        x = torch.ones(64 * 2**20, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        torch.mul(x, 2.0, out=y)
        torch.cuda.synchronize()
        if args.workload == "c2":
            # built on the host (same draws; no generator kernels among the counted dispatches)
            P = load_batch(args.count, None)
            log("batch built")
            mats = [(fm.to_device(p.A, dev), fm.to_device(p.B, dev)) for p in P]
            b = fm.FeastBatch(mats, (0j, 1.0, 1.0), m0=[p.m0 for p in P], q=16,
                              precision=args.mode, pivoting=args.pivoting)
            torch.cuda.synchronize()
            b.close()
        else:
            P, U0h, ref, g = load_workload(args.workload)
            F = fm.Feast(fm.to_device(P.A, dev), fm.to_device(P.B, dev), P.center, P.radius, 1.0, P.q, P.m0,
                         precision=args.mode)
            torch.cuda.synchronize()
            F.close()
        log("counters run done")
        return
    if args.workload == "c2":
        bench_batch(args, fm, torch, dev)
        return
    if args.workload == "c4":
        bench_m0(args, fm, torch, dev)
        return
    if args.workload == "real4096":
        bench_conj(args, fm, torch, dev)
        return
    if args.workload == "domains":
        bench_domains(args, fm, torch, dev)
        return
    variant = args.variant or ("Bi" if args.workload == "c3" else "R")
    P, U0h, ref, g = load_workload(args.workload)
    log(f"workload {P.name}: n={P.n} q={P.q} m0={P.m0} R*={P.radius:.6g} m={g['m']}")
    A = fm.to_device(P.A, dev)
    B = fm.to_device(P.B, dev)
    U0 = fm.to_device(U0h, dev)
    nbytes = max(fm.workspace_size(P.n, P.m0, fm.binding.make_contour(P.center, P.radius, 1.0, P.q),
                                   fm.binding.make_options(m, variant, pivoting=args.pivoting), True)
                   for m in ("fp32", "fp64"))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    modes = [args.mode] + ([] if args.no_compare else [m for m in ("fp64", "fp32", "fp16") if m != args.mode])
    tuning = tune_panels(fm, P.q, modes, dev) if args.tune else None
    tiles = tune_tiles(fm, P.q, modes, dev)
    out = {}
    for mode in modes:
        steps = args.steps if mode == args.mode else max(1, min(args.steps, 2))
        wall, results, phases = run_steps(fm, torch, A, B, U0, P, mode, steps, args.warmup, ws, timing=True,
                                          variant=variant, pivoting=args.pivoting)
        iters = sum(r.iterations for r in results)
        errs = [match_err(r.lam, ref) for r in results]
        out[mode] = dict(ms_per_step=1e3 * wall / steps, iters_per_s=iters / wall, iterations=results[0].iterations,
                         converged=all(r.converged for r in results), m=len(results[0].lam),
                         max_resid=float(max((r.resid.max() if len(r.resid) else np.nan) for r in results)),
                         eig_err_vs_oracle=max(errs),
                         ir_sweeps=results[0].ir_sweeps, escalated_to_fp32=bool(results[0].escalated),
                         phases={k: dict(ms=v["ms"] / steps, launches=v["launches"] // steps,
                                         tflops=(v["flops"] / (v["ms"] * 1e-3) / 1e12) if v["ms"] > 0 else None)
                                 for k, v in phases.items()})
        log(f"{mode}: {out[mode]['ms_per_step']:.1f} ms/solve, {out[mode]['iterations']} iterations, "
            f"m={out[mode]['m']}, err {out[mode]['eig_err_vs_oracle']:.1e}")
        for k, v in out[mode]["phases"].items():
            log(f"   {k:14s} {v['ms']:9.2f} ms  {v['launches']:6d} launches  {v['tflops']} TF/s")

    head = out[args.mode]
    # dominant phase of the headline mode and its roofline
    # the dominant kernel: the trailing update (the largest single kernel by device time on every
    # workload, rocprofv3), or with partial pivoting the panel's column steps when they take longer
    hp = head["phases"]
    dom = "lu_panel" if (args.pivoting == "partial" and hp["lu_panel"]["ms"] > hp["lu_update"]["ms"]) else "lu_update"
    ph_all = None
    kw = dict(center=P.center, radius=P.radius, aspect=1.0, q=P.q, m0=P.m0, precision=args.mode, workspace=ws,
              variant=variant, pivoting=args.pivoting)
    with fm.Feast(A, B, timing=True, **kw) as F:
        F.iterate(U0)
        ph_all = F.timing()
    dph = ph_all[dom]
    if dom == "lu_panel":
        # the column steps of the panels: latency-bound launches that read and write the active part
        # of the panel (HBM / infinity-cache traffic, no matrix-core work)
        elem = 16 if args.mode == "fp64" else 8
        nbytes, launches = panel_bytes(P.n, P.q, elem)
        achieved = nbytes / (dph["ms"] * 1e-3) / 1e9
        roofline = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK, unit="GB/s", frac=achieved / HBM_PEAK,
                        traffic=measured_traffic("panel_step_kernel", args.workload, args.mode),
                        traffic_unit="bytes per launch (PMC FETCH_SIZE + WRITE_SIZE, calibrated)",
                        kernel="panel_step_kernel", kernel_phase=dom,
                        avg_launch_ms=dph["ms"] / launches, bytes_per_launch=nbytes / launches, launches=launches)
    elif dom == "lu_update":
        # the MFMA trailing update (grouped over four panels); algorithmic bytes per launch from its
        # operand and block sizes, measured HBM traffic from the PMC record
        prec_of_phase = "fp16" if args.mode == "fp16" else args.mode
        elem = 16 if args.mode == "fp64" else 8
        nbytes, launches = update_bytes(P.n, P.q, elem)
        achieved = dph["flops"] / (dph["ms"] * 1e-3) / 1e12
        roofline = dict(**update_roof_fields(achieved, args.mode),
                        traffic=measured_traffic("lu_update", args.workload, args.mode),
                        traffic_unit="bytes per launch (PMC FETCH_SIZE + WRITE_SIZE, calibrated)",
                        kernel_phase=dom,
                        avg_launch_ms=dph["ms"] / max(1, dph["launches"]), launches=dph["launches"],
                        flops_per_launch=dph["flops"] / max(1, dph["launches"]),
                        algorithmic_bytes_per_launch=nbytes / max(1, launches),
                        achieved_gbs=nbytes / max(1, launches) / (dph["ms"] / max(1, dph["launches"]) * 1e-3) / 1e9)
    else:
        prec_of_phase = "fp64" if (args.mode == "fp64" or dom in ("refine", "rayleigh_ritz")) else (
            "fp16" if (args.mode == "fp16" and dom == "lu_update") else "fp32")
        achieved = dph["flops"] / (dph["ms"] * 1e-3) / 1e12 if dph["ms"] > 0 else 0.0
        # a phase whose spans hold many kernel launches (the solves): figures per span
        roofline = dict(bound="mfma", achieved=achieved, peak=PEAK[prec_of_phase], unit="TFLOP/s",
                        frac=achieved / PEAK[prec_of_phase], traffic=None, kernel_phase=dom,
                        avg_span_ms=dph["ms"] / max(1, dph["launches"]),
                        flops_per_span=dph["flops"] / max(1, dph["launches"]),
                        note="phase spans of several GEMM launches; per-launch figures of the update in lu_update_roofline")
    lu = ph_all["lu_update"]
    lu_roof = update_roof_fields(lu["flops"] / (lu["ms"] * 1e-3) / 1e12 if lu["ms"] > 0 else 0.0, args.mode)
    lu_roof["avg_launch_ms"] = lu["ms"] / max(1, lu["launches"])
    # (with FP16 updates escalated to FP32 the last factorisation's updates ran in FP32)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(P, U0h, out.get("fp64", head)["iterations"], variant=variant)

    line = {
        "metric": METRIC,
        "value": head["iters_per_s"],
        "unit": "FEAST iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32+f64", "fp16": "f16+f32+f64", "fp64": "f64"}[args.mode],
        "data": "synthetic",
        "config": {"workload": f"complex-symmetric generalized pencil n={P.n}, circle c={P.center}, "
                               f"R*={P.radius:.6g} (m={g['m']} inside), q={P.q} trapezoid nodes, m0={P.m0}, "
                               f"{variant}-FEAST, tol 1e-10",
                   "mode": {"fp32": "FP32 LU (trailing updates on FP16 matrix cores, split operands) + FP64 shifted-residual correction", "fp16": "FP16-update LU + FP64 shifted-residual correction",
                            "fp64": "FP64"}[args.mode],
                   "step": "setup (assembly + q LUs) + iterations to 1e-10",
                   "pivoting": args.pivoting},
        "time_to_1e10_s": head["ms_per_step"] / 1e3,
        "iterations": head["iterations"],
        "eig_err_vs_oracle": head["eig_err_vs_oracle"],
        "modes": out,
        "speedup_vs_fp64": (out["fp64"]["ms_per_step"] / head["ms_per_step"]) if "fp64" in out else None,
        "roofline": roofline,
        "lu_update_roofline": lu_roof,
        "panel_tuning": tuning,
        "tile_tuning": tiles,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
