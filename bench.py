#!/usr/bin/env python
"""Benchmark of the solver's per-iteration hot path on one MI355X.

Workload: 256^3 Voronoi polycrystal (500 grains, seed 2), cubic elasticity
(168/121/75 GPa) with random orientations, bending through Dirichlet x faces
(curvature 1e-4 per voxel), Neumann y and z faces, TETRA2 scheme, B0 Green
operator (lambda0 = 121, mu0 = 75), equilibrium tolerance 1e-6.

A step is one complete solve of that problem from a zero displacement
(material map already resident on the device): every iteration runs the
whole hot path (strain, law, divergence, FP64 reductions and Anderson,
forward transforms, Green operator, inverse transforms, update).  The headline
value is voxel-iterations per second of the FP32-mixed path; the plain FP64
path is timed on the same GPU for the speedup and the macroscopic-stress
agreement.  The roofline entry is the dominant kernel of the FP32-mixed
iteration, timed with HIP events on the plan's stream; the CPU baseline is the
FP64 oracle on a bounded sample of the same workload family.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_polycrystal256.json")


def kernel_source_hash():
    """SHA-256 over the HIP sources, to tell whether stored counter readings
    still describe the kernels that run."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2607_05929_amd", "csrc")
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()


def stored_traffic(kernel, size):
    """HBM bytes per launch of `kernel` from the stored FETCH_SIZE / WRITE_SIZE
    readings (each scaled by the reading of a plain 1 GiB copy), or None when
    there are none for this workload or the kernels changed since."""
    if size != 256 or not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_source_hash() or kernel not in t.get("kernels", {}):
        return None
    k = t["kernels"][kernel]
    return 1024.0 * (k["fetch_KiB"] * t["fetch_factor"] + k["write_KiB"] * t["write_factor"])


def kernel_bytes(prob, plan_geom, rbytes, n_d=1.0, n_b=0.0, n_gram=1.0):
    """Algorithmic HBM bytes per launch of each iteration kernel (each field
    read or written once), FP32-mixed or FP64 storage."""
    n = prob.n
    N = [v + 1 for v in n]
    Nn = N[0] * N[1] * N[2]
    Nv = n[0] * n[1] * n[2]
    nppv = 2 if prob.scheme == 1 else 1
    R = rbytes
    s1 = plan_geom["s1"]
    s2 = plan_geom["s2"]
    kept_rows = plan_geom["kept"]     # kept nodes summed over components
    b = {}
    # fused stress + divergence: u^f (FP64) and material ids in, residual out
    b["stress_div"] = Nn * 3 * 8 + Nv * 2 + Nn * 3 * R
    b["gram"] = Nn * 3 * R * n_gram
    b["x_fwd"] = kept_rows * R * n_d + sum(s1) * R
    b["y_fwd"] = (sum(s1) + sum(s2)) * R
    b["z_green"] = 2 * sum(s2) * R
    b["y_inv"] = (sum(s1) + sum(s2)) * R
    b["x_inv_update"] = sum(s1) * R + Nn * 3 * (8 + 8 + R) + Nn * 3 * R * n_b
    return b


def geometry(prob):
    """Spectral buffer sizes (reals) and kept-node count from the transform
    chosen per axis by the pair of face conditions (Table 1): P/P DFT (n
    kept, r2c-halved on the first periodic axis), N/N DCT-I (n+1), D/D DST-I
    (n-1), N/D DCT-III and D/N DST-III (n)."""
    n = prob.n
    N = [v + 1 for v in n]
    s1, s2, kept = [], [], 0
    for q in range(3):
        M, cplx, cx = [], [], False
        k = 1
        for a in range(3):
            left, right = int(prob.bc[q][a][0]), int(prob.bc[q][a][1])
            if left == 0:
                M.append(n[a] if cx else n[a] // 2 + 1)
                cx = True
                k *= n[a]
            elif left == 2 and right == 2:
                M.append(n[a] + 1); k *= n[a] + 1
            elif left == 1 and right == 1:
                M.append(n[a] - 1); k *= n[a] - 1
            else:
                M.append(n[a]); k *= n[a]
            cplx.append(cx)
        s1.append(M[0] * N[1] * N[2] * (2 if cplx[0] else 1))
        s2.append(M[0] * M[1] * N[2] * (2 if cplx[1] else 1))
        kept += k
    return {"s1": s1, "s2": s2, "kept": kept}


def cpu_baseline():
    """FP64 oracle on a 128^3 sample of the polycrystal family (62 grains, the
    grain size of 500 grains in 256^3), its first iterations (about 30 s of
    host time; at 256^3 one oracle iteration takes minutes)."""
    import resource
    import workloads as W
    from oracle import solver as osolver
    nv = 128
    prob = W.config_polycrystal_bending(nv=nv, n_grains=62, seed=2)
    prob.max_iter = 2
    ru0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.time()
    r = osolver.solve(prob)
    wall = time.time() - t0
    ru1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (ru1.ru_utime - ru0.ru_utime) + (ru1.ru_stime - ru0.ru_stime)
    iters = sum(r["iters"])
    value = nv ** 3 * iters / wall
    cores = max(1, round(cpu / wall))
    return {"value": value, "unit": "voxel-iter/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle, 128^3 polycrystal (62 grains), TETRA2, {iters} iterations "
                      f"incl. setup, {wall:.1f} s wall, {os.cpu_count()} host cpus visible"}


def batch_sample(B, W, count=512, tol=1e-6, log=None):
    """The batched configuration in full: 512 independent two-phase elastic
    RVEs (seed 4: grids 32^3-96^3, 8-32 spheres, contrast 2-100, random
    per-axis BCs).  The transform kernels of every plan are autotuned (one
    timing per transform signature, the library keeps the choice), then all
    solves run as one FP32-mixed batch; the same solves run one at a time in
    FP64.  Both stop at the configuration's tolerance 1e-6; plan set-up and
    tuning are timed apart.  Parity: <sigma> FP32 batch vs FP64 for every
    member, and both against the oracle's stored results for eight members."""
    import numpy as np
    import torch
    log = log or (lambda m: None)
    t0 = time.time()
    probs = W.config_batch(count=count, prec=W.FP32_MIXED, tol=tol)
    gen_s = time.time() - t0
    vox = np.array([p.n[0] * p.n[1] * p.n[2] for p in probs], dtype=np.float64)
    torch.cuda.synchronize()
    t0 = time.time()
    plans32 = [B.Plan(p, W.FP32_MIXED) for p in probs]
    torch.cuda.synchronize()
    setup32 = time.time() - t0
    t0 = time.time()
    choices = {}
    for pl in plans32:
        c = "".join(str(v) for v in pl.autotune(n_iter=3)["choice"])
        choices[c] = choices.get(c, 0) + 1
    tune_s = time.time() - t0
    log(f"batch: {count} problems generated in {gen_s:.1f} s, FP32 plans {setup32:.2f} s, autotuned in {tune_s:.1f} s")
    torch.cuda.synchronize()
    t0 = time.time()
    res = B.batch_solve(probs, plans=plans32)
    torch.cuda.synchronize()
    t32 = time.time() - t0
    for pl in plans32:
        pl.close()
    vi32 = float(sum(v * sum(r["iters"]) for v, r in zip(vox, res)))
    t0 = time.time()
    plans64 = [B.Plan(p, W.FP64) for p in probs]
    torch.cuda.synchronize()
    setup64 = time.time() - t0
    t0 = time.time()
    r64 = [pl.solve(fields=False) for pl in plans64]
    torch.cuda.synchronize()
    t64 = time.time() - t0
    for pl in plans64:
        pl.close()
    vi64 = float(sum(v * sum(r["iters"]) for v, r in zip(vox, r64)))

    def rel(a, b):
        return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())
    diffs = [rel(a["macro_sigma"], b["macro_sigma"]) for a, b in zip(res, r64)]
    gold = {}
    gpath = os.path.join(ROOT, "tests", "golden", "batch_members.json")
    if os.path.exists(gpath):
        with open(gpath) as f:
            for m in json.load(f)["members"]:
                k = m["index"]
                gold[k] = (rel(res[k]["macro_sigma"], m["macro_sigma"]), rel(r64[k]["macro_sigma"], m["macro_sigma"]))
    ok = all(r["rc"] == 0 for r in res) and all(all(r["converged"]) for r in r64)
    return {"solves": count, "sizes": sorted({int(p.n[0]) for p in probs}), "voxels": float(vox.sum()),
            "tol_fp32": tol, "tol_fp64": tol, "generate_s": gen_s, "plan_setup_s_fp32": setup32,
            "autotune_s": tune_s, "transform_choices": choices, "plan_setup_s_fp64": setup64,
            "fp32_batch_s": t32, "fp32_batch_voxel_iter_s": vi32 / t32,
            "fp64_one_at_a_time_s": t64, "fp64_one_at_a_time_voxel_iter_s": vi64 / t64,
            "iterations_fp32_over_fp64": vi32 / vi64,
            "speedup": (vi64 / t32) / (vi64 / t64), "speedup_note": "FP64 one at a time time / FP32 batch time",
            "max_macro_rel_diff_fp32_vs_fp64": max(diffs),
            "oracle_macro_rel_err": {str(k): {"fp32_batch": a, "fp64": b} for k, (a, b) in gold.items()},
            "all_converged": ok}


def serving_sample(B, W, prec, count=16, rate=200.0, sizes=(32, 64, 96), n_steps=10, arena_gib=48, log=None):
    """Continuous batching of a Poisson stream of crystal-plasticity
    torsion-bending solves through the server API, in real time: latency from
    arrival to completion (queueing included)."""
    reqs = W.serving_stream(count=count, rate=rate, sizes=sizes, n_steps=n_steps, prec=prec)
    srv = B.Server(arena_bytes=arena_gib << 30, max_active=64)
    t0 = time.time()
    tickets, k, n_done = [], 0, 0
    while True:
        now = time.time() - t0
        while k < len(reqs) and reqs[k].arrival_s <= now:
            tickets.append(srv.submit(reqs[k].problem, arrival_s=reqs[k].arrival_s, now_s=now, prec=prec))
            k += 1
        srv.step(4, time.time() - t0)
        done = sum(1 for t in tickets if srv.poll(t)[0] == 2)
        if log and done > n_done:
            log(f"serving: {done}/{len(reqs)} requests done after {time.time() - t0:.1f} s")
        n_done = done
        if k == len(reqs) and done == len(reqs):
            break
    wall = time.time() - t0
    st = srv.stats()
    srv.close()
    return {"requests": count, "rate_req_s": rate, "sizes": list(sizes), "increments": n_steps,
            "prec": "fp32-mixed" if prec == W.FP32_MIXED else "fp64",
            "law": "FCC crystal plasticity, TETRA2, tol 1e-6", "completed": st["completed"],
            "p50_latency_s": st["p50_latency_s"], "p99_latency_s": st["p99_latency_s"],
            "mean_latency_s": st["mean_latency_s"], "wall_s": wall,
            "throughput_voxel_iter_s": st["voxel_iters"] / wall, "arena_peak_bytes": st["arena_peak"]}


def serving_sweep(B, W, rates=(2.0, 4.0, 8.0, 16.0, 32.0), count=40, sizes=(32,), log=None):
    """Offered-rate sweep on 32^3 requests (FP32-mixed): the highest rate at
    which p99 latency stays within twice the p50 of the lowest rate."""
    out = []
    for r in rates:
        s = serving_sample(B, W, W.FP32_MIXED, count=count, rate=r, sizes=sizes, n_steps=10, arena_gib=16, log=log)
        out.append(s)
        if log:
            log(f"sweep rate {r}: p50 {s['p50_latency_s']:.3f} s p99 {s['p99_latency_s']:.3f} s")
    base = out[0]["p50_latency_s"]
    stable = [s["rate_req_s"] for s in out if s["p99_latency_s"] <= 2.0 * base]
    return {"rates": [s["rate_req_s"] for s in out], "p50": [s["p50_latency_s"] for s in out],
            "p99": [s["p99_latency_s"] for s in out], "highest_stable_rate": max(stable) if stable else None,
            "criterion": "p99 <= 2 x p50 at the lowest rate", "sizes": list(sizes), "requests_per_rate": count}


FP32_VECTOR_PEAK_TFLOPS = 157.3      # MI355X, 256 CUs at 2.4 GHz
FP64_VECTOR_PEAK_TFLOPS = 78.6


def sdiv_flops_per_voxel(prob):
    """Algorithmic flops of the fused real-space step per voxel (TETRA2 with an
    anisotropic elastic law; HEX1 has one integration point):
    strain per point 51 (9 tetrahedron derivatives of 4 signed corner values
    and a scale: 36; plus the prescribed-field gradient: 9; symmetrisation:
    6); law per point 66 (6 x 6 stiffness times the strain); divergence per
    node 72 (3 components x 24 signed voxel-point terms); reductions 46
    (w |sigma|^2 and <sigma> per point, |D|^2 per node)."""
    npts = 2 if prob.scheme == 1 else 1
    return npts * (51 + 66 + 14 + 6) + 72 + 6


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--serving-full", action="store_true",
                    help="also serve a sample spanning the configuration's grid range 32^3-192^3")
    ap.add_argument("--serving-sweep", action="store_true",
                    help="also sweep the offered rate for the highest stable p99")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; sharding a solve or a batch "
                                   "across GPUs is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    from paper_2607_05929_amd import binding as B

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    # a plain 1 GiB device copy: the on-box copy ceiling (also the reference
    # reading that scales the FETCH_SIZE / WRITE_SIZE counters)
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    t = time.time()
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * (1 << 30) / (time.time() - t) / 1e9
    log(f"copy ceiling: 1 GiB read + 1 GiB write per launch, {copy_gbs:.0f} GB/s")
    del a, b

    t = time.time()
    prob = W.config_polycrystal_bending(nv=args.size)
    log(f"generated {args.size}^3 polycrystal in {time.time() - t:.1f} s")
    Nv = prob.n_vox

    p32 = B.Plan(prob, prec=W.FP32_MIXED)
    log("FP32-mixed plan ready")
    for _ in range(args.warmup):
        p32.reset()
        r = p32.solve(fields=False)
        log(f"warmup solve: {r['iters']} iterations")
    torch.cuda.synchronize()
    iters32 = 0
    macro32 = None
    t0 = time.time()
    for _ in range(args.steps):
        p32.reset(sync=False)
        r = p32.solve(fields=False)
        iters32 += sum(r["iters"])
        macro32 = r["macro_sigma"][-1]
        conv32 = all(r["converged"])
    torch.cuda.synchronize()
    t32 = time.time() - t0
    value = Nv * iters32 / t32
    log(f"FP32-mixed: {iters32} iterations in {t32:.3f} s -> {value:.3e} voxel-iter/s")

    prof = p32.profile(n_iter=12)
    log("per-kernel ms: " + ", ".join(f"{k}={v:.3f}" for k, v in prof.items()))
    geom = geometry(prob)
    aa_frac = 1.0 / prob.aa_period
    nbytes = kernel_bytes(prob, geom, 4, n_d=1 + aa_frac * (prob.aa_depth - 1),
                          n_b=aa_frac * (prob.aa_depth - 1), n_gram=prob.aa_depth)
    dom = max((k for k in prof if k in nbytes), key=lambda k: prof[k])
    iter_ms = sum(prof.values())
    iter_bytes = sum(nbytes.values())
    passes = {k: {"ms": prof[k], "algorithmic_bytes": nbytes[k],
                  "GBs": nbytes[k] / (prof[k] * 1e-3) / 1e9,
                  "frac_of_8TBs": nbytes[k] / (prof[k] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                  "frac_of_copy": nbytes[k] / (prof[k] * 1e-3) / 1e9 / copy_gbs}
              for k in ("x_fwd", "y_fwd", "z_green", "y_inv", "x_inv_update")}
    tp_ms = sum(v["ms"] for v in passes.values())
    tp_bytes = sum(v["algorithmic_bytes"] for v in passes.values())
    if dom == "stress_div":
        # the fused real-space step is bound by vector ALU issue (measured VALU busy
        # fraction; its HBM traffic runs far below the copy ceiling)
        flops = sdiv_flops_per_voxel(prob) * Nv
        achieved = flops / (prof[dom] * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                "traffic": stored_traffic(dom, args.size), "algorithmic_flops": flops,
                "flops_per_voxel": sdiv_flops_per_voxel(prob),
                "algorithmic_bytes": nbytes[dom], "hbm_GBs": nbytes[dom] / (prof[dom] * 1e-3) / 1e9}
    else:
        achieved = nbytes[dom] / (prof[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic(dom, args.size),
                "algorithmic_bytes": nbytes[dom]}
    roof.update({"ms": prof[dom], "iteration_ms": iter_ms, "iteration_bytes": iter_bytes,
                 "iteration_GBs": iter_bytes / (iter_ms * 1e-3) / 1e9, "per_kernel_ms": prof,
                 "transform_passes": passes,
                 "transform_passes_GBs": tp_bytes / (tp_ms * 1e-3) / 1e9,
                 "transform_passes_frac_of_8TBs": tp_bytes / (tp_ms * 1e-3) / 1e9 / HBM_PEAK_GBS})
    p32.close()

    fp64 = None
    if not args.no_fp64:
        p64 = B.Plan(prob, prec=W.FP64)
        p64.reset()
        torch.cuda.synchronize()
        t1 = time.time()
        r64 = p64.solve(fields=False)
        torch.cuda.synchronize()
        t64 = time.time() - t1
        it64 = sum(r64["iters"])
        m64 = r64["macro_sigma"][-1]
        rel = float(np.abs(macro32 - m64).max() / np.abs(m64).max())
        fp64 = {"value": Nv * it64 / t64, "iters": it64, "s_per_solve": t64,
                "converged": all(r64["converged"]), "macro_rel_diff_fp32_vs_fp64": rel}
        p64.close()
        log(f"FP64: {it64} iterations in {t64:.3f} s; <sigma> FP32 vs FP64 rel diff {rel:.2e}")

    parity = None
    gpath = os.path.join(ROOT, "tests", "golden", f"polycrystal{args.size}.json")
    if not args.no_parity and os.path.exists(gpath):
        # against the FP64 oracle's stored solution (tol 1e-8): <sigma> and
        # the stress at 1024 sampled voxels (faces and corners included)
        with open(gpath) as f:
            g = json.load(f)
        parity = {"oracle_tol": g["oracle_tol"]}
        vox = g["voxels_xyz"]
        gs = np.array(g["sigma"])
        for name, prec in (("fp32", W.FP32_MIXED), ("fp64", W.FP64)):
            pl = B.Plan(prob, prec=prec)
            r = pl.solve(fields=True)
            pl.close()
            sig = np.array([[[r["sig"][c, ip, z, y, x] for c in range(6)] for ip in range(r["sig"].shape[1])]
                            for x, y, z in vox])
            mo = np.array(g["macro_sigma"])
            parity[name] = {"macro_rel_err": float(np.abs(r["macro_sigma"] - mo).max() / np.abs(mo).max()),
                            "sigma_rel_L2_sampled": float(np.sqrt(np.sum((sig - gs) ** 2) / np.sum(gs ** 2)))}
        log(f"parity vs oracle: {parity}")

    batch = None
    if not args.no_batch:
        batch = batch_sample(B, W, log=log)
        log(f"batch: {batch['solves']} solves, FP32 batch {batch['fp32_batch_voxel_iter_s']:.3e} voxel-iter/s "
            f"({batch['fp32_batch_s']:.2f} s), FP64 one at a time {batch['fp64_one_at_a_time_voxel_iter_s']:.3e} "
            f"({batch['fp64_one_at_a_time_s']:.2f} s), max macro diff {batch['max_macro_rel_diff_fp32_vs_fp64']:.2e}")

    serving = None
    if not args.no_serving:
        serving = {}
        for name, prec in (("fp32", W.FP32_MIXED), ("fp64", W.FP64)):
            serving[name] = serving_sample(B, W, prec, log=log if args.serving_full else None)
            sv = serving[name]
            log(f"serving {name}: {sv['completed']} requests, p50 {sv['p50_latency_s']:.3f} s, "
                f"p99 {sv['p99_latency_s']:.3f} s, {sv['throughput_voxel_iter_s']:.3e} voxel-iter/s")
        if args.serving_full:
            for name, prec in (("fp32_full_range", W.FP32_MIXED), ("fp64_full_range", W.FP64)):
                serving[name] = serving_sample(B, W, prec, count=12, sizes=(32, 64, 96, 128, 160, 192), log=log)
                sv = serving[name]
                log(f"serving {name}: p50 {sv['p50_latency_s']:.3f} s, p99 {sv['p99_latency_s']:.3f} s, "
                    f"{sv['throughput_voxel_iter_s']:.3e} voxel-iter/s")
        if args.serving_sweep:
            serving["sweep"] = serving_sweep(B, W, log=log)

    cpu = None if args.no_cpu_baseline else cpu_baseline()
    out = {
        "metric": "voxel-iter/s (FP32-mixed, macro-stress parity vs FP64)",
        "value": value,
        "unit": "voxel-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 reductions, Anderson, displacement accumulator)",
        "data": "synthetic",
        "config": {"workload": f"polycrystal{args.size}: {args.size}^3 Voronoi, 500 grains, cubic "
                               "elasticity, bending, TETRA2, B0, tol 1e-6",
                   "voxels": Nv, "iterations_per_solve": iters32 / args.steps,
                   "converged": conv32},
        "roofline": roof,
        "copy_GBs": copy_gbs,
        "fp64": fp64,
        "speedup_fp32_vs_fp64": (value / fp64["value"]) if fp64 else None,
        "parity_vs_oracle": parity,
        "batch": batch,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
