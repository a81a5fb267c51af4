#!/usr/bin/env python3
"""Throughput of the 4PCF hot path on one MI355X.

Workload: 4PCF, lmax = 5, 10 linear radial bins over [20, 160] Mpc/h, on a
synthetic data-minus-randoms catalog -- 200,000 Neyman-Scott clustered points
plus 600,000 uniform randoms weighted -N_D/N_R -- in a periodic 1000 Mpc/h box:
800,000 primaries, ~13,700 neighbours each.

One step = the whole hot path on device-resident inputs: cell-grid build (with
the D-R weighting) + harmonic-coefficient gather + coupling + FP64 sum over
primaries + contraction to zeta, ending with zeta on the host.  The default path
is FP32 harmonic coefficients with the split-bf16 matrix-core coupling; the plain
FP64 path is timed in the same run and the two results are compared.

Besides the JSON fields of the step, the line carries: the roofline of the
dominant kernel (the gather, ALU-bound), the matrix-core figures of the coupling,
the FP64 oracle on the host cores, a batched leg (uneven catalogs in one
persistent launch) and a served leg (Poisson arrivals, p50/p99 latency).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "4PCF primaries/s (ℓmax=5, 10 bins) vs plain FP64 path; p50/p99 job latency"
PEAK_ALU_TFLOPS = 78.6    # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz, non-packed VALU (FP32 or FP64)
PEAK_BF16_TFLOPS = 2500.0  # dense bf16 matrix cores


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def gather_flops_per_pair(L):
    """Algorithmic flops of one accepted pair in the gather (counted from the method):
    separation + r^2 in FP64 (8), unit vector (r^2, rsqrt, 3 mul: 9), (x+iy)^m for
    m = 2..L (6 per complex product), Legendre recurrence (3 per entry with l >= m+2,
    plus z*w), accumulation of w Y (1 per m = 0 entry, 4 per complex entry)."""
    f = 8 + 9 + 6 * max(L - 1, 0) + 1
    f += 3 * sum(max(L - m - 1, 0) for m in range(L + 1))
    f += (L + 1) + 4 * sum(L - m + 1 for m in range(1, L + 1))
    return f


def gather_traffic(pairs):
    """HBM bytes per gather launch from the committed counter summary, or None when
    the gather source has changed since the counters were taken."""
    import hashlib
    src = os.path.join(ROOT, "paper_2105_08722_amd", "csrc", "gather.hip")
    summ = os.path.join(ROOT, "profiles", "k_gather_traffic.json")
    if not os.path.exists(summ):
        return None
    rec = json.load(open(summ))
    if rec.get("gather_source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    if rec.get("pairs_per_launch") != pairs:
        return None
    return rec["hbm_bytes_per_launch"]


def cpu_baseline(cfg, target_s):
    """The FP64 oracle on the host cores, over a seeded sample of primaries (all
    800k points stay secondaries)."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    w = oracle.dmr_weights(cfg["w"][:cfg["n_data"]], cfg["w"][cfg["n_data"]:])
    n = len(w)
    rng = np.random.default_rng(99)
    cores = os.cpu_count() or 1
    probe = rng.choice(n, 16 * cores, replace=False)
    t0 = time.perf_counter()
    oracle.zeta(cfg["pos"], w, 4, 5, cfg["edges"], box=cfg["box"], primaries=probe, nthreads=cores)
    dt = time.perf_counter() - t0
    k = int(min(20000, max(len(probe), target_s * len(probe) / max(dt, 1e-3))))
    sample = rng.choice(n, k, replace=False)
    log("cpu baseline: oracle over %d sampled primaries on %d threads" % (k, cores))
    t0 = time.perf_counter()
    oracle.zeta(cfg["pos"], w, 4, 5, cfg["edges"], box=cfg["box"], primaries=sample, nthreads=cores)
    dt = time.perf_counter() - t0
    return {"value": k / dt, "unit": "primaries/s", "cores": cores, "kind": "oracle",
            "sample": "%d seeded primaries of the 800k-point catalog, all 800k points as "
                      "secondaries, FP64 C oracle (full M sum), %.1f s" % (k, dt)}


def batched_leg(ctx, edges, precision, njobs, seed=4000):
    """Uneven mock catalogs (N_D ~ U[50k, 400k] Neyman-Scott data + 3 N_D randoms each,
    periodic 1000 Mpc/h) in one encore_npcf_batch call (one persistent gather launch
    per slice over all catalogs)."""
    from paper_2105_08722_amd import encore, synth
    sizes = synth.batch_sizes(njobs, seed)
    grids = []
    tot = 0
    try:
        for k, nd in enumerate(sizes):
            pos, w = synth.mock_dmr_catalog(int(nd), 1000.0, seed + k)
            grids.append(encore.build_grid(ctx, pos, w, r_max=edges[-1], box=1000.0, n_data=int(nd)))
            tot += len(w)
        encore.npcf_batch(ctx, grids[:2], 4, 5, edges, precision=precision)   # warm
        t0 = time.perf_counter()
        encore.npcf_batch(ctx, grids, 4, 5, edges, precision=precision)
        dt = time.perf_counter() - t0
    finally:
        for g in grids:
            g.free()
    return {"value": tot / dt, "unit": "primaries/s", "jobs": njobs, "primaries": int(tot),
            "seconds": dt, "precision": precision,
            "workload": "%d Neyman-Scott D-R catalogs, N_D ~ U[50k, 400k] + 3 N_D randoms, periodic "
                        "1000 Mpc/h, 4PCF lmax=5, 10 bins, one batched call (grids prebuilt)" % njobs}


def served_leg(ctx, edges, njobs, rate, seed=5000):
    """Poisson request stream (mean `rate` jobs/s) mixing 3PCF lmax=10 (FP32), 4PCF
    lmax=5 and 5PCF lmax=4 (split-bf16) jobs on Neyman-Scott D-R catalogs of
    log-uniform size; latency = arrival (submit) to result ready."""
    import numpy as np
    from paper_2105_08722_amd import encore, synth
    rng = np.random.default_rng(seed)
    kinds = [(3, 10, "fp32"), (4, 5, "splitbf16"), (5, 4, "splitbf16")]
    jobs = []
    for k in range(njobs):
        N, L, prec = kinds[int(rng.integers(0, 3))]
        ntot = int(np.exp(rng.uniform(np.log(1e4), np.log(1e6))))
        nd = max(ntot // 4, 1)
        pos, w = synth.mock_dmr_catalog(nd, 1000.0, seed + 13 * k)
        jobs.append((N, L, prec, pos, w, nd))
    gaps = rng.exponential(1.0 / rate, size=njobs)
    ids = [None] * njobs
    with encore.Server(ctx, hbm_budget=64 << 30, n_lanes=3, max_active=16, slice_rows=262144) as srv:
        def feed():
            for k, (N, L, prec, pos, w, nd) in enumerate(jobs):
                time.sleep(float(gaps[k]))
                ids[k] = srv.submit(pos, w, N, L, edges, box=1000.0, n_data=nd, precision=prec)

        t0 = time.perf_counter()
        th = threading.Thread(target=feed)
        th.start()
        th.join()
        lat = []
        for k in range(njobs):
            _, t = srv.wait(ids[k])
            lat.append(t["done"] - t["submit"])
        dt = time.perf_counter() - t0
        st = srv.stats()
    lat = np.array(lat)
    return {"jobs": njobs, "rate_jobs_per_s": rate, "jobs_per_s": njobs / dt,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()), "primaries_run": st["primaries_run"],
            "peak_bytes_held": st["peak_bytes_held"],
            "workload": "Poisson arrivals (mean %.1f jobs/s), jobs uniform over {3PCF lmax=10 fp32, "
                        "4PCF lmax=5 split-bf16, 5PCF lmax=4 split-bf16}, 1e4-1e6 points "
                        "(log-uniform, 1:3 data:randoms, Neyman-Scott D-R, periodic 1000 Mpc/h), "
                        "10 bins [20,160]; 3 lanes" % rate}


def splits_leg(ctx, edges, precision, nparts, seed=6000):
    """Random-split co-adding (Section 4.2): 200k Neyman-Scott data and random parts
    of 1.5 N_D uniform points each, 4PCF lmax=5, in two regimes: the benchmark's
    density (periodic 1000 Mpc/h, nparts parts, the bench precision) and 8x that
    density (500 Mpc/h, 4 parts, FP64: the precision in which the data part is kept).  One encore_npcf_splits call (the data part of a~ gathered once; per
    part, data primaries against the part's randoms only) against one
    encore_npcf_batch call over the same D + R_k catalogs (every pair of every part
    gathered)."""
    import numpy as np
    from paper_2105_08722_amd import encore, synth
    out = {}
    for name, box, K, prec in (("box1000", 1000.0, nparts, precision), ("box500_fp64", 500.0, 4, "fp64")):
        nd = 200_000
        nr = 3 * nd // 2
        dpos, dw = synth.neyman_scott(nd, box, seed)
        rpos, rw = synth.uniform_box(K * nr, box, seed + 7919)
        gd, gs = encore.build_split_grids(ctx, dpos, dw, rpos, rw, [nr] * K, edges[-1], box=box)
        try:
            encore.npcf_splits(ctx, gd, gs, 4, 5, edges, precision=prec)   # warm; builds the randoms-only grids
            t0 = time.perf_counter()
            zs = encore.npcf_splits(ctx, gd, gs, 4, 5, edges, precision=prec)
            t_split = time.perf_counter() - t0
            tm_s = ctx.last_timings()
            encore.npcf_batch(ctx, gs, 4, 5, edges, precision=prec)   # warm
            t0 = time.perf_counter()
            zb = encore.npcf_batch(ctx, gs, 4, 5, edges, precision=prec)
            t_batch = time.perf_counter() - t0
            tm_b = ctx.last_timings()
        finally:
            for g in gs:
                g.free()
            gd.free()
        zm = zb.mean(axis=0)
        prim = K * (nd + nr)
        out[name] = {"parts": K, "n_data": nd, "randoms_per_part": nr, "precision": prec,
                     "coadded_s": t_split, "batch_s": t_batch, "speedup": t_batch / t_split,
                     "primaries_per_s": prim / t_split, "primaries_per_s_batch": prim / t_batch,
                     "pairs_coadded": tm_s["pairs"], "pairs_batch": tm_b["pairs"],
                     "data_part_kept": bool(tm_s["pairs"] < tm_b["pairs"]),
                     "gather_ms": tm_s["gather_ms"], "gather_ms_batch": tm_b["gather_ms"],
                     "max_rel_diff_vs_batch": float(np.max(np.abs(zs - zm)) / np.max(np.abs(zm))),
                     "workload": "200k Neyman-Scott data + %d random parts of 300k uniform points (D-R per "
                                 "part), periodic %g Mpc/h, 4PCF lmax=5, 10 bins, grids prebuilt" % (K, box)}
    return out


def mfma_figures(N, L, nbins, nprim, couple_ms):
    """Matrix-core figures of a split-bf16 coupling from the plan: MFMA flops issued
    (three 16x16x32 bf16 MFMAs per output tile per 16 primaries) and useful flops
    (4 per T entry per primary: the real part of a complex product)."""
    from paper_2105_08722_amd import encore
    st = encore.mfma_plan_stats(N, L, nbins)
    raw = st["tiles_per_16"] * 3 * 16 * 16 * 32 * 2 / 16.0 * nprim
    useful = 4.0 * st["t_entries"] * nprim
    sec = couple_ms * 1e-3
    return {"issued_tflops": raw / sec / 1e12, "issued_frac": raw / sec / 1e12 / PEAK_BF16_TFLOPS,
            "useful_tflops": useful / sec / 1e12,
            "useful_frac_of_split_peak": useful / sec / 1e12 / (PEAK_BF16_TFLOPS / 3.0),
            "tiles_per_16_primaries": st["tiles_per_16"], "t_entries_per_primary": st["t_entries"]}


def config1_leg(ctx):
    """The 3PCF workload: 2000 uniform points, periodic 500 Mpc/h, lmax=10, 10 bins
    [20,160], plain FP64 path, every point a primary (grid build included)."""
    from paper_2105_08722_amd import encore, synth
    cfg = synth.config(1)
    def run():
        with encore.build_grid(ctx, cfg["pos"], cfg["w"], r_max=160.0, box=cfg["box"]) as g:
            return encore.npcf(ctx, g, 3, 10, cfg["edges"], precision="fp64")
    run()
    t0 = time.perf_counter()
    run()
    dt = time.perf_counter() - t0
    tm = ctx.last_timings()
    return {"value": 2000 / dt, "unit": "primaries/s", "seconds": dt, "gather_ms": tm["gather_ms"],
            "couple_ms": tm["couple_ms"], "precision": "fp64", "workload": cfg["name"]}


def config3_leg(ctx, precision, tune=True, n6=200_000):
    """The survey-wedge workload (500k clustered data + 1.5M randoms, non-periodic
    wedge with holes, FKP weights, D-R): the 5PCF at lmax=4 over all 2M primaries and
    the 6PCF at lmax=3 over a seeded subset of n6 primaries (all 2M points are
    secondaries), with the coupling's matrix-core figures."""
    import numpy as np
    from paper_2105_08722_amd import encore, synth
    cfg = synth.config(3)
    n = len(cfg["w"])
    out = {}
    # the library's autotuner on this catalog (10x the benchmark's density: finer
    # cells and fewer bins per item win), before the grid is built with its choice;
    # the 6PCF keeps its default bins per item (the tuner's sample, runs of
    # cell-sorted primaries, does not represent a random subset of primaries)
    if tune:
        t0 = time.perf_counter()
        tuned = encore.autotune(ctx, cfg["pos"], cfg["w"], 5, 4, cfg["edges"], n_data=cfg["n_data"],
                                precision=precision, n_sample=131072)
        tuned["tuning_s"] = time.perf_counter() - t0
        out["autotune_5pcf"] = tuned
    with encore.build_grid(ctx, cfg["pos"], cfg["w"], r_max=160.0, n_data=cfg["n_data"]) as g:
        for N, L, prim in [(5, 4, None), (6, 3, np.random.default_rng(6).choice(n, n6, replace=False))]:
            k = n if prim is None else len(prim)
            encore.npcf(ctx, g, N, L, cfg["edges"], precision=precision, primaries=prim[:4096] if prim is not None else np.arange(4096))
            t0 = time.perf_counter()
            encore.npcf(ctx, g, N, L, cfg["edges"], precision=precision, primaries=prim)
            dt = time.perf_counter() - t0
            tm = ctx.last_timings()
            rec = {"value": k / dt, "unit": "primaries/s", "primaries": k, "seconds": dt,
                   "gather_ms": tm["gather_ms"], "couple_ms": tm["couple_ms"], "precision": precision}
            if precision == "splitbf16":
                rec["coupling_mfma"] = mfma_figures(N, L, len(cfg["edges"]) - 1, k, tm["couple_ms"])
            out["%dpcf_lmax%d" % (N, L)] = rec
    out["workload"] = cfg["name"] + "; 5PCF lmax=4 over all primaries, 6PCF lmax=3 over %d seeded primaries" % n6
    return out


def mesh_leg(ctx, edges, precision, n=128, box=1000.0):
    """Gridded data (Section 3.2): a clustered overdensity field (200k Neyman-Scott
    points counted on a periodic n^3 mesh of the 1000 Mpc/h box, delta = rho/mean - 1,
    so every cell is a primary), 4PCF lmax=5, 10 bins, through encore_npcf_mesh.  The
    field stage (kernel fields, forward and inverse FP64 transforms, products) is
    bounded by HBM.  `value` is a call with the shape of the previous call (the
    kernel-field transforms reused, as for many fields on one mesh); `first_call`
    is the same call with the kernel fields built and transformed."""
    import torch
    from paper_2105_08722_amd import encore, synth
    delta = torch.from_numpy(synth.mesh_overdensity(n, box, 200_000, 7001)).to("cuda:0")
    # untimed: the transform library compiles its kernels for this length on first
    # use (done on other edges, so that the timed first call below builds and
    # transforms its own kernel fields)
    encore.npcf_mesh(ctx, delta, box, 4, 5, edges * 0.999, precision=precision)
    runs = []
    for _ in range(2):   # first call of the shape, then a call reusing its kernel transforms
        t0 = time.perf_counter()
        encore.npcf_mesh(ctx, delta, box, 4, 5, edges, precision=precision)
        runs.append((time.perf_counter() - t0, ctx.last_timings()))
    (dt0, tm0), (dt, tm) = runs
    nf = (len(edges) - 1) * 21
    # passes over the nf fields of n^3 complex FP64 values: first call 7 (kernel
    # fill; read + write of the forward transform, the product and the inverse
    # transform), a call reusing the kernel transforms 4 (product, inverse)
    full_bytes = 7.0 * nf * n ** 3 * 16
    field_bytes = 4.0 * nf * n ** 3 * 16
    def roof(b, ms):
        return {"bound": "hbm", "unit": "GB/s", "peak": 8000.0, "algorithmic_bytes": b,
                "achieved": b / (ms * 1e-3) / 1e9, "frac": b / (ms * 1e-3) / 1e9 / 8000.0}
    return {"value": n ** 3 / dt, "unit": "cells/s", "seconds": dt, "nmesh": n, "cells": n ** 3,
            "precision": precision, "field_stage_ms": tm["gather_ms"], "coupling_ms": tm["couple_ms"],
            "kernel_transforms_reused": bool(tm["pairs"]),
            "field_stage_roofline": roof(field_bytes, tm["gather_ms"]),
            "first_call": {"value": n ** 3 / dt0, "unit": "cells/s", "seconds": dt0,
                           "kernel_transforms_reused": bool(tm0["pairs"]),
                           "field_stage_ms": tm0["gather_ms"], "coupling_ms": tm0["couple_ms"],
                           "field_stage_roofline": roof(full_bytes, tm0["gather_ms"])},
            "workload": "gridded 4PCF lmax=5, 10 bins [20,160], %d^3 mesh of a periodic %g Mpc/h box "
                        "(Neyman-Scott overdensity, every cell a primary)" % (n, box)}


def edge_leg(ctx):
    """Edge correction of the paper's analyses (Section 5.4): 4PCF measured at
    lmax = 6 for output lmax = 5, 5PCF measured at lmax = 4 for output lmax = 3, and
    the survey workload's 6PCF at lmax = 3 for output lmax = 2, 10 radial bins;
    synthetic window multiplets (R_0 dominant, per-cent higher multiplets) and data
    multiplets.  Device time from HIP events around the two kernels; the first call
    also builds the Gaunt-integral table on the host (seconds for the 6PCF)."""
    import numpy as np
    from paper_2105_08722_amd import encore
    out = {}
    for N, lm in [(4, 6), (5, 4), (6, 3)]:
        n = encore.num_multiplets(N, lm)
        nB = encore.num_bin_tuples(N, 10)
        rng = np.random.default_rng(77 + N)
        R = rng.normal(0.0, 0.03, (n, nB))
        R[0] = rng.uniform(1.0, 3.0, nB)
        Nm = rng.normal(size=(n, nB))
        t0 = time.perf_counter()
        encore.edge_correct(ctx, N, lm, 10, Nm, R, lmax_out=lm - 1)
        first = time.perf_counter() - t0
        t0 = time.perf_counter()
        z = encore.edge_correct(ctx, N, lm, 10, Nm, R, lmax_out=lm - 1)
        call = time.perf_counter() - t0
        dev_ms = float(ctx.last_timings()["total_ms"])
        flops = nB * (2.0 * n ** 3 / 3.0 + 2.0 * n * n)   # elimination + back substitution
        stream = nB * 16.0 * n ** 3 / (3.0 * 32)            # trailing matrix read + written once per 32-column panel
        out["%dpcf" % N] = {"lmax_measured": lm, "lmax_out": lm - 1, "multiplets": n,
                            "multiplets_out": int(z.shape[0]), "bin_tuples": nB,
                            "device_ms": dev_ms, "call_ms": call * 1e3, "first_call_s": first,
                            "solve_gflops": flops / max(dev_ms, 1e-9) / 1e6,
                            "trailing_stream_gb_s": stream / max(dev_ms, 1e-9) / 1e6}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="splitbf16", choices=["fp32", "fp64", "splitbf16"])
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-edge", action="store_true", help="skip the edge-correction leg")
    ap.add_argument("--no-mesh", action="store_true", help="skip the gridded-data leg")
    ap.add_argument("--no-configs", action="store_true", help="skip the 3PCF (config 1) and survey-wedge legs")
    ap.add_argument("--split-parts", type=int, default=8, help="random parts of the co-adding leg (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--batched-jobs", type=int, default=64, help="0: skip the batched leg")
    ap.add_argument("--served-jobs", type=int, default=256, help="0: skip the served leg")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of MIB MiB (the reference "
                         "dispatch for scaling FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(primaries would shard across GPUs with one FP64 all-reduce of zeta).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2105_08722_amd import encore, synth

    log("generating the synthetic catalog")
    cfg = synth.config(2)
    n = len(cfg["w"])
    N, L, edges = 4, 5, cfg["edges"]
    dev = torch.device("cuda:0")
    tp = torch.from_numpy(cfg["pos"]).to(dev)
    tw = torch.from_numpy(cfg["w"]).to(dev)
    torch.cuda.synchronize()
    if args.calibrate_copy > 0:
        src = torch.empty(args.calibrate_copy << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: %d MiB read + %d MiB written" % (args.calibrate_copy, args.calibrate_copy))
        del src, dst
    ctx = encore.Context(0)
    tuned = None
    if not args.no_tune:
        t0 = time.perf_counter()
        tuned = encore.autotune(ctx, cfg["pos"], cfg["w"], N, L, edges, box=cfg["box"],
                                n_data=cfg["n_data"], precision=args.precision, n_sample=131072)
        tuned["tuning_s"] = time.perf_counter() - t0
        log("autotune: %s" % tuned)

    def step(prec):
        g = encore.build_grid_device(ctx, tp, tw, r_max=edges[-1], box=cfg["box"], n_data=cfg["n_data"])
        z = encore.npcf(ctx, g, N, L, edges, precision=prec)
        g.free()
        return z, ctx.last_timings()

    for i in range(args.warmup):
        step(args.precision)
        log("warmup %d/%d done" % (i + 1, args.warmup))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gather_ms = couple_ms = 0.0
    pairs = 0
    z = None
    for i in range(args.steps):
        z, tm = step(args.precision)
        gather_ms += tm["gather_ms"]
        couple_ms += tm["couple_ms"]
        pairs = tm["pairs"]
        log("step %d/%d: %.1f ms (gather %.1f, couple %.1f)" % (i + 1, args.steps, tm["total_ms"],
                                                               tm["gather_ms"], tm["couple_ms"]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    value = n / (ms / 1e3)
    g_ms = gather_ms / args.steps
    c_ms = couple_ms / args.steps
    flops = gather_flops_per_pair(L) * pairs
    achieved = flops / (g_ms * 1e-3) / 1e12
    nbg = tuned["bins_per_item"] if tuned else 2
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_ALU_TFLOPS, "traffic": gather_traffic(pairs),
                "kernel": "k_gather<float,5,%d,0,5,false,false> (harmonic-coefficient gather)" % nbg,
                "launch_ms": g_ms, "pairs_per_launch": pairs,
                "flops_per_pair": gather_flops_per_pair(L)}

    extra = {}
    if args.precision == "splitbf16":
        ms_ = encore.mfma_plan_stats(N, L, len(edges) - 1)
        raw = ms_["tiles_per_16"] * 3 * 16 * 16 * 32 * 2 / 16.0 * n      # MFMA flops issued per step
        useful = 4.0 * ms_["t_entries"] * n                               # real triple products x (re, im) x FMA
        extra["coupling_mfma"] = {
            "bound": "mfma", "unit": "TFLOP/s", "peak": PEAK_BF16_TFLOPS, "coupling_ms": c_ms,
            "issued": raw / (c_ms * 1e-3) / 1e12, "issued_frac": raw / (c_ms * 1e-3) / 1e12 / PEAK_BF16_TFLOPS,
            "useful": useful / (c_ms * 1e-3) / 1e12,
            "useful_frac_of_split_peak": useful / (c_ms * 1e-3) / 1e12 / (PEAK_BF16_TFLOPS / 3.0),
            "tiles_per_16_primaries": ms_["tiles_per_16"], "t_entries_per_primary": ms_["t_entries"]}
    if not args.no_fp64 and args.precision != "fp64":
        log("plain FP64 path, one step")
        step("fp64")
        t2 = time.perf_counter()
        z64, tm64 = step("fp64")
        t3 = time.perf_counter()
        num = np.linalg.norm(z - z64, axis=1)
        den = np.linalg.norm(z64, axis=1)
        keep = den > 0
        extra["fp64_path"] = {"value": n / (t3 - t2), "unit": "primaries/s", "ms_per_step": (t3 - t2) * 1e3,
                              "gather_ms": tm64["gather_ms"], "couple_ms": tm64["couple_ms"]}
        extra["speedup_vs_fp64_path"] = extra["fp64_path"]["ms_per_step"] / ms
        extra["accuracy_vs_fp64_path"] = {"max_e_lambda": float(np.max(num[keep] / den[keep])),
                                          "median_e_lambda": float(np.median(num[keep] / den[keep]))}
        if args.precision != "fp32":
            # the plain FP32 path (FP32 terms summed in FP64, FP32 VALU coupling)
            log("FP32 path, one step")
            step("fp32")
            t2 = time.perf_counter()
            z32, tm32 = step("fp32")
            t3 = time.perf_counter()
            e32 = np.linalg.norm(z32 - z64, axis=1)[keep] / den[keep]
            extra["fp32_path"] = {"value": n / (t3 - t2), "unit": "primaries/s", "ms_per_step": (t3 - t2) * 1e3,
                                  "gather_ms": tm32["gather_ms"], "couple_ms": tm32["couple_ms"],
                                  "max_e_lambda_vs_fp64_path": float(np.max(e32)),
                                  "median_e_lambda_vs_fp64_path": float(np.median(e32))}
    if args.batched_jobs > 0:
        log("batched leg: %d catalogs" % args.batched_jobs)
        extra["batched"] = batched_leg(ctx, edges, args.precision, args.batched_jobs)
        log("batched: %.3g primaries/s" % extra["batched"]["value"])
    if args.served_jobs > 0:
        log("served leg: %d jobs" % args.served_jobs)
        extra["served"] = served_leg(ctx, edges, args.served_jobs, 4.0)
        log("served: p50 %.2f s, p99 %.2f s" % (extra["served"]["p50_latency_s"],
                                                 extra["served"]["p99_latency_s"]))
    if args.split_parts > 0:
        log("random-split co-adding leg: %d parts" % args.split_parts)
        extra["random_splits"] = splits_leg(ctx, edges, args.precision, args.split_parts)
        log("random splits: %s" % ", ".join("%s co-added %.3f s vs batch %.3f s" % (k, v["coadded_s"], v["batch_s"])
                                              for k, v in extra["random_splits"].items()))
    if not args.no_configs:
        log("3PCF leg")
        extra["config1_3pcf"] = config1_leg(ctx)
        log("3PCF: %.3g primaries/s" % extra["config1_3pcf"]["value"])
        log("survey-wedge leg")
        extra["config3_wedge"] = config3_leg(ctx, args.precision, tune=not args.no_tune)
        log("wedge: 5PCF %.3g primaries/s, 6PCF %.3g primaries/s"
            % (extra["config3_wedge"]["5pcf_lmax4"]["value"], extra["config3_wedge"]["6pcf_lmax3"]["value"]))
    if not args.no_mesh:
        log("gridded-data leg")
        extra["gridded"] = mesh_leg(ctx, edges, args.precision)
        log("gridded: %.1f ms (fields %.1f ms, %.0f GB/s; coupling %.1f ms)"
            % (extra["gridded"]["seconds"] * 1e3, extra["gridded"]["field_stage_ms"],
               extra["gridded"]["field_stage_roofline"]["achieved"], extra["gridded"]["coupling_ms"]))
    if not args.no_edge:
        log("edge-correction leg")
        extra["edge_correction"] = edge_leg(ctx)
        log("edge correction: %s" % ", ".join("%s %.2f ms" % (k, v["device_ms"])
                                                for k, v in extra["edge_correction"].items()))
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, args.cpu_seconds)
    ctx.close()

    out = {
        "metric": METRIC, "value": value, "unit": "primaries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "splitbf16": "f32+bf16x3"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "4PCF lmax=5, 10 bins [20,160] Mpc/h, Neyman-Scott 200k data + "
                               "600k uniform randoms (D-R), periodic 1000 Mpc/h box",
                   "N": N, "lmax": L, "nbins": 10, "primaries": n, "precision": args.precision,
                   "gather_ms": g_ms, "couple_ms": c_ms, "pairs": pairs, "autotune": tuned},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
