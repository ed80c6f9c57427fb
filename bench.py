#!/usr/bin/env python3
"""Benchmark: filtered lookups/s on one MI355X, stochastic vs deterministic
tricubic B-spline filtering of a sparse voxel grid.

Workload: a 512^3 sparse grid of dense 8^3 FP32 leaves holding thresholded
5-octave fBm value noise (about 6% of the leaves active), queried at
16,777,216 positions along 65,536 random rays (256 samples per ray, ray-major
order).  One step = one stf_filter call over the whole batch, inputs already
resident in HBM.  The headline value is stochastic tricubic lookups/s; the
deterministic 64-tap filter and the trilinear pair are timed beside it, on the
same inputs.  The FP64 CPU oracle checks sampled outputs of every timed
configuration and is timed on a bounded sample of the same workload
(cpu_baseline).

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "filtered lookups/s, stochastic vs deterministic tricubic, at stated error; p99 batch latency"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_launches(fn, steps, warmup, torch):
    """Warm up, then time `steps` calls: wall clock between two device
    synchronisations, and per-call HIP events on the launch stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = np.array([a.elapsed_time(b) for a, b in ev])
    return wall, kern_ms


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fmt", default="f32", choices=["f32", "f16", "bf16", "fp8_e4m3"])
    ap.add_argument("--order", default="ray", choices=["ray", "shuffled"])
    ap.add_argument("--cpu-sample", type=int, default=1 << 24, help="queries in the CPU-oracle timing sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle timing")
    ap.add_argument("--only", default="", help="time only this variant (e.g. stoch_cubic)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2305_05810_amd as stf
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    dims = (512, 512, 512)
    t0 = time.time()
    grid = synth.fbm_grid(dims, seed=3)
    pts = synth.ray_queries(dims, n_rays=65536, samples_per_ray=256, seed=4, shuffle=args.order == "shuffled")
    n = pts.shape[0]
    log(f"inputs: {grid.n_leaves} leaves ({100 * grid.occupancy():.2f}% of slots), {n} queries, "
        f"{time.time() - t0:.1f}s")
    raw = grid.encoded(args.fmt)
    tex = stf.stf_create_sparse_grid3d(dims, stf.FORMATS[args.fmt], grid.origins, raw)
    q = torch.from_numpy(pts).to(dev)
    out = torch.empty((n, 1), dtype=torch.float32, device=dev)
    texel_b = stf.FORMAT_BYTES[stf.FORMATS[args.fmt]]

    variants = [("stoch_cubic", stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 64),
                ("det_cubic", stf.STF_CUBIC_BSPLINE, stf.STF_DETERMINISTIC, 64),
                ("stoch_linear", stf.STF_LINEAR, stf.STF_STOCHASTIC, 8),
                ("det_linear", stf.STF_LINEAR, stf.STF_DETERMINISTIC, 8)]
    if args.only:
        variants = [v for v in variants if v[0] == args.only]
    res = {}
    seed = 0x5EED
    for name, filt, mode, taps in variants:
        fn = lambda: stf.stf_filter(tex, q, filt, mode, seed, out)
        wall, kern = time_launches(fn, args.steps, args.warmup, torch)
        b_alg = 12 + 4 + (texel_b if mode == stf.STF_STOCHASTIC else taps * texel_b)
        kmean = float(kern.mean())
        res[name] = dict(lookups_per_s=n * args.steps / wall, ms_per_step=1e3 * wall / args.steps,
                         kernel_ms_mean=kmean, kernel_ms_p50=float(np.percentile(kern, 50)),
                         kernel_ms_p99=float(np.percentile(kern, 99)), bytes_per_lookup=b_alg,
                         achieved_gbs=b_alg * n / (kmean * 1e-3) / 1e9)
        log(f"{name}: {res[name]['lookups_per_s'] / 1e9:.2f} G lookups/s, kernel {kmean * 1e3:.1f} us, "
            f"{res[name]['achieved_gbs']:.0f} GB/s algorithmic")

    # sampled parity of every timed configuration against the FP64 oracle
    import oracle
    ofmt = {"f32": oracle.F32, "f16": oracle.F16, "bf16": oracle.BF16, "fp8_e4m3": oracle.FP8_E4M3}[args.fmt]
    og = oracle.Grid(dims, ofmt, grid.origins, raw)
    rng = np.random.default_rng(12)
    qids = np.sort(rng.choice(n, 1 << 16, replace=False))
    parity = {}
    for name, filt, mode, _ in variants:
        ofilt = oracle.CUBIC if filt == stf.STF_CUBIC_BSPLINE else oracle.LINEAR
        if mode == stf.STF_STOCHASTIC:
            idx = torch.empty((n, 3), dtype=torch.int32, device=dev)
            stf.stf_filter(tex, q, filt, mode, seed, out, idx)
            gv = out[:, 0].cpu().numpy()[qids]
            gi = idx.cpu().numpy()[qids]
            ov, oi = og.filter_at(pts, qids, ofilt, oracle.STOCH, seed)
            parity[name] = dict(sampled=int(qids.size), index_mismatches=int(np.any(gi != oi, axis=1).sum()),
                                value_mismatches=int((gv != ov.astype(np.float32)).sum()))
        else:
            stf.stf_filter(tex, q, filt, mode, seed, out)
            gv = out[:, 0].cpu().numpy()[qids].astype(np.float64)
            ov, _ = og.filter_at(pts, qids, ofilt, oracle.DET, 0)
            err = np.abs(gv - ov)
            rel = np.where(ov != 0, err / np.where(ov == 0, 1, np.abs(ov)), np.where(err == 0, 0, np.inf))
            parity[name] = dict(sampled=int(qids.size), max_rel_err=float(rel.max()),
                                within_1e6=bool(np.all(err <= 1e-6 * np.abs(ov))))
        log(f"parity {name}: {parity[name]}")

    cpu = None
    if not args.no_cpu and "stoch_cubic" in res:
        m = min(args.cpu_sample, n)
        sample = np.ascontiguousarray(pts[:m])
        threads = oracle.max_threads()
        t1 = time.perf_counter()
        og.filter(sample, oracle.CUBIC, oracle.STOCH, seed, want_index=False, nthreads=threads)
        dt = time.perf_counter() - t1
        cpu = dict(value=m / dt, unit="lookups/s", cores=threads, kind="oracle",
                   sample=f"first {m} of the {n} ray-ordered queries, stochastic tricubic, FP64 C oracle "
                          f"with OpenMP, {dt:.2f} s")
        log(f"cpu oracle: {m / dt / 1e6:.2f} M lookups/s on {threads} threads")

    head = res.get("stoch_cubic") or next(iter(res.values()))
    det = res.get("det_cubic")
    line = {
        "metric": METRIC,
        "value": head["lookups_per_s"],
        "unit": "lookups/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.fmt,
        "data": "synthetic",
        "config": {"workload": f"sparse fBm voxel grid 512^3 of dense 8^3 {args.fmt} leaves "
                               f"({grid.n_leaves} leaves), {n} {args.order}-ordered ray queries, "
                               f"stochastic tricubic B-spline (deterministic 64-tap beside it)",
                   "n_queries": n, "n_leaves": grid.n_leaves, "order": args.order},
        "p50_batch_ms": head["kernel_ms_p50"],
        "p99_batch_ms": head["kernel_ms_p99"],
        "deterministic_lookups_per_s": det["lookups_per_s"] if det else None,
        "stochastic_over_deterministic": head["lookups_per_s"] / det["lookups_per_s"] if det else None,
        "variants": res,
        "parity": parity,
        "roofline": {"bound": "hbm", "achieved": head["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["achieved_gbs"] / HBM_PEAK_GBS, "traffic": None},
        "cpu_baseline": cpu,
    }
    tex.destroy()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
