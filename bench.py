#!/usr/bin/env python3
"""Benchmark of the stochastic texture filtering library on one MI355X.

Default workload (`--workload grid`, the headline): a 512^3 sparse grid of
dense 8^3 binary32 leaves holding thresholded 5-octave fBm value noise (about
6% of the leaves active), queried at 16,777,216 positions along 65,536 random
rays (256 samples per ray, ray-major order).  One step = one stf_filter call
over the whole batch with inputs resident in HBM.  The headline value is
stochastic tricubic lookups/s; the deterministic 64-tap filter and the
trilinear pair are timed beside it on the same inputs.  The FP64 CPU oracle
checks sampled outputs of every timed configuration and is timed on the same
workload (cpu_baseline).

Other workloads (one JSON line each): `tex2d` (256^2 RGBA texture, 65,536
uv queries), `shade` (4096^2 material, 8M shading queries, three filter
orders), `neural` (4096^2 x 8 texture as a 1024^2 x 8 latent grid + MLP:
training and BF16-MFMA inference), `serving` (three resident textures,
Poisson arrivals of log-normal request sizes at 0.5 / 1 / 2 G lookups/s),
`dct` (4096^2 x 9 DCT-compressed texture set, a 4K frame of uv queries, one
decode per stochastic lookup), `gauss` (Gaussian FIS vs discrete 4x4 at sigma
0.3 / 0.5 / 0.8 on the same set and frame), `ewa` (EWA over a 4096^2 RGBA8
MIP pyramid for a frame of queries with derivatives).  The grid workload also times the interpolating cubics
(Keys, Mitchell-Netravali; positivized two-tap stochastic vs 64-tap).

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
# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by a
# plain copy, each with the sha256 (first 16 hex digits) of the kernel
# sources the counters were taken on: a figure whose sources have changed
# since is reported as null until the counters are taken again.
KERNEL_SOURCES = {
    "grid": ["filter3d.hip", "device_common.h", "interp.h", "stf_internal.h"],
    "tex2d": ["filter2d.hip", "dct_decode.h", "device_common.h", "interp.h", "stf_internal.h"],
    "ewa": ["ewa.hip", "device_common.h", "interp.h", "stf_internal.h"],
    "shade": ["shade.hip", "device_common.h", "stf_internal.h"],
    "neural": ["neural.hip", "device_common.h", "stf_internal.h"],
}
# the headline kernel (stochastic tricubic, binary32 grid, ray order)
HEADLINE_TRAFFIC = {("f32", "ray"): (378.5e6, "grid", "d6208be92b350ea6")}
# the DCT workload's stochastic bilinear kernel over the 4K frame (uv in, 9
# results out; the 12.6 MB of blocks mostly cache-resident)
DCT_STOCH_LINEAR_TRAFFIC = (412.1e6, "tex2d", "ebf1d22f40a85333")
# the EWA workload's stochastic kernel at max anisotropy 8 (24-byte records
# in, 16-byte results out, one texel of the pyramid per lookup)
EWA_STOCH_TRAFFIC = (536.6e6, "ewa", "f3c297209a2c17c9")
# the Gaussian workload's FIS draw at sigma 0.5 on the DCT set (uv in, 9
# results out, block lines mostly cache-resident)
GAUSS_FIS_TRAFFIC = (416.4e6, "tex2d", "ebf1d22f40a85333")
# the shading workload's filter-after-shade kernel (36-byte records, 16 taps
# of the tiled material gathered per query, RGB out)
SHADE_FAS_TRAFFIC = (3613.7e6, "shade", "2aeefab2f9320123")
# the small 2D workload's stochastic bicubic (the 1 MiB texture fetched into
# each XCD's L2 as its lookups touch it)
TEX2D_STOCH_CUBIC_TRAFFIC = (6.91e6, "tex2d", "ebf1d22f40a85333")
# the neural workload's deterministic bicubic decode (latent quads through the
# caches, 8 channels out)
NEURAL_DET_CUBIC_TRAFFIC = (5780.0e6, "neural", "afa71d1e5c1dbf5d")


def sources_sha(kind):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_2305_05810_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(entry):
    """The recorded traffic of a kernel, or None if its sources changed since."""
    if entry is None:
        return None
    nbytes, kind, sha = entry
    if sources_sha(kind) != sha:
        log(f"traffic figure not reported: the {kind} kernel sources changed since the counters were taken")
        return None
    return nbytes
MFMA_BF16_PEAK_TFLOPS = 2500.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
METRIC = "filtered lookups/s, stochastic vs deterministic tricubic, at stated error; p99 batch latency"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_launches(fn, steps, warmup, torch):
    """Warm up, then time `steps` calls: wall clock between two device
    synchronisations, and per-call HIP events on the launch stream (torch's
    current stream, which the library launches on)."""
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


def cpu_model():
    """The host CPU's model name (Linux), or the platform's processor string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or None


def base_line(args, value, unit, ms_per_step, dtype, config, higher=True):
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": higher, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def variant_stats(n, steps, wall, kern, b_alg):
    kmean = float(kern.mean())
    return dict(lookups_per_s=n * steps / wall, ms_per_step=1e3 * wall / steps, kernel_ms_mean=kmean,
                kernel_ms_p50=float(np.percentile(kern, 50)), kernel_ms_p99=float(np.percentile(kern, 99)),
                bytes_per_lookup=b_alg, achieved_gbs=b_alg * n / (kmean * 1e-3) / 1e9)


# ----------------------------------------------------------------------------
# headline: sparse grid
# ----------------------------------------------------------------------------
STREAMS = {"ray": "ray-ordered ray queries", "shuffled": "shuffled ray queries",
           "morton": "ray queries Morton-sorted by the library (sort timed apart)",
           "medium": "ray samples inside the medium (taps meet a stored leaf)",
           "medium-morton": "ray samples inside the medium, Morton-sorted by the library (sort timed apart)"}


def run_grid(args, torch, stf, synth):
    dev = torch.device("cuda:0")
    dims = (512, 512, 512)
    t0 = time.time()
    grid = synth.fbm_grid(dims, seed=3)
    if args.order.startswith("medium"):   # ray samples whose taps meet a stored leaf
        pts = synth.medium_ray_queries(grid, 1 << 24, seed=4)
    else:
        pts = synth.ray_queries(dims, n_rays=65536, samples_per_ray=256, seed=4, shuffle=args.order == "shuffled")
    n = pts.shape[0]
    log(f"inputs: {grid.n_leaves} leaves ({100 * grid.occupancy():.2f}% of slots), {n} queries, "
        f"{time.time() - t0:.1f}s")
    raw = grid.encoded(args.fmt)
    tex = stf.stf_create_sparse_grid3d(dims, stf.FORMATS[args.fmt], grid.origins, raw)
    q = torch.from_numpy(pts).to(dev)
    out = torch.empty((n, 1), dtype=torch.float32, device=dev)
    sort_info = None
    call = lambda filt, mode, seed_, o, idx=None: stf.stf_filter(tex, q, filt, mode, seed_, o, idx)
    if args.order.endswith("morton"):
        # the library's Morton sort of the batch, timed on its own;
        # filtering then runs on the sorted stream (results in sorted order)
        sq = torch.empty_like(q)
        order = torch.empty(n, dtype=torch.int32, device=dev)
        ws = torch.empty(stf.stf_sort_workspace_bytes(n), dtype=torch.uint8, device=dev)
        wall, kern = time_launches(lambda: stf.stf_sort_queries(tex, q, sq, order, ws), args.steps, args.warmup,
                                   torch)
        sort_info = {"sort_ms": 1e3 * wall / args.steps}
        log(f"morton sort of {n} queries: {sort_info['sort_ms']:.3f} ms")
        call = lambda filt, mode, seed_, o, idx=None: stf.stf_filter_ordered(tex, sq, order, filt, mode, seed_, o, idx)
    texel_b = stf.FORMAT_BYTES[stf.FORMATS[args.fmt]]
    variants = [("stoch_cubic", stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 64),
                ("det_cubic", stf.STF_CUBIC_BSPLINE, stf.STF_DETERMINISTIC, 64),
                ("stoch_linear", stf.STF_LINEAR, stf.STF_STOCHASTIC, 8),
                ("det_linear", stf.STF_LINEAR, stf.STF_DETERMINISTIC, 8),
                ("stoch_keys", stf.STF_CUBIC_KEYS, stf.STF_STOCHASTIC, 64),
                ("det_keys", stf.STF_CUBIC_KEYS, stf.STF_DETERMINISTIC, 64),
                ("stoch_mitchell", stf.STF_CUBIC_MITCHELL, stf.STF_STOCHASTIC, 64),
                ("det_mitchell", stf.STF_CUBIC_MITCHELL, stf.STF_DETERMINISTIC, 64)]
    if args.only:
        variants = [v for v in variants if v[0] == args.only]
    res = {}
    seed = 0x5EED
    for name, filt, mode, taps in variants:
        fn = lambda: call(filt, mode, seed, out)
        wall, kern = time_launches(fn, args.steps, args.warmup, torch)
        # stochastic: one texel, two for the positivized interpolating cubics
        drawn = 2 if filt in stf.POSITIVIZED_FILTERS else 1
        b_alg = 12 + 4 + (drawn * texel_b if mode == stf.STF_STOCHASTIC else taps * texel_b)
        res[name] = variant_stats(n, args.steps, wall, kern, b_alg)
        if sort_info is not None:   # the sort and this filter, back to back
            res[name]["end_to_end_ms_with_sort"] = sort_info["sort_ms"] + res[name]["ms_per_step"]
        log(f"{name}: {res[name]['lookups_per_s'] / 1e9:.2f} G lookups/s, kernel "
            f"{res[name]['kernel_ms_mean'] * 1e3:.1f} us, {res[name]['achieved_gbs']:.0f} GB/s algorithmic")

    parity, cpu, quant = {}, None, {}
    if not args.no_check:
        import oracle
        ofmt = {"f32": oracle.F32, "f16": oracle.F16, "bf16": oracle.BF16, "fp8_e4m3": oracle.FP8_E4M3}[args.fmt]
        og = oracle.Grid(dims, ofmt, grid.origins, raw)
        rng = np.random.default_rng(12)
        qids = np.sort(rng.choice(n, 1 << 16, replace=False))
        ofilts = {stf.STF_LINEAR: oracle.LINEAR, stf.STF_CUBIC_BSPLINE: oracle.CUBIC, stf.STF_CUBIC_KEYS: oracle.KEYS,
                  stf.STF_CUBIC_MITCHELL: oracle.MITCHELL}
        sampled_gpu = {}
        for name, filt, mode, _ in variants:
            ofilt = ofilts[filt]
            if mode == stf.STF_STOCHASTIC and filt in stf.POSITIVIZED_FILTERS:
                idx = torch.empty((n, 6), dtype=torch.int32, device=dev)
                call(filt, mode, seed, out, idx)
                gv = out[:, 0].cpu().numpy()
                gi = idx.cpu().numpy()
                if args.order.endswith("morton"):
                    inv = np.empty(n, np.int64)
                    inv[order.cpu().numpy()] = np.arange(n)
                    gv, gi = gv[inv], gi[inv]
                gv, gi = gv[qids].astype(np.float64), gi[qids]
                ov, oi = og.filter_at(pts, qids, ofilt, oracle.STOCH, seed)
                scale = positivized_scale(oracle, og, pts[qids], oi, ofilt)
                err = np.abs(gv - ov)
                parity[name] = dict(sampled=int(qids.size), index_mismatches=int(np.any(gi != oi, axis=1).sum()),
                                    max_rel_err=float(np.max(np.where(scale > 0, err / np.where(scale > 0, scale, 1),
                                                                      np.where(err == 0, 0, np.inf)))),
                                    within_1e6=bool(np.all(err <= 1e-6 * scale)))
            elif mode == stf.STF_STOCHASTIC:
                idx = torch.empty((n, 3), dtype=torch.int32, device=dev)
                call(filt, mode, seed, out, idx)
                gv = out[:, 0].cpu().numpy()
                gi = idx.cpu().numpy()
                if args.order.endswith("morton"):   # back to the caller's order
                    inv = np.empty(n, np.int64)
                    inv[order.cpu().numpy()] = np.arange(n)
                    gv, gi = gv[inv], gi[inv]
                gv, gi = gv[qids], gi[qids]
                ov, oi = og.filter_at(pts, qids, ofilt, oracle.STOCH, seed)
                parity[name] = dict(sampled=int(qids.size), index_mismatches=int(np.any(gi != oi, axis=1).sum()),
                                    value_mismatches=int((gv != ov.astype(np.float32)).sum()))
                sampled_gpu[name] = gv
            else:
                call(filt, mode, seed, out)
                gv = out[:, 0].cpu().numpy()
                if args.order.endswith("morton"):
                    inv = np.empty(n, np.int64)
                    inv[order.cpu().numpy()] = np.arange(n)
                    gv = gv[inv]
                gv = gv[qids].astype(np.float64)
                sampled_gpu[name] = gv
                ov, _ = og.filter_at(pts, qids, ofilt, oracle.DET, 0)
                scale, _ = og.filter_at(pts, qids, ofilt, oracle.DET_ABS, 0)   # sum |w_k t_k|
                err = np.abs(gv - ov)
                rel = np.where(scale != 0, err / np.where(scale == 0, 1, scale), np.where(err == 0, 0, np.inf))
                parity[name] = dict(sampled=int(qids.size), max_rel_err=float(rel.max()),
                                    within_1e6=bool(np.all(err <= 1e-6 * scale)))
            log(f"parity {name}: {parity[name]}")
        if args.fmt != "f32":
            # precision: the results from 16- / 8-bit texels against the FP64
            # oracle on the binary32 grid they were rounded from
            og32 = oracle.Grid(dims, oracle.F32, grid.origins, grid.values)
            for name, filt, mode, _ in variants:
                if name not in sampled_gpu or filt in stf.POSITIVIZED_FILTERS:
                    continue
                if mode == stf.STF_STOCHASTIC:
                    ref, _ = og32.filter_at(pts, qids, ofilts[filt], oracle.STOCH, seed)
                    scale = np.abs(ref)
                else:
                    ref, _ = og32.filter_at(pts, qids, ofilts[filt], oracle.DET, 0)
                    scale, _ = og32.filter_at(pts, qids, ofilts[filt], oracle.DET_ABS, 0)
                quant[name] = quantization_error(sampled_gpu[name], ref, scale)
                log(f"{args.fmt} vs the FP64 oracle on the f32 grid, {name}: {quant[name]}")
        if not args.no_cpu and "stoch_cubic" in res:
            m = min(args.cpu_sample, n)
            sample = np.ascontiguousarray(pts[:m])
            threads = oracle.max_threads()
            # whole passes over the sample until about --cpu-seconds of work
            passes, t1 = 0, time.perf_counter()
            while True:
                og.filter(sample, oracle.CUBIC, oracle.STOCH, seed, want_index=False, nthreads=threads)
                passes += 1
                dt = time.perf_counter() - t1
                if dt >= args.cpu_seconds:
                    break
            cpu = dict(value=passes * m / dt, unit="lookups/s", cores=threads, kind="oracle", cpu_model=cpu_model(),
                       sample=f"{passes} pass(es) over {'all' if m == n else 'the first ' + str(m) + ' of the'} "
                              f"{n} queries of the batch, stochastic tricubic, FP64 C oracle with OpenMP, "
                              f"{dt:.2f} s in all")
            log(f"cpu oracle: {passes * m / dt / 1e6:.2f} M lookups/s on {threads} threads ({passes} passes, {dt:.1f} s)")

    # the same query stream against an empty grid of the same domain (every
    # walk ends at the root): the stream-only floor of the stochastic kernel
    stream_only = None
    if not args.only and not args.order.endswith("morton") and not args.no_stream_floor:
        empty = stf.stf_create_sparse_grid3d(dims, stf.FORMATS[args.fmt], np.zeros((0, 3), np.int32),
                                             np.zeros(0, raw.dtype))
        wall, kern = time_launches(lambda: stf.stf_filter(empty, q, stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, seed, out),
                                   args.steps, args.warmup, torch)
        stream_only = variant_stats(n, args.steps, wall, kern, 12 + 4)
        empty.destroy()
        log(f"stream only (empty grid): {stream_only['lookups_per_s'] / 1e9:.2f} G lookups/s, kernel "
            f"{stream_only['kernel_ms_mean'] * 1e3:.1f} us, {stream_only['achieved_gbs']:.0f} GB/s of query + result")

    medium = None
    if args.order == "ray" and not args.only and not args.no_medium:
        medium = run_grid_medium(args, torch, stf, synth, grid, tex, raw, out, seed, texel_b)

    # context for the roofline: a plain 1 GiB device-to-device copy (read +
    # write) timed the same way -- the practically reachable HBM rate
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    cw, ck = time_launches(lambda: dst.copy_(src), 5, 2, torch)
    copy_gbs = 2 * src.numel() * 4 / (float(np.mean(ck)) * 1e-3) / 1e9
    del src, dst
    log(f"device copy: {copy_gbs:.0f} GB/s")
    head = res.get("stoch_cubic") or next(iter(res.values()))
    det = res.get("det_cubic")
    line = base_line(args, head["lookups_per_s"], "lookups/s", head["ms_per_step"], args.fmt,
                     {"workload": f"sparse fBm voxel grid 512^3 of dense 8^3 {args.fmt} leaves "
                                  f"({grid.n_leaves} leaves), {n} "
                                  f"{STREAMS[args.order]}, "
                                  f"stochastic tricubic B-spline (deterministic 64-tap beside it)",
                      "n_queries": n, "n_leaves": grid.n_leaves, "order": args.order})
    line.update({
        "p50_batch_ms": head["kernel_ms_p50"],
        "p99_batch_ms": head["kernel_ms_p99"],
        "deterministic_lookups_per_s": det["lookups_per_s"] if det else None,
        "stochastic_over_deterministic": head["lookups_per_s"] / det["lookups_per_s"] if det else None,
        "interpolating_stochastic_over_deterministic": {
            k: res[f"stoch_{k}"]["lookups_per_s"] / res[f"det_{k}"]["lookups_per_s"]
            for k in ("keys", "mitchell") if f"stoch_{k}" in res and f"det_{k}" in res},
        "variants": res,
        "in_medium": medium,
        "stream_only_empty_grid": stream_only,
        "sort": sort_info,
        "parity": parity,
        "error_vs_f32_oracle": quant or None,
        "hbm_copy_gbs": copy_gbs,
        "roofline": {"bound": "hbm", "achieved": head["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["achieved_gbs"] / HBM_PEAK_GBS,
                     "traffic": args.traffic if args.traffic is not None
                     else measured_traffic(HEADLINE_TRAFFIC.get((args.fmt, args.order)))},
        "cpu_baseline": cpu,
    })
    tex.destroy()
    return line


def run_grid_medium(args, torch, stf, synth, grid, tex, raw, out, seed, texel_b):
    """Stochastic vs deterministic tricubic on the ray samples whose taps meet
    a stored leaf (the lookups a renderer makes inside the medium, empty space
    skipped), same grid, same count; with an oracle parity sample."""
    dev = out.device
    n = out.shape[0]
    t1 = time.time()
    mp = synth.medium_ray_queries(grid, n, seed=4)
    qm = torch.from_numpy(mp).to(dev)
    log(f"in-medium stream: {n} ray samples whose taps meet a leaf, {time.time() - t1:.1f}s")
    res = {}
    for name, mode in (("stoch_cubic", stf.STF_STOCHASTIC), ("det_cubic", stf.STF_DETERMINISTIC)):
        wall, kern = time_launches(lambda: stf.stf_filter(tex, qm, stf.STF_CUBIC_BSPLINE, mode, seed, out),
                                   args.steps, args.warmup, torch)
        res[name] = variant_stats(n, args.steps, wall, kern, 12 + 4 + (1 if mode == stf.STF_STOCHASTIC else 64) * texel_b)
        log(f"in-medium {name}: {res[name]['lookups_per_s'] / 1e9:.2f} G lookups/s, kernel "
            f"{res[name]['kernel_ms_mean'] * 1e3:.1f} us")
    res["stochastic_over_deterministic"] = res["stoch_cubic"]["lookups_per_s"] / res["det_cubic"]["lookups_per_s"]
    if not args.no_check:
        import oracle
        ofmt = {"f32": oracle.F32, "f16": oracle.F16, "bf16": oracle.BF16, "fp8_e4m3": oracle.FP8_E4M3}[args.fmt]
        og = oracle.Grid(grid.dims, ofmt, grid.origins, raw)
        qids = np.sort(np.random.default_rng(13).choice(n, 1 << 14, replace=False))
        idx = torch.empty((n, 3), dtype=torch.int32, device=dev)
        stf.stf_filter(tex, qm, stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, seed, out, idx)
        gv, gi = out[:, 0].cpu().numpy()[qids], idx.cpu().numpy()[qids]
        ov, oi = og.filter_at(mp, qids, oracle.CUBIC, oracle.STOCH, seed)
        par = {"sampled": int(qids.size), "index_mismatches": int(np.any(gi != oi, axis=1).sum()),
               "value_mismatches": int((gv != ov.astype(np.float32)).sum())}
        del idx
        stf.stf_filter(tex, qm, stf.STF_CUBIC_BSPLINE, stf.STF_DETERMINISTIC, 0, out)
        gd = out[:, 0].cpu().numpy()[qids].astype(np.float64)
        od, _ = og.filter_at(mp, qids, oracle.CUBIC, oracle.DET, 0)
        scale, _ = og.filter_at(mp, qids, oracle.CUBIC, oracle.DET_ABS, 0)
        par["det_within_1e6"] = bool(np.all(np.abs(gd - od) <= 1e-6 * scale))
        res["parity"] = par
        if args.fmt != "f32":
            og32 = oracle.Grid(grid.dims, oracle.F32, grid.origins, grid.values)
            sref, _ = og32.filter_at(mp, qids, oracle.CUBIC, oracle.STOCH, seed)
            dref, _ = og32.filter_at(mp, qids, oracle.CUBIC, oracle.DET, 0)
            dscale, _ = og32.filter_at(mp, qids, oracle.CUBIC, oracle.DET_ABS, 0)
            res["error_vs_f32_oracle"] = {"stoch_cubic": quantization_error(gv, sref, np.abs(sref)),
                                          "det_cubic": quantization_error(gd, dref, dscale)}
            log(f"in-medium {args.fmt} vs the FP64 oracle on the f32 grid: {res['error_vs_f32_oracle']}")
        log(f"in-medium parity: {par}")
    del qm
    return res


def quantization_error(got, ref32, scale):
    """Error of results from 16- or 8-bit texels against the FP64 oracle on
    the binary32 texture (same queries, same taps): max abs, RMS, and the
    max relative to the absolute scale (|value| for a drawn texel, sum
    |w t| for the deterministic filter) over results with a non-zero scale."""
    err = np.abs(got.astype(np.float64) - ref32)
    live = scale > 0
    return {"max_abs": float(err.max()), "rms": float(np.sqrt(np.mean(err ** 2))),
            "max_rel": float(np.max(err[live] / scale[live])) if live.any() else 0.0,
            "sampled": int(got.size)}


def positivized_scale(oracle, og, pts, oi, ofilt):
    """S+|t(j+)| + S-|t(j-)| per query: the scale of the positivized tolerance."""
    out = np.zeros(pts.shape[0])
    for k in range(pts.shape[0]):
        if not np.all(np.isfinite(pts[k])) or np.any(np.abs(pts[k]) >= 2 ** 24):
            continue
        t = pts[k].astype(np.float64) - np.floor(pts[k].astype(np.float64))
        sp, sn = oracle.positivized_masses(ofilt, t)
        s = sp * abs(og.texel(*(int(v) for v in oi[k, :3])))
        if oi[k, 3] != oracle.BAD_INDEX:
            s += sn * abs(og.texel(*(int(v) for v in oi[k, 3:])))
        out[k] = s
    return out


# ----------------------------------------------------------------------------
# 2D texture
# ----------------------------------------------------------------------------
def run_tex2d(args, torch, stf, synth):
    dev = torch.device("cuda:0")
    tex_np = synth.texture2d(256, 256, 4, seed=1)
    uv = synth.uv_queries(65536, seed=2)
    n = uv.shape[0]
    tex = stf.stf_create_texture2d(256, 256, 4, stf.STF_FMT_F32, [tex_np])
    q = torch.from_numpy(uv).to(dev)
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    res = {}
    for name, filt, mode, taps in (("stoch_cubic", stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 16),
                                   ("det_cubic", stf.STF_CUBIC_BSPLINE, stf.STF_DETERMINISTIC, 16),
                                   ("stoch_linear", stf.STF_LINEAR, stf.STF_STOCHASTIC, 4),
                                   ("det_linear", stf.STF_LINEAR, stf.STF_DETERMINISTIC, 4)):
        wall, kern = time_launches(lambda: stf.stf_filter(tex, q, filt, mode, 7, out), args.steps, args.warmup, torch)
        res[name] = variant_stats(n, args.steps, wall, kern, 8 + 16 + (16 if mode == stf.STF_STOCHASTIC else 16 * taps))
        log(f"{name}: {res[name]['lookups_per_s'] / 1e9:.2f} G lookups/s, kernel {res[name]['kernel_ms_mean'] * 1e3:.1f} us")
    head = res["stoch_cubic"]
    line = base_line(args, head["lookups_per_s"], "lookups/s", head["ms_per_step"], "f32",
                     {"workload": "2D texture 256x256 RGBA f32, 65,536 uniform uv queries, clamp, stochastic bicubic "
                                  "B-spline (deterministic 16-tap beside it)", "n_queries": n})
    line.update({"variants": res,
                 "stochastic_over_deterministic": head["lookups_per_s"] / res["det_cubic"]["lookups_per_s"],
                 "roofline": {"bound": "hbm", "achieved": head["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": head["achieved_gbs"] / HBM_PEAK_GBS,
                              "traffic": measured_traffic(TEX2D_STOCH_CUBIC_TRAFFIC)},
                 "cpu_baseline": None})
    tex.destroy()
    return line


# ----------------------------------------------------------------------------
# DCT-compressed texture set
# ----------------------------------------------------------------------------
def run_dct(args, torch, stf, synth):
    dev = torch.device("cuda:0")
    t0 = time.time()
    size, C = 4096, 9
    tex_np = synth.texture_set_u8(size, seed=51)
    words = stf.stf_dct_encode(tex_np)
    tex = stf.stf_create_dct_texture2d(size, size, C, words)
    uv = synth.screen_uv_queries(3840, 2160, seed=53)   # a 4K frame of the textured ground plane
    uv_rand = synth.uv_queries(uv.shape[0], seed=52)     # the same count, uniform and unordered
    n = uv.shape[0]
    log(f"inputs and host encoding {time.time() - t0:.1f}s, {stf.stf_texture_bytes(tex) / 1e6:.1f} MB of blocks")
    q = torch.from_numpy(uv).to(dev)
    q_rand = torch.from_numpy(uv_rand).to(dev)
    out = torch.empty((n, C), dtype=torch.float32, device=dev)
    block_b = 4 * ((C + 3) // 4 * 4)   # one decode reads its block's channel words
    res = {}
    for name, filt, mode, taps, qq in (("stoch_linear", stf.STF_LINEAR, stf.STF_STOCHASTIC, 4, q),
                                       ("det_linear", stf.STF_LINEAR, stf.STF_DETERMINISTIC, 4, q),
                                       ("stoch_cubic", stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 16, q),
                                       ("det_cubic", stf.STF_CUBIC_BSPLINE, stf.STF_DETERMINISTIC, 16, q),
                                       ("stoch_keys", stf.STF_CUBIC_KEYS, stf.STF_STOCHASTIC, 16, q),
                                       ("det_keys", stf.STF_CUBIC_KEYS, stf.STF_DETERMINISTIC, 16, q),
                                       ("stoch_linear_random_uv", stf.STF_LINEAR, stf.STF_STOCHASTIC, 4, q_rand),
                                       ("det_linear_random_uv", stf.STF_LINEAR, stf.STF_DETERMINISTIC, 4, q_rand),
                                       ("stoch_cubic_random_uv", stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 16, q_rand),
                                       ("det_cubic_random_uv", stf.STF_CUBIC_BSPLINE, stf.STF_DETERMINISTIC, 16, q_rand)):
        decodes = (2 if filt in stf.POSITIVIZED_FILTERS else 1) if mode == stf.STF_STOCHASTIC else taps
        wall, kern = time_launches(lambda: stf.stf_filter(tex, qq, filt, mode, 11, out), args.steps, args.warmup,
                                   torch)
        res[name] = variant_stats(n, args.steps, wall, kern, 8 + 4 * C + decodes * block_b)
        res[name]["decodes_per_lookup"] = decodes
        log(f"{name}: {res[name]['lookups_per_s'] / 1e9:.2f} G lookups/s, kernel "
            f"{res[name]['kernel_ms_mean'] * 1e3:.1f} us")
    # the frame Morton-sorted by the library (sort timed apart): deterministic
    # bicubic blocks then decode each texel of their taps once into LDS
    sq = torch.empty_like(q)
    order = torch.empty(n, dtype=torch.int32, device=dev)
    ws = torch.empty(stf.stf_sort_workspace_bytes(n), dtype=torch.uint8, device=dev)
    wall, _ = time_launches(lambda: stf.stf_sort_queries(tex, q, sq, order, ws), args.steps, args.warmup, torch)
    sort_ms = 1e3 * wall / args.steps
    log(f"morton sort of the frame: {sort_ms:.3f} ms")
    for name, filt, mode, taps in (("stoch_cubic_sorted", stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 16),
                                   ("det_cubic_sorted", stf.STF_CUBIC_BSPLINE, stf.STF_DETERMINISTIC, 16)):
        decodes = 1 if mode == stf.STF_STOCHASTIC else taps
        wall, kern = time_launches(lambda: stf.stf_filter_ordered(tex, sq, order, filt, mode, 11, out),
                                   args.steps, args.warmup, torch)
        res[name] = variant_stats(n, args.steps, wall, kern, 8 + 4 * C + decodes * block_b)
        res[name]["decodes_per_lookup"] = decodes
        log(f"{name}: {res[name]['lookups_per_s'] / 1e9:.2f} G lookups/s, kernel "
            f"{res[name]['kernel_ms_mean'] * 1e3:.1f} us")
    del sq, order, ws
    # quality of the compression: bilinear at texel centres returns decoded texels
    js, is_ = np.meshgrid(np.arange(size), np.arange(size), indexing="ij")
    cen = np.stack([(is_ + 0.5) / size, (js + 0.5) / size], axis=-1).reshape(-1, 2).astype(np.float32)
    dec = torch.empty((cen.shape[0], C), dtype=torch.float32, device=dev)
    stf.stf_filter(tex, torch.from_numpy(cen).to(dev), stf.STF_LINEAR, stf.STF_DETERMINISTIC, 0, dec)
    ref = torch.from_numpy(tex_np.reshape(-1, C)).to(dev).float() / 255.0
    mse = float(((dec - ref) ** 2).mean().item())
    head = res["stoch_linear"]
    stream_b = 8 + 4 * C
    stream_gbs = stream_b * n / (head["kernel_ms_mean"] * 1e-3) / 1e9   # per launch, over the kernel's duration
    line = base_line(args, head["lookups_per_s"], "lookups/s", head["ms_per_step"], "f32",
                     {"workload": f"DCT-compressed {size}^2 x {C} texture set (8x8 blocks, 6 coefficients per channel "
                                  f"in 32 bits), {n} uv queries of a 3840x2160 frame of a textured ground plane "
                                  "(pixel order), stochastic bilinear (1 decode) vs deterministic (4 decodes); "
                                  "bicubic, Keys and uniformly random uv beside it", "n_queries": n})
    line.update({"variants": res,
                 "stochastic_over_deterministic": head["lookups_per_s"] / res["det_linear"]["lookups_per_s"],
                 "bicubic_stochastic_over_deterministic":
                     res["stoch_cubic"]["lookups_per_s"] / res["det_cubic"]["lookups_per_s"],
                 "sorted_bicubic_stochastic_over_deterministic":
                     res["stoch_cubic_sorted"]["lookups_per_s"] / res["det_cubic_sorted"]["lookups_per_s"],
                 "sort_ms": sort_ms,
                 "compression": {"block_bytes": stf.stf_texture_bytes(tex), "u8_bytes": int(tex_np.nbytes),
                                 "psnr_db": 10 * np.log10(1.0 / mse)},
                 # streamed bytes only (uv in, results out); the block words are
                 # a cache-resident 12.6 MB table, as the grid's tree nodes are
                 "roofline": {"bound": "hbm", "achieved": stream_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": stream_gbs / HBM_PEAK_GBS, "stream_bytes_per_lookup": stream_b,
                              "traffic": measured_traffic(DCT_STOCH_LINEAR_TRAFFIC)},
                 "cpu_baseline": None})
    tex.destroy()
    return line


# ----------------------------------------------------------------------------
# Gaussian filters and filter importance sampling
# ----------------------------------------------------------------------------
def run_gauss(args, torch, stf, synth):
    """The sigma in {0.3, 0.5, 0.8} comparison of FIS and discrete 4x4
    sampling on the DCT texture set over a 4K frame: throughput of each mode
    and, per sigma, how far the discrete 4x4 filter's mean lies from the
    box-convolved Gaussian that FIS estimates (RMS over the frame)."""
    dev = torch.device("cuda:0")
    size, C = 4096, 9
    tex_np = synth.texture_set_u8(size, seed=51)
    tex = stf.stf_create_dct_texture2d(size, size, C, stf.stf_dct_encode(tex_np))
    uv = synth.screen_uv_queries(3840, 2160, seed=53)
    n = uv.shape[0]
    q = torch.from_numpy(uv).to(dev)
    out = torch.empty((n, C), dtype=torch.float32, device=dev)
    ref = torch.empty_like(out)
    res, quality = {}, {}
    block_b = 4 * ((C + 3) // 4 * 4)
    for sigma in (0.3, 0.5, 0.8):
        for name, mode in (("fis", stf.STF_GAUSS_FIS), ("discrete", stf.STF_GAUSS_DISCRETE),
                           ("fis_mean", stf.STF_GAUSS_FIS_MEAN), ("discrete_mean", stf.STF_GAUSS_DISCRETE_MEAN)):
            taps = {"fis": 1, "discrete": 1, "discrete_mean": 16,
                    "fis_mean": (2 * (int(np.ceil(6 * sigma)) + 1) + 2) ** 2}[name]
            wall, kern = time_launches(lambda: stf.stf_filter_gaussian(tex, q, sigma, mode, 5, out), args.steps,
                                       args.warmup, torch)
            key = f"{name}_sigma{sigma}"
            res[key] = variant_stats(n, args.steps, wall, kern, 8 + 4 * C + taps * block_b)
            res[key]["decodes_per_lookup"] = taps
            log(f"{key}: {res[key]['lookups_per_s'] / 1e9:.2f} G lookups/s, kernel {res[key]['kernel_ms_mean'] * 1e3:.1f} us")
        stf.stf_filter_gaussian(tex, q, sigma, stf.STF_GAUSS_FIS_MEAN, 0, ref)
        stf.stf_filter_gaussian(tex, q, sigma, stf.STF_GAUSS_DISCRETE_MEAN, 0, out)
        quality[f"sigma{sigma}"] = {"rms_discrete_mean_minus_fis_mean": float(torch.sqrt(((out - ref) ** 2).mean()).item())}
        log(f"sigma {sigma}: {quality[f'sigma{sigma}']}")
    head = res["fis_sigma0.5"]
    stream_b = 8 + 4 * C
    stream_gbs = stream_b * n / (head["kernel_ms_mean"] * 1e-3) / 1e9   # per launch, over the kernel's duration
    line = base_line(args, head["lookups_per_s"], "lookups/s", head["ms_per_step"], "f32",
                     {"workload": f"Gaussian filtering (sigma 0.3 / 0.5 / 0.8 texels) of the DCT-compressed {size}^2 x "
                                  f"{C} texture set over a 3840x2160 frame ({n} uv): FIS (Box-Muller + nearest, 1 "
                                  "decode) and discrete 4x4 sampling vs their deterministic means", "n_queries": n})
    line.update({"variants": res, "quality": quality,
                 "fis_over_fis_mean_sigma0.5": head["lookups_per_s"] / res["fis_mean_sigma0.5"]["lookups_per_s"],
                 # streamed bytes only (uv in, results out), as on the DCT line
                 "roofline": {"bound": "hbm", "achieved": stream_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": stream_gbs / HBM_PEAK_GBS, "stream_bytes_per_lookup": stream_b,
                              "traffic": measured_traffic(GAUSS_FIS_TRAFFIC)},
                 "cpu_baseline": None})
    tex.destroy()
    return line


# ----------------------------------------------------------------------------
# elliptically weighted average filtering
# ----------------------------------------------------------------------------
def run_ewa(args, torch, stf, synth):
    """EWA over the full MIP pyramid of a 4096^2 RGBA8 texture (the albedo and
    roughness of the texture set) for the EWA queries of a 3840x2160 frame of
    the ground plane (texture tiled every 2 units: minified, anisotropic
    towards the horizon): one texel per stochastic lookup vs the full
    two-level EWA."""
    dev = torch.device("cuda:0")
    size = 4096
    rgba = np.ascontiguousarray(synth.texture_set_u8(size, seed=51)[:, :, :4])
    lv = synth.mip_levels(rgba)
    tex = stf.stf_create_texture2d(size, size, 4, stf.STF_FMT_U8, lv)
    qn = synth.screen_ewa_queries(3840, 2160, seed=53)
    n = qn.shape[0]
    q = torch.from_numpy(qn).to(dev)
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    res = {}
    for _ in range(40):   # let the clocks settle before the first timed variant
        stf.stf_filter_ewa(tex, q, 8.0, stf.STF_DETERMINISTIC, 9, out)
    torch.cuda.synchronize()
    for aniso in (8.0, 64.0):
        for name, mode in (("stoch", stf.STF_STOCHASTIC), ("det", stf.STF_DETERMINISTIC)):
            wall, kern = time_launches(lambda: stf.stf_filter_ewa(tex, q, aniso, mode, 9, out), args.steps,
                                       args.warmup, torch)
            key = f"{name}_aniso{int(aniso)}"
            res[key] = variant_stats(n, args.steps, wall, kern, 24 + 16 + 4)
            log(f"{key}: {res[key]['lookups_per_s'] / 1e9:.2f} G lookups/s, kernel {res[key]['kernel_ms_mean'] * 1e3:.1f} us")
    head = res["stoch_aniso8"]
    line = base_line(args, head["lookups_per_s"], "lookups/s", head["ms_per_step"], "f32",
                     {"workload": f"EWA over the MIP pyramid of a {size}^2 RGBA8 texture, {n} queries of a 3840x2160 "
                                  "frame (uv + derivatives), max anisotropy 8 and 64: stochastic (level draw + one "
                                  "texel) vs deterministic two-level EWA", "n_queries": n})
    line.update({"variants": res,
                 "stochastic_over_deterministic": head["lookups_per_s"] / res["det_aniso8"]["lookups_per_s"],
                 "stochastic_over_deterministic_aniso64":
                     res["stoch_aniso64"]["lookups_per_s"] / res["det_aniso64"]["lookups_per_s"],
                 "roofline": {"bound": "hbm", "achieved": head["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": head["achieved_gbs"] / HBM_PEAK_GBS, "traffic": measured_traffic(EWA_STOCH_TRAFFIC)},
                 "cpu_baseline": None})
    tex.destroy()
    return line


# ----------------------------------------------------------------------------
# filtering with shading
# ----------------------------------------------------------------------------
GGX_FLOPS = 120   # binary32 operations of one shading evaluation (see the design notes)


def run_shade(args, torch, stf, synth):
    dev = torch.device("cuda:0")
    t0 = time.time()
    lv = synth.material_levels(4096, seed=21, levels=3)
    recs = synth.shade_queries(1 << 23, seed=22)
    n = recs.shape[0]
    log(f"inputs {time.time() - t0:.1f}s")
    mat = stf.stf_create_material2d(4096, 4096, lv)
    q = torch.from_numpy(recs).to(dev)
    out = torch.empty((n, 3), dtype=torch.float32, device=dev)
    res = {}
    for name, mode, evals in (("stochastic", stf.STF_SHADE_STOCHASTIC, 1),
                              ("filter_after_shade", stf.STF_FILTER_AFTER_SHADE, 16),
                              ("shade_after_filter", stf.STF_SHADE_AFTER_FILTER, 1)):
        wall, kern = time_launches(lambda: stf.stf_shade_filter(mat, q, stf.STF_CUBIC_BSPLINE, mode, 5, out),
                                   args.steps, args.warmup, torch)
        taps = 1 if mode == stf.STF_SHADE_STOCHASTIC else 16
        res[name] = variant_stats(n, args.steps, wall, kern, 36 + 12 + 8 * taps)
        res[name]["shading_evals"] = evals
        res[name]["achieved_tflops"] = evals * GGX_FLOPS * n / (res[name]["kernel_ms_mean"] * 1e-3) / 1e12
        log(f"{name}: {res[name]['lookups_per_s'] / 1e9:.2f} G lookups/s, kernel {res[name]['kernel_ms_mean'] * 1e3:.1f} us")
    head = res["stochastic"]
    fas = res["filter_after_shade"]
    line = base_line(args, head["lookups_per_s"], "lookups/s", head["ms_per_step"], "f32",
                     {"workload": "filter-after-shading, 4096^2 material (RGB8 albedo, U8 roughness, 2xf16 normal, "
                                  "3 levels), 8,388,608 GGX shading queries, bicubic: stochastic (1 eval) vs "
                                  "deterministic filter-after-shade (16 evals) vs shade-after-filter",
                      "n_queries": n})
    line.update({"variants": res,
                 "stochastic_over_filter_after_shade": head["lookups_per_s"] / fas["lookups_per_s"],
                 # the 16 taps of uniformly scattered queries are gathered from a 128 MiB
                 # material: the kernel waits on memory, not on its GGX arithmetic
                 "roofline": {"bound": "hbm", "achieved": fas["achieved_gbs"], "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": fas["achieved_gbs"] / HBM_PEAK_GBS,
                              "traffic": measured_traffic(SHADE_FAS_TRAFFIC), "kernel": "filter_after_shade",
                              "alu_tflops": fas["achieved_tflops"], "alu_peak_tflops": FP32_VECTOR_PEAK_TFLOPS},
                 "cpu_baseline": None})
    mat.destroy()
    return line


# ----------------------------------------------------------------------------
# neural texture
# ----------------------------------------------------------------------------
DECODE_FLOPS = 2 * (8 * 64 + 64 * 64 + 64 * 8)   # useful multiply-adds of one decode, x2


def run_neural(args, torch, stf, synth):
    dev = torch.device("cuda:0")
    t0 = time.time()
    size, lsize = args.neural_size, args.neural_size // 4
    target = synth.neural_target(size, seed=41)
    lat, mlp = synth.neural_init(lsize, seed=42)
    uv = synth.neural_queries(1 << 24, seed=43)
    n = uv.shape[0]
    log(f"inputs {time.time() - t0:.1f}s")
    nt = stf.stf_ntex_create(size, size, lat, mlp)
    tgt = torch.from_numpy(target).to(dev)
    steps = args.neural_steps
    loss = torch.empty(steps, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stf.stf_ntex_train(nt, tgt, steps, 1 << 18, 1e-2, 1e-3, 7, loss)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    loss_np = loss.cpu().numpy()
    log(f"training: {steps} steps in {train_s:.2f}s, loss {loss_np[0]:.4g} -> {loss_np[-1]:.4g}")
    stf.stf_ntex_prepare_inference(nt)
    q = torch.from_numpy(uv).to(dev)
    out = torch.empty((n, 8), dtype=torch.float32, device=dev)
    res = {}
    for name, filt, mode, dec in (("stoch_cubic", stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 1),
                                  ("det_cubic", stf.STF_CUBIC_BSPLINE, stf.STF_DETERMINISTIC, 16),
                                  ("stoch_linear", stf.STF_LINEAR, stf.STF_STOCHASTIC, 1),
                                  ("det_linear", stf.STF_LINEAR, stf.STF_DETERMINISTIC, 4)):
        wall, kern = time_launches(lambda: stf.stf_ntex_filter(nt, q, filt, mode, 3, out), args.steps, args.warmup,
                                   torch)
        res[name] = variant_stats(n, args.steps, wall, kern, 8 + 32 + 64 * dec)
        res[name]["decodes_per_lookup"] = dec
        res[name]["achieved_tflops"] = dec * DECODE_FLOPS * n / (res[name]["kernel_ms_mean"] * 1e-3) / 1e12
        log(f"{name}: {res[name]['lookups_per_s'] / 1e9:.2f} G lookups/s, "
            f"{res[name]['achieved_tflops']:.1f} TFLOP/s useful")
    # quality: decode every texel (bilinear at texel centres) against the stored texture
    js, is_ = np.meshgrid(np.arange(size), np.arange(size), indexing="ij")
    cen = np.stack([(is_ + 0.5) / size, (js + 0.5) / size], axis=-1).reshape(-1, 2).astype(np.float32)
    cq = torch.from_numpy(cen).to(dev)
    dec = torch.empty((cen.shape[0], 8), dtype=torch.float32, device=dev)
    stf.stf_ntex_filter(nt, cq, stf.STF_LINEAR, stf.STF_DETERMINISTIC, 0, dec)
    mse = float(((dec - tgt.reshape(-1, 8)) ** 2).mean().item())
    head = res["det_cubic"]
    line = base_line(args, res["stoch_cubic"]["lookups_per_s"], "lookups/s", res["stoch_cubic"]["ms_per_step"], "bf16",
                     {"workload": f"neural texture {size}^2 x 8 as {lsize}^2 x 8 latents + MLP 8-64-64-8, "
                                  f"{n} uv queries, bicubic: stochastic (1 decode) vs deterministic (16 decodes), "
                                  "BF16 MFMA decode", "n_queries": n})
    line.update({"variants": res,
                 "stochastic_over_deterministic": res["stoch_cubic"]["lookups_per_s"] / head["lookups_per_s"],
                 "training": {"steps": steps, "batch": 1 << 18, "seconds": train_s,
                              "samples_per_s": steps * (1 << 18) / train_s, "loss_first": float(loss_np[0]),
                              "loss_last": float(loss_np[-1])},
                 "psnr_db": 10 * np.log10(1.0 / mse),
                 "roofline": {"bound": "mfma", "achieved": head["achieved_tflops"], "peak": MFMA_BF16_PEAK_TFLOPS,
                              "unit": "TFLOP/s", "frac": head["achieved_tflops"] / MFMA_BF16_PEAK_TFLOPS,
                              "traffic": measured_traffic(NEURAL_DET_CUBIC_TRAFFIC), "kernel": "det_cubic"},
                 "cpu_baseline": None})
    nt.destroy()
    return line


# ----------------------------------------------------------------------------
# serving
# ----------------------------------------------------------------------------
def run_serving(args, torch, stf, synth):
    dev = torch.device("cuda:0")
    t0 = time.time()
    g1 = synth.fbm_grid((512, 512, 512), seed=3)
    g2 = synth.coarse_fbm_grid((2048, 2048, 2048), occupancy=0.02, seed=13)
    mat = synth.material_levels(4096, seed=21, levels=1)[0]
    t1 = stf.stf_create_sparse_grid3d(g1.dims, stf.STF_FMT_F16, g1.origins, g1.encoded("f16"))
    t2 = stf.stf_create_sparse_grid3d(g2.dims, stf.STF_FMT_F16, g2.origins, g2.encoded("f16"))
    t3 = stf.stf_create_material2d(4096, 4096, [mat])   # filtered as six channels
    pool_n = 1 << 24
    pools = [torch.from_numpy(synth.ray_queries(g1.dims, 65536, 256, seed=4)).to(dev),
             torch.from_numpy(synth.ray_queries(g2.dims, 65536, 256, seed=14)).to(dev),
             torch.from_numpy(synth.uv_queries(pool_n, seed=15)).to(dev)]
    texs = [(t1, 3, 1), (t2, 3, 1), (t3, 2, 6)]
    outs = [torch.empty((pool_n, c), dtype=torch.float32, device=dev) for _, _, c in texs]
    log(f"inputs {time.time() - t0:.1f}s: grid512 {g1.n_leaves} leaves, grid2048 {g2.n_leaves} leaves")
    srv = stf.stf_server_create(1 << 30, args.serve_resident, 1 << 18)
    rng = np.random.default_rng(99)
    loads = {}
    flags = stf.STF_SERVE_QUERIES_ON_DEVICE | stf.STF_SERVE_RESULTS_ON_DEVICE
    # warm-up: one second at the first load, untimed (first launches of every
    # serving kernel, the server's pool of completion events)
    for warm, load in [(True, args.loads[0])] + [(False, l) for l in args.loads]:
        sizes = np.clip(np.exp(rng.normal(np.log(16384.0), 1.0, 1 << 16)), 1024, 1 << 20).astype(np.int64)
        rate = load / sizes.mean()
        count = int(rate * (1.0 if warm else args.serve_seconds))
        if count > sizes.size:
            more = np.exp(rng.normal(np.log(16384.0), 1.0, count - sizes.size))
            sizes = np.concatenate([sizes, np.clip(more, 1024, 1 << 20).astype(np.int64)])
        sizes = sizes[:count]
        arrivals = np.cumsum(rng.exponential(1.0 / rate, count))
        which = rng.integers(0, 3, count)
        cubic = rng.random(count) < 0.5
        offs = (rng.random(count) * (pool_n - sizes)).astype(np.int64)
        reqs = []
        for k in range(count):
            tex, dims, ch = texs[which[k]]
            reqs.append((tex, pools[which[k]].data_ptr() + 4 * dims * int(offs[k]), int(sizes[k]),
                         stf.STF_CUBIC_BSPLINE if cubic[k] else stf.STF_LINEAR, k,
                         outs[which[k]].data_ptr() + 4 * ch * int(offs[k]), None, float(arrivals[k])))
        stf.stf_server_reset_stats(srv)
        torch.cuda.synchronize()
        stf.stf_server_replay(srv, reqs, flags, timeout_s=120.0)
        if warm:
            continue
        st = stf.stf_server_stats(srv)
        st["offered_lookups_per_s"] = load
        st["requests"] = count
        st["saturated"] = st["lookups_per_s"] < 0.9 * load
        loads[f"{load:.2g}"] = st
        log(f"load {load / 1e9:.1f} G/s: {count} requests, served {st['lookups_per_s'] / 1e9:.2f} G/s, "
            f"p50 {st['p50_ms']:.3f} ms, p99 {st['p99_ms']:.3f} ms, peak resident {st['peak_resident']}")
    top = loads[f"{args.loads[-1]:.2g}"]
    line = base_line(args, top["lookups_per_s"], "lookups/s", None, "f16",
                     {"workload": "serving: open-loop Poisson arrivals, log-normal request sizes (median 16,384, "
                                  "clamp 1,024..1,048,576), 3 resident textures (512^3 fBm grid f16, 2048^3 grid "
                                  "f16 at 2%, 4096^2 material: RGB8 albedo, U8 roughness, 2xf16 normal, six "
                                  "channels), stochastic tri/bi-linear and -cubic 50/50",
                      "offered_loads": list(args.loads)})
    line.update({"p50_batch_ms": top["p50_ms"], "p99_batch_ms": top["p99_ms"], "loads": loads,
                 "roofline": None, "cpu_baseline": None})
    srv.destroy()
    for t, _, _ in texs:
        t.destroy()
    return line


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grid", choices=["grid", "tex2d", "shade", "neural", "serving", "dct", "gauss", "ewa"])
    ap.add_argument("--fmt", default="f32", choices=["f32", "f16", "bf16", "fp8_e4m3"])
    ap.add_argument("--order", default="ray", choices=list(STREAMS),
                    help="grid query stream: ray samples in ray order, shuffled or Morton-sorted by the library, "
                         "or only the ray samples whose taps meet a stored leaf (inside the medium), as they come "
                         "or Morton-sorted")
    ap.add_argument("--cpu-sample", type=int, default=1 << 24, help="queries in the CPU-oracle timing sample")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="repeat the CPU-oracle timing over the sample for at least this long")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle timing")
    ap.add_argument("--no-stream-floor", action="store_true",
                    help="skip the stream-only run against an empty grid (grid workload)")
    ap.add_argument("--no-medium", action="store_true",
                    help="skip the in-medium stream beside the ray stream (grid workload)")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle parity sample and the CPU timing")
    ap.add_argument("--only", default="", help="time only this variant (e.g. stoch_cubic)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 256 MiB device copy first (hardware-counter calibration)")
    ap.add_argument("--traffic", type=float, default=None,
                    help="measured HBM bytes per launch of the headline kernel, overriding the recorded value")
    ap.add_argument("--neural-size", type=int, default=4096)
    ap.add_argument("--neural-steps", type=int, default=1000)
    ap.add_argument("--loads", type=float, nargs="+", default=[0.5e9, 1e9, 2e9])
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-resident", type=int, default=4096, help="requests resident at once in the server")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2305_05810_amd as stf
    import synth

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain device copy of known size, for scaling hardware byte counters
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("copy calibration: 3 x 268435456 bytes read and written")
    run = {"grid": run_grid, "tex2d": run_tex2d, "shade": run_shade, "neural": run_neural, "dct": run_dct, "gauss": run_gauss, "ewa": run_ewa,
           "serving": run_serving}[args.workload]
    line = run(args, torch, stf, synth)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
