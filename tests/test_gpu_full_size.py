"""Parity at the benchmark's full size: the 512^3 fBm grid with 16,777,216
ray-ordered queries, and with the 16,777,216 samples of its in-medium stream,
in the same single-call launches the benchmark times.
The oracle recomputes 65,536 sampled queries (as members of the whole batch,
since a query's draw depends on its index), index-exact and value-exact for
the stochastic filters and within 1e-6 for the deterministic ones.  Properties
that hold at any size are checked on the whole batch."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_05810_amd as stf
import synth

pytestmark = pytest.mark.gpu

DIMS = (512, 512, 512)
ORC_FMT = {"f32": oracle.F32, "f16": oracle.F16, "bf16": oracle.BF16, "fp8_e4m3": oracle.FP8_E4M3}


@pytest.fixture(scope="module")
def workload():
    grid = synth.fbm_grid(DIMS, seed=3)
    pts = synth.ray_queries(DIMS, n_rays=65536, samples_per_ray=256, seed=4)
    rng = np.random.default_rng(12)
    qids = np.sort(rng.choice(pts.shape[0], 1 << 16, replace=False))
    return grid, pts, qids


@pytest.fixture(scope="module")
def medium(workload):
    """The in-medium stream of the same grid: 16,777,216 ray samples whose 4^3
    tap blocks meet a stored leaf, so every lookup reads texels."""
    grid = workload[0]
    pts = synth.medium_ray_queries(grid, 1 << 24, seed=4)
    rng = np.random.default_rng(13)
    qids = np.sort(rng.choice(pts.shape[0], 1 << 16, replace=False))
    return pts, qids


@pytest.mark.parametrize("fmt", ["f32", "fp8_e4m3"])
def test_full_size_in_medium(dev, workload, medium, fmt):
    # The stream the in-medium benchmark line times, in the same single-call
    # launch: every lookup walks to a leaf and reads stored texels.
    grid = workload[0]
    pts, qids = medium
    raw = grid.encoded(fmt)
    tex = stf.stf_create_sparse_grid3d(DIMS, stf.FORMATS[fmt], grid.origins, raw)
    og = oracle.Grid(DIMS, ORC_FMT[fmt], grid.origins, raw)
    n = pts.shape[0]
    print(f"in-medium {fmt}: {n} queries, {qids.size} sampled", flush=True)
    q = torch.from_numpy(pts).to(dev)
    out = torch.empty((n, 1), dtype=torch.float32, device=dev)
    idx = torch.empty((n, 3), dtype=torch.int32, device=dev)
    seed = 0x5EED
    for gf, of in ((stf.STF_CUBIC_BSPLINE, oracle.CUBIC), (stf.STF_LINEAR, oracle.LINEAR)):
        stf.stf_filter(tex, q, gf, stf.STF_STOCHASTIC, seed, out, idx)
        v = out[:, 0].cpu().numpy()
        ix = idx.cpu().numpy()
        ov, oi = og.filter_at(pts, qids, of, oracle.STOCH, seed)
        assert np.array_equal(ix[qids], oi)
        assert np.array_equal(v[qids], ov.astype(np.float32))
        assert np.all(np.isfinite(v))
        stf.stf_filter(tex, q, gf, stf.STF_DETERMINISTIC, 0, out)
        d = out[:, 0].cpu().numpy().astype(np.float64)
        od, _ = og.filter_at(pts, qids, of, oracle.DET, 0)
        err = np.abs(d[qids] - od)
        assert np.all(err <= 1e-6 * np.abs(od) + 1e-12), err.max()
    tex.destroy()


@pytest.mark.parametrize("fmt", ["f32", "f16", "bf16", "fp8_e4m3"])
def test_full_size_parity(dev, workload, fmt):
    grid, pts, qids = workload
    raw = grid.encoded(fmt)
    tex = stf.stf_create_sparse_grid3d(DIMS, stf.FORMATS[fmt], grid.origins, raw)
    og = oracle.Grid(DIMS, ORC_FMT[fmt], grid.origins, raw)
    n = pts.shape[0]
    q = torch.from_numpy(pts).to(dev)
    out = torch.empty((n, 1), dtype=torch.float32, device=dev)
    idx = torch.empty((n, 3), dtype=torch.int32, device=dev)
    seed = 0x5EED
    for gf, of in ((stf.STF_CUBIC_BSPLINE, oracle.CUBIC), (stf.STF_LINEAR, oracle.LINEAR)):
        stf.stf_filter(tex, q, gf, stf.STF_STOCHASTIC, seed, out, idx)
        v = out[:, 0].cpu().numpy()
        ix = idx.cpu().numpy()
        ov, oi = og.filter_at(pts, qids, of, oracle.STOCH, seed)
        assert np.array_equal(ix[qids], oi)
        assert np.array_equal(v[qids], ov.astype(np.float32))
        # whole batch: every chosen tap is within the filter's support of its query
        lo = np.floor(pts).astype(np.int64)
        off = ix.astype(np.int64) - lo
        rng = (-1, 2) if gf == stf.STF_CUBIC_BSPLINE else (0, 1)
        assert off.min() >= rng[0] and off.max() <= rng[1]
        assert np.all(np.isfinite(v)) and v.min() >= 0.0
        if fmt == "f32":
            stf.stf_filter(tex, q, gf, stf.STF_DETERMINISTIC, 0, out)
            d = out[:, 0].cpu().numpy().astype(np.float64)
            od, _ = og.filter_at(pts, qids, of, oracle.DET, 0)
            err = np.abs(d[qids] - od)
            assert np.all(err <= 1e-6 * np.abs(od)), err.max()
    tex.destroy()


@pytest.mark.parametrize("gf,of", [(stf.STF_CUBIC_KEYS, oracle.KEYS), (stf.STF_CUBIC_MITCHELL, oracle.MITCHELL)])
def test_full_size_interpolating_cubics(dev, workload, gf, of):
    """Positivized stochastic (two taps) and 64-tap deterministic filtering
    with the interpolating cubics on the whole batch, checked at the sampled
    queries: indices exact, values within 1e-6 of S+|t+| + S-|t-| (stochastic)
    and of sum |w t| (deterministic)."""
    grid, pts, qids = workload
    tex = stf.stf_create_sparse_grid3d(DIMS, stf.STF_FMT_F32, grid.origins, grid.values)
    og = oracle.Grid(DIMS, oracle.F32, grid.origins, grid.values)
    n = pts.shape[0]
    q = torch.from_numpy(pts).to(dev)
    out = torch.empty((n, 1), dtype=torch.float32, device=dev)
    idx = torch.empty((n, 6), dtype=torch.int32, device=dev)
    seed = 0xC0FFEE
    sub = qids[:8192]
    stf.stf_filter(tex, q, gf, stf.STF_STOCHASTIC, seed, out, idx)
    v = out[:, 0].cpu().numpy().astype(np.float64)
    ix = idx.cpu().numpy()
    ov, oi = og.filter_at(pts, sub, of, oracle.STOCH, seed)
    assert np.array_equal(ix[sub], oi)
    scale = np.zeros(sub.size)
    for k, qi in enumerate(sub):
        t = pts[qi].astype(np.float64) - np.floor(pts[qi].astype(np.float64))
        sp, sn = oracle.positivized_masses(of, t)
        scale[k] = sp * abs(og.texel(*(int(c) for c in oi[k, :3])))
        if oi[k, 3] != oracle.BAD_INDEX:
            scale[k] += sn * abs(og.texel(*(int(c) for c in oi[k, 3:])))
    assert np.all(np.abs(v[sub] - ov) <= 1e-6 * scale)
    # whole batch: both taps lie in the 4^3 support of their query
    lo = np.floor(pts).astype(np.int64)
    off = ix[:, :3].astype(np.int64) - lo
    assert off.min() >= -1 and off.max() <= 2
    has = ix[:, 3] != oracle.BAD_INDEX
    offn = ix[has, 3:].astype(np.int64) - lo[has]
    assert offn.min() >= -1 and offn.max() <= 2
    stf.stf_filter(tex, q, gf, stf.STF_DETERMINISTIC, 0, out)
    d = out[:, 0].cpu().numpy().astype(np.float64)
    od, _ = og.filter_at(pts, qids, of, oracle.DET, 0)
    sc, _ = og.filter_at(pts, qids, of, oracle.DET_ABS, 0)
    assert np.all(np.abs(d[qids] - od) <= 1e-6 * sc)
    tex.destroy()


def test_full_size_sort(dev, workload):
    # the benchmark's 16M ray queries sorted by leaf Morton code: the stable
    # order of the keys (recomputed on the host) and the queries in that order
    import test_gpu_sort as ts
    grid, pts, _ = workload
    tex = stf.stf_create_sparse_grid3d(DIMS, stf.STF_FMT_F32, grid.origins, grid.values)
    q = torch.from_numpy(pts).to(dev)
    sq, order = stf.sort_queries(tex, q)
    o = order.cpu().numpy()
    keys = ts._keys3d(pts, DIMS)
    assert np.array_equal(o, np.argsort(keys, kind="stable"))
    assert np.array_equal(sq.cpu().numpy(), pts[o])
    tex.destroy()
