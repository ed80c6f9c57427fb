"""GPU parity: the HIP filters (through the C ABI) against the FP64 oracle on
identical seeded inputs.

Bar: stochastic mode -- the texel index equals the oracle's for every query
and the value is the decoded texel exactly; deterministic mode -- within
1e-6 of the oracle relative to sum_k |w_k t_k| (= |F| for the non-negative
texels used here), and exactly 0 where the oracle is 0."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_05810_amd as stf
import synth
from tests._util import leaves_from_dense

pytestmark = pytest.mark.gpu

FMTS = ["f32", "f16", "bf16", "fp8_e4m3", "u8"]
ORC_FMT = {"f32": oracle.F32, "f16": oracle.F16, "bf16": oracle.BF16, "fp8_e4m3": oracle.FP8_E4M3, "u8": oracle.U8}
FILTERS = [("linear", stf.STF_LINEAR, oracle.LINEAR), ("cubic", stf.STF_CUBIC_BSPLINE, oracle.CUBIC)]
REL = 1e-6


def _as_f32(x):
    return np.asarray(x, np.float64).astype(np.float32)


def check_stochastic(gv, gi, ov, oi, fmt, label):
    gv = gv.reshape(ov.shape)
    assert np.array_equal(gi, oi), f"{label}: {np.sum(np.any(gi != oi, axis=1))} index mismatches"
    ref = _as_f32(ov)   # exact for every format but u8, which the GPU rounds once from v/255
    same = (gv == ref) | (np.isnan(gv) & np.isnan(ref))
    assert same.all(), f"{label}: {np.sum(~same)} value mismatches"


def check_deterministic(gv, ov, label):
    gv = gv.reshape(ov.shape).astype(np.float64)
    both_nan = np.isnan(gv) & np.isnan(ov)
    err = np.abs(gv - ov)
    ok = both_nan | (err <= REL * np.abs(ov))
    worst = np.nanmax(np.where(ov != 0, err / np.abs(np.where(ov == 0, 1, ov)), 0))
    assert ok.all(), f"{label}: {np.sum(~ok)} outside 1e-6 (worst rel {worst:.3g})"
    return worst


# ----------------------------------------------------------------------------
# 2D textures: the 256x256 RGBA workload with 65,536 uniform queries
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def tex2d_inputs():
    tex = synth.texture2d(256, 256, 4, seed=1)
    uv = synth.uv_queries(65536, seed=2)
    uv[:64] = np.round(uv[:64] * 256 - 0.5) / 256 + np.float32(0.5 / 256)   # texel centres (t = 0)
    uv[64:80] = np.array([0.0, 1.0 - 2 ** -24], np.float32)[np.arange(16) % 2, None]  # borders
    uv[80:84] = [[np.nan, 0.5], [0.5, np.inf], [1e30, 0.5], [-0.7, 1.4]]
    return tex, uv


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("fname,gf,of", FILTERS)
def test_2d_parity(dev, tex2d_inputs, fmt, fname, gf, of):
    tex, uv = tex2d_inputs
    raw = synth.encode(tex, fmt)
    H, W, Cc = tex.shape
    t = stf.stf_create_texture2d(W, H, Cc, stf.FORMATS[fmt], [raw])
    q = torch.from_numpy(uv).to(dev)
    seed = 0x1234_5678_9ABC
    gv, gi = stf.filter(t, q, gf, stf.STF_STOCHASTIC, seed, want_index=True)
    ov, oi = oracle.filter2d(raw, ORC_FMT[fmt], uv, of, oracle.STOCH, seed)
    check_stochastic(gv.cpu().numpy(), gi.cpu().numpy(), ov, oi, fmt, f"2d {fmt} {fname} stoch")
    gd, _ = stf.filter(t, q, gf, stf.STF_DETERMINISTIC, 0)
    od, _ = oracle.filter2d(raw, ORC_FMT[fmt], uv, of, oracle.DET)
    check_deterministic(gd.cpu().numpy(), od, f"2d {fmt} {fname} det")
    t.destroy()


@pytest.mark.parametrize("fmt", ["fp8_e4m3", "u8"])
def test_2d_every_8bit_code(dev, fmt):
    # A 16 x 16 texture holding each of the 256 codes once (NaN codes
    # included), read at the texel centres: every decode against the
    # oracle's, bit for bit (NaN for NaN).
    raw = np.arange(256, dtype=np.uint8).reshape(16, 16, 1)
    t = stf.stf_create_texture2d(16, 16, 1, stf.FORMATS[fmt], [raw])
    ys, xs = np.mgrid[0:16, 0:16]
    uv = np.stack([(xs + 0.5) / 16, (ys + 0.5) / 16], axis=-1).reshape(-1, 2).astype(np.float32)
    gv, gi = stf.filter(t, torch.from_numpy(uv).to(dev), stf.STF_LINEAR, stf.STF_STOCHASTIC, 5, want_index=True)
    ov, oi = oracle.filter2d(raw, ORC_FMT[fmt], uv, oracle.LINEAR, oracle.STOCH, 5)
    check_stochastic(gv.cpu().numpy(), gi.cpu().numpy(), ov, oi, fmt, f"every {fmt} code")
    assert np.array_equal(oi[:, 1] * 16 + oi[:, 0], np.arange(256))   # each code read once
    t.destroy()


@pytest.mark.parametrize("channels", [1, 2, 3])
def test_2d_channel_counts(dev, channels):
    tex = synth.texture2d(40, 24, channels, seed=3)
    uv = synth.uv_queries(5000, seed=4) * np.float32(1.2) - np.float32(0.1)
    t = stf.stf_create_texture2d(40, 24, channels, stf.STF_FMT_F32, [tex])
    q = torch.from_numpy(uv).to(dev)
    for _, gf, of in FILTERS:
        gv, gi = stf.filter(t, q, gf, stf.STF_STOCHASTIC, 7, want_index=True)
        ov, oi = oracle.filter2d(tex, oracle.F32, uv, of, oracle.STOCH, 7)
        check_stochastic(gv.cpu().numpy(), gi.cpu().numpy(), ov, oi, "f32", f"2d c{channels}")
        gd, _ = stf.filter(t, q, gf, stf.STF_DETERMINISTIC, 0)
        od, _ = oracle.filter2d(tex, oracle.F32, uv, of, oracle.DET)
        check_deterministic(gd.cpu().numpy(), od, f"2d c{channels} det")
    t.destroy()


# ----------------------------------------------------------------------------
# 3D sparse grids: a small fBm grid with queries inside and outside the domain
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small_grid():
    g = synth.fbm_grid((64, 64, 64), base_period=16.0, seed=7)
    assert 0 < g.n_leaves < 512
    p = synth.uniform_box_queries(g.dims, 60000, seed=8, margin=3.0)
    p[:500] = np.round(p[:500])                                  # voxel centres (t = 0)
    p[500:510] = [[np.nan, 1, 1], [1, np.inf, 1], [1, 1, -np.inf], [1e9, 1, 1], [2 ** 24, 2, 2],
                  [-2.0 ** 24, 0, 0], [0, 0, 0], [63, 63, 63], [-0.5, -0.5, -0.5], [63.5, 63.5, 63.5]]
    return g, p


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("fname,gf,of", FILTERS)
def test_3d_parity(dev, small_grid, fmt, fname, gf, of):
    g, p = small_grid
    raw = g.encoded(fmt)
    t = stf.stf_create_sparse_grid3d(g.dims, stf.FORMATS[fmt], g.origins, raw)
    og = oracle.Grid(g.dims, ORC_FMT[fmt], g.origins, raw)
    q = torch.from_numpy(p).to(dev)
    seed = 99
    gv, gi = stf.filter(t, q, gf, stf.STF_STOCHASTIC, seed, want_index=True)
    ov, oi = og.filter(p, of, oracle.STOCH, seed)
    check_stochastic(gv.cpu().numpy(), gi.cpu().numpy(), ov, oi, fmt, f"3d {fmt} {fname} stoch")
    gd, _ = stf.filter(t, q, gf, stf.STF_DETERMINISTIC, 0)
    od, _ = og.filter(p, of, oracle.DET)
    check_deterministic(gd.cpu().numpy(), od, f"3d {fmt} {fname} det")
    t.destroy()


def test_3d_ragged_domain_and_background(dev):
    # a domain that is not a multiple of 8, a non-zero background and leaves
    # that stick out of the domain
    rng = np.random.default_rng(5)
    field = rng.random((16, 24, 24)).astype(np.float32)
    keep = rng.random((2, 3, 3)) < 0.7
    o, v = leaves_from_dense(field, keep)
    dims = (21, 19, 13)
    inside = (o[:, 0] < dims[0]) & (o[:, 1] < dims[1]) & (o[:, 2] < dims[2])
    o, v = o[inside], v[inside]
    t = stf.stf_create_sparse_grid3d(dims, stf.STF_FMT_F32, o, v, background=0.5)
    og = oracle.Grid(dims, oracle.F32, o, v, background=0.5)
    p = synth.uniform_box_queries(dims, 20000, seed=6, margin=3.0)
    q = torch.from_numpy(p).to(dev)
    for fname, gf, of in FILTERS:
        gv, gi = stf.filter(t, q, gf, stf.STF_STOCHASTIC, 5, want_index=True)
        ov, oi = og.filter(p, of, oracle.STOCH, 5)
        check_stochastic(gv.cpu().numpy(), gi.cpu().numpy(), ov, oi, "f32", f"ragged {fname}")
        gd, _ = stf.filter(t, q, gf, stf.STF_DETERMINISTIC, 0)
        od, _ = og.filter(p, of, oracle.DET)
        check_deterministic(gd.cpu().numpy(), od, f"ragged {fname} det")
    t.destroy()


@pytest.mark.parametrize("fmt", FMTS)
def test_3d_every_row_window_offset(dev, fmt):
    # The deterministic filter reads each row of taps as aligned chunks along
    # x; sweep the first tap over every offset within a leaf and across leaf
    # boundaries, next to missing leaves and a domain edge inside a leaf
    # (x = 29 of the 32 voxels the last leaves hold), with a background that
    # differs from every texel.
    rng = np.random.default_rng(11)
    field = rng.random((16, 16, 32)).astype(np.float32)   # (z, y, x)
    keep = rng.random((2, 2, 4)) < 0.75
    keep[0, 0, :] = True
    o, v = leaves_from_dense(field, keep)
    dims = (29, 16, 13)
    inside = (o[:, 0] < dims[0]) & (o[:, 1] < dims[1]) & (o[:, 2] < dims[2])
    o, v = o[inside], v[inside]
    raw = synth.encode(v, fmt)
    t = stf.stf_create_sparse_grid3d(dims, stf.FORMATS[fmt], o, raw, background=0.75)
    og = oracle.Grid(dims, ORC_FMT[fmt], o, raw, background=0.75)
    xs = np.arange(-3.0, 33.0, 0.125, dtype=np.float32)   # every cell offset, several t per cell
    yz = rng.random((xs.size * 8, 2)).astype(np.float32) * np.array([19.0, 16.0], np.float32) - 2.0
    p = np.stack([np.repeat(xs, 8), yz[:, 0], yz[:, 1]], axis=1).astype(np.float32)
    q = torch.from_numpy(p).to(dev)
    for fname, gf, of in FILTERS:
        gd, _ = stf.filter(t, q, gf, stf.STF_DETERMINISTIC, 0)
        od, _ = og.filter(p, of, oracle.DET)
        check_deterministic(gd.cpu().numpy(), od, f"row windows {fmt} {fname}")
    t.destroy()


def test_3d_empty_grid_reads_background(dev):
    t = stf.stf_create_sparse_grid3d((32, 32, 32), stf.STF_FMT_F32, np.zeros((0, 3), np.int32),
                                     np.zeros(0, np.float32), background=0.25)
    p = synth.uniform_box_queries((32, 32, 32), 1000, seed=1)
    q = torch.from_numpy(p).to(dev)
    for _, gf, _ in FILTERS:
        v, _ = stf.filter(t, q, gf, stf.STF_STOCHASTIC, 1)
        assert torch.all(v == 0.25)
        d, _ = stf.filter(t, q, gf, stf.STF_DETERMINISTIC, 0)
        assert torch.allclose(d, torch.full_like(d, 0.25), rtol=1e-6, atol=0)
    t.destroy()


def test_zero_queries_and_argument_errors(dev):
    g = synth.fbm_grid((32, 32, 32), base_period=8.0, seed=2)
    t = stf.stf_create_sparse_grid3d(g.dims, stf.STF_FMT_F32, g.origins, g.values)
    q0 = torch.empty((0, 3), dtype=torch.float32, device=dev)
    out0 = torch.empty((0, 1), dtype=torch.float32, device=dev)
    stf.stf_filter(t, q0, stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 0, out0)
    L = stf.lib()
    host = np.zeros((4, 3), np.float32)
    out = torch.empty((4, 1), dtype=torch.float32, device=dev)
    rc = L.stf_filter(t.handle, host.ctypes.data, 4, 1, 1, 0, out.data_ptr(), None, 0, None)
    assert rc == stf.STF_E_INVALID and "device" in stf.stf_last_error()
    q = torch.zeros((4, 3), dtype=torch.float32, device=dev)
    idx = torch.empty((4, 3), dtype=torch.int32, device=dev)
    rc = L.stf_filter(t.handle, q.data_ptr(), 4, 1, 0, 0, out.data_ptr(), idx.data_ptr(), 0, None)
    assert rc == stf.STF_E_INVALID
    rc = L.stf_filter(t.handle, q.data_ptr() + 2, 4, 1, 1, 0, out.data_ptr(), None, 0, None)
    assert rc == stf.STF_E_INVALID and "aligned" in stf.stf_last_error()
    rc = L.stf_filter(t.handle, q.data_ptr(), 4, 7, 1, 0, out.data_ptr(), None, 0, None)
    assert rc == stf.STF_E_INVALID
    t.destroy()


def test_repeatable_and_launch_independent(dev, small_grid):
    g, p = small_grid
    t = stf.stf_create_sparse_grid3d(g.dims, stf.STF_FMT_F32, g.origins, g.values)
    q = torch.from_numpy(p).to(dev)
    a, ia = stf.filter(t, q, stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 3, want_index=True)
    b, ib = stf.filter(t, q, stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 3, want_index=True)
    assert torch.equal(ia, ib) and torch.equal(a.nan_to_num(7), b.nan_to_num(7))
    # a sub-batch draws differently (query ids restart), a different seed too
    c, ic = stf.filter(t, q, stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 4, want_index=True)
    assert not torch.equal(ia, ic)
    t.destroy()


# ----------------------------------------------------------------------------
# unbiasedness: binary64 moments on the device over many seeds
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("fname,gf,of", FILTERS)
def test_moments_unbiased_5_sigma(dev, fname, gf, of):
    g = synth.fbm_grid((64, 64, 64), base_period=16.0, seed=7)
    t = stf.stf_create_sparse_grid3d(g.dims, stf.STF_FMT_F32, g.origins, g.values)
    og = oracle.Grid(g.dims, oracle.F32, g.origins, g.values)
    # queries within a voxel of positive density, so the estimator has variance
    rng = np.random.default_rng(3)
    leaf, vz, vy, vx = np.nonzero(g.values > 0)
    pick = rng.integers(0, leaf.size, 1024)
    vox = g.origins[leaf[pick]] + np.stack([vx[pick], vy[pick], vz[pick]], axis=1)
    p = (vox + rng.random((1024, 3)) * 2.0 - 1.0).astype(np.float32)
    q = torch.from_numpy(p).to(dev)
    K = 16384
    s1 = torch.empty(1024, dtype=torch.float64, device=dev)
    s2 = torch.empty_like(s1)
    stf.stf_filter_moments(t, q, gf, 1000, K, s1, s2)
    s1, s2 = s1.cpu().numpy(), s2.cpu().numpy()
    mean, var = og.moments(p, of)
    live = var > 1e-12
    assert live.sum() > 900
    z = (s1 / K - mean)[live] / np.sqrt(var[live] / K)
    assert np.all(np.abs(z) < 5.0), np.abs(z).max()
    # the device's second moment agrees with the exact variance too (in
    # aggregate: a single query's sample variance can be far off when one
    # tap of small probability carries a large value)
    v_hat = s2 / K - (s1 / K) ** 2
    ratio = v_hat[live] / var[live]
    assert 0.95 < np.median(ratio) < 1.05
    assert 0.95 < v_hat[live].sum() / var[live].sum() < 1.05
    t.destroy()


def test_moments_equal_sum_of_stochastic_calls(dev):
    g = synth.fbm_grid((32, 32, 32), base_period=8.0, seed=2)
    t = stf.stf_create_sparse_grid3d(g.dims, stf.STF_FMT_F32, g.origins, g.values)
    p = synth.uniform_box_queries(g.dims, 64, seed=9, margin=0.0)
    q = torch.from_numpy(p).to(dev)
    K = 300
    acc1 = np.zeros(64)
    acc2 = np.zeros(64)
    for k in range(K):
        v, _ = stf.filter(t, q, stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 50 + k)
        v = v.cpu().numpy()[:, 0].astype(np.float64)
        acc1 += v
        acc2 += v * v
    s1 = torch.empty(64, dtype=torch.float64, device=dev)
    s2 = torch.empty_like(s1)
    stf.stf_filter_moments(t, q, stf.STF_CUBIC_BSPLINE, 50, K, s1, s2)
    assert np.allclose(s1.cpu().numpy(), acc1, rtol=1e-13, atol=1e-13)
    assert np.allclose(s2.cpu().numpy(), acc2, rtol=1e-13, atol=1e-13)
    t.destroy()
