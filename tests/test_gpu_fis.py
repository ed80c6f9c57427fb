"""GPU parity of filter importance sampling and the Gaussian filters
through the C ABI against the FP64 oracle.

Bar: FIS of the tent / cubic B-spline -- taps and values exactly equal to the
oracle's (the tap is the binary64 floor(x + s + 1/2) on both sides; the
kernels form it in binary32 and integers where that sum is exact, |x| >=
2^-29); Gaussian FIS and discrete sampling -- taps equal to the oracle's
except where the oracle's binary64 sample lies
within 1e-9 of a decision boundary (transcendental functions round
differently on the two sides), values the texel at the tap; Gaussian means --
within 1e-6 of the oracle relative to sum |w t| (= the value here: weights
and texels are non-negative)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_05810_amd as stf
import synth

pytestmark = pytest.mark.gpu

SIGMAS = [0.2, 0.3, 0.5, 0.8, 2.5]   # 0.2 < 1/4: the discrete draw is binary64 only


@pytest.fixture(scope="module")
def tex_inputs():
    tex = synth.texture2d(72, 56, 4, seed=41)
    uv = synth.uv_queries(30000, seed=42) * np.float32(1.1) - np.float32(0.05)
    uv[:4] = [[np.nan, 0.5], [0.5, np.inf], [1e30, 0.5], [-0.7, 1.4]]
    # raster positions near 0 (x = u 72 - 1/2): below 2^-29 the draw's binary64
    # sum rounds x, at and above it the kernels take their exact integer path
    h = np.float32(0.5 / 72)
    uv[4:10, 0] = [h, np.nextafter(h, np.float32(0)), np.nextafter(h, np.float32(1)),
                   h * np.float32(1 + 2 ** -20), h * np.float32(1 - 2 ** -20), h * np.float32(1 + 2 ** -10)]
    return tex, uv.astype(np.float32)


@pytest.mark.parametrize("gf,of", [(stf.STF_LINEAR, oracle.LINEAR), (stf.STF_CUBIC_BSPLINE, oracle.CUBIC)])
def test_fis_bspline_family_2d_and_3d(dev, tex_inputs, gf, of):
    tex, uv = tex_inputs
    t = stf.stf_create_texture2d(72, 56, 4, stf.STF_FMT_F32, [tex])
    gv, gi = stf.filter(t, torch.from_numpy(uv).to(dev), gf, stf.STF_STOCHASTIC_FIS, 77, want_index=True)
    ov, oi = oracle.filter2d(tex, oracle.F32, uv, of, oracle.STOCH_FIS, 77)
    assert np.array_equal(gi.cpu().numpy(), oi)
    gv = gv.cpu().numpy()
    assert np.array_equal(np.nan_to_num(gv, nan=-1), np.nan_to_num(ov.astype(np.float32), nan=-1))
    t.destroy()
    g = synth.fbm_grid((64, 64, 64), base_period=16.0, seed=7)
    p = synth.uniform_box_queries(g.dims, 30000, seed=43, margin=3.0)
    p[:3] = [[np.nan, 1, 1], [1e9, 1, 1], [-0.5, -0.5, -0.5]]
    # coordinates near 0, on both sides of 2^-29 (the exact integer path's bound)
    tiny = np.array([1e-30, -1e-30, 2.0 ** -30, -2.0 ** -30, 2.0 ** -29, -2.0 ** -29, 3e-9, -3e-9, -1e-6, 0.0, -0.0,
                     -2.0 ** -29 * (1 + 2.0 ** -23)], np.float32)
    p[3:3 + 3 * len(tiny)] = np.repeat(tiny[:, None], 3, axis=1).repeat(3, axis=0)
    tg = stf.stf_create_sparse_grid3d(g.dims, stf.STF_FMT_F32, g.origins, g.values)
    og = oracle.Grid(g.dims, oracle.F32, g.origins, g.values)
    q = torch.from_numpy(p).to(dev)
    gv, gi = stf.filter(tg, q, gf, stf.STF_STOCHASTIC_FIS, 78, want_index=True)
    ov, oi = og.filter(p, of, oracle.STOCH_FIS, 78)
    assert np.array_equal(gi.cpu().numpy(), oi)
    gv = gv.cpu().numpy()[:, 0]
    assert np.array_equal(np.nan_to_num(gv, nan=-1), np.nan_to_num(ov.astype(np.float32), nan=-1))
    # ordered stream: same results bit for bit
    sq, order = stf.sort_queries(tg, q)
    out = torch.empty((p.shape[0], 1), dtype=torch.float32, device=dev)
    idx = torch.empty((p.shape[0], 3), dtype=torch.int32, device=dev)
    stf.stf_filter_ordered(tg, sq, order, gf, stf.STF_STOCHASTIC_FIS, 78, out, idx, stf.STF_ORDER_SCATTER)
    assert np.array_equal(idx.cpu().numpy(), oi)
    tg.destroy()


def test_fis_on_dct_texture(dev):
    rng = np.random.default_rng(5)
    tex8 = rng.integers(0, 256, (64, 48, 9), dtype=np.uint8)
    words = stf.stf_dct_encode(tex8)
    t = stf.stf_create_dct_texture2d(48, 64, 9, words)
    uv = synth.uv_queries(20000, seed=44)
    gv, gi = stf.filter(t, torch.from_numpy(uv).to(dev), stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC_FIS, 5,
                        want_index=True)
    ov, oi = oracle.dct_filter2d(words, uv, oracle.CUBIC, oracle.STOCH_FIS, 5)
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.allclose(gv.cpu().numpy(), ov, rtol=0, atol=4e-6)   # binary32 decode of |values| <= ~3.5
    t.destroy()


@pytest.mark.parametrize("sigma", SIGMAS)
def test_gaussian_modes(dev, tex_inputs, sigma):
    tex, uv = tex_inputs
    sigma = float(np.float32(sigma))   # the call takes binary32 sigma: the oracle gets the same value
    t = stf.stf_create_texture2d(72, 56, 4, stf.STF_FMT_F32, [tex])
    q = torch.from_numpy(uv).to(dev)
    n = uv.shape[0]
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    idx = torch.empty((n, 2), dtype=torch.int32, device=dev)
    # FIS: taps equal except within 1e-9 of a boundary
    stf.stf_filter_gaussian(t, q, sigma, stf.STF_GAUSS_FIS, 91, out, idx)
    ov, oi = oracle.gauss_filter2d(tex, oracle.F32, uv, sigma, oracle.G_FIS, 91)
    gi = idx.cpu().numpy()
    pos = oracle.gauss_fis_positions(72, 56, uv, sigma, 91)
    with np.errstate(invalid="ignore"):   # non-finite queries have non-finite positions
        near = np.abs(pos - (np.floor(pos + 0.5) - 0.5)) < 1e-9
        near |= np.abs(pos - (np.floor(pos + 0.5) + 0.5)) < 1e-9
    diff = np.any(gi != oi, axis=1)
    assert not np.any(diff & ~np.any(near, axis=1)), int(diff.sum())
    gv = out.cpu().numpy()
    same = ~diff
    assert np.array_equal(np.nan_to_num(gv[same], nan=-1), np.nan_to_num(ov[same].astype(np.float32), nan=-1))
    # discrete 4x4 sampling
    stf.stf_filter_gaussian(t, q, sigma, stf.STF_GAUSS_DISCRETE, 92, out, idx)
    ov, oi = oracle.gauss_filter2d(tex, oracle.F32, uv, sigma, oracle.G_DISCRETE, 92)
    assert np.array_equal(idx.cpu().numpy(), oi)
    assert np.array_equal(np.nan_to_num(out.cpu().numpy(), nan=-1), np.nan_to_num(ov.astype(np.float32), nan=-1))
    # the two means
    for gm, om in ((stf.STF_GAUSS_DISCRETE_MEAN, oracle.G_DISCRETE_MEAN), (stf.STF_GAUSS_FIS_MEAN, oracle.G_FIS_MEAN)):
        if gm == stf.STF_GAUSS_FIS_MEAN and sigma > 4:
            continue
        stf.stf_filter_gaussian(t, q, sigma, gm, 0, out)
        od, _ = oracle.gauss_filter2d(tex, oracle.F32, uv, sigma, om)
        gd = out.cpu().numpy().astype(np.float64)
        err = np.abs(gd - od)
        ok = (np.isnan(gd) & np.isnan(od)) | (err <= 1e-6 * np.abs(od) + 1e-12)
        assert ok.all(), (gm, np.nanmax(err / np.maximum(np.abs(od), 1e-30)))
    t.destroy()


@pytest.mark.parametrize("sigma", [0.2, 0.8, 2.5])
def test_gaussian_taps_at_scale(dev, sigma):
    sigma = float(np.float32(sigma))   # the call takes binary32 sigma: the oracle gets the same value
    # 4M queries on a small texture, so the draws that are redone in binary64
    # (FIS: samples within sigma 2^-14 of a texel edge; discrete: u * total
    # within total 2^-12 of a cumulative sum, or every draw for sigma < 1/4)
    # occur hundreds to thousands of times; every tap must equal the
    # oracle's binary64 decision except within 1e-9 of a boundary.
    rng = np.random.default_rng(int(sigma * 100))
    tex = rng.random((48, 40, 1)).astype(np.float32)
    n = 1 << 22
    uv = rng.random((n, 2), dtype=np.float32)
    t = stf.stf_create_texture2d(40, 48, 1, stf.STF_FMT_F32, [tex])
    q = torch.from_numpy(uv).to(dev)
    out = torch.empty((n, 1), dtype=torch.float32, device=dev)
    idx = torch.empty((n, 2), dtype=torch.int32, device=dev)
    stf.stf_filter_gaussian(t, q, sigma, stf.STF_GAUSS_FIS, 17, out, idx)
    _, oi = oracle.gauss_filter2d(tex, oracle.F32, uv, sigma, oracle.G_FIS, 17)
    pos = oracle.gauss_fis_positions(40, 48, uv, sigma, 17)
    dist = np.abs(pos - (np.floor(pos + 0.5) + 0.5))
    dist = np.minimum(dist, np.abs(pos - (np.floor(pos + 0.5) - 0.5)))
    redone = np.any(dist < sigma * 2.0 ** -14, axis=1)
    assert redone.sum() >= 100, int(redone.sum())        # the binary64 branch ran (about 1000 sigma times)
    diff = np.any(idx.cpu().numpy() != oi, axis=1)
    assert not np.any(diff & ~np.any(dist < 1e-9, axis=1)), int(diff.sum())
    stf.stf_filter_gaussian(t, q, sigma, stf.STF_GAUSS_DISCRETE, 18, out, idx)
    _, oi = oracle.gauss_filter2d(tex, oracle.F32, uv, sigma, oracle.G_DISCRETE, 18)
    assert np.array_equal(idx.cpu().numpy(), oi)
    t.destroy()


def test_gaussian_argument_errors(dev):
    t = stf.stf_create_texture2d(16, 16, 1, stf.STF_FMT_F32, [np.zeros((16, 16, 1), np.float32)])
    q = torch.zeros((4, 2), dtype=torch.float32, device=dev)
    out = torch.empty((4, 1), dtype=torch.float32, device=dev)
    idx = torch.empty((4, 2), dtype=torch.int32, device=dev)
    L = stf.lib()
    assert L.stf_filter_gaussian(t.handle, q.data_ptr(), 4, 0.0, 0, 0, out.data_ptr(), None, None) == stf.STF_E_INVALID
    assert L.stf_filter_gaussian(t.handle, q.data_ptr(), 4, 17.0, 0, 0, out.data_ptr(), None, None) == stf.STF_E_INVALID
    assert L.stf_filter_gaussian(t.handle, q.data_ptr(), 4, 5.0, 1, 0, out.data_ptr(), None, None) == stf.STF_E_UNSUPPORTED
    assert L.stf_filter_gaussian(t.handle, q.data_ptr(), 4, 1.0, 3, 0, out.data_ptr(), idx.data_ptr(),
                                 None) == stf.STF_E_INVALID
    assert L.stf_filter(t.handle, q.data_ptr(), 4, stf.STF_CUBIC_KEYS, stf.STF_STOCHASTIC_FIS, 0, out.data_ptr(), None,
                        0, None) == stf.STF_E_INVALID
    t.destroy()
