"""Parity at the benchmark's full sizes for the 2D workloads, in the single
launches the benchmark times:

- the DCT-compressed 4096^2 x 9 texture set over a 3840x2160 frame
  (8,294,400 uv in pixel order): bilinear, bicubic and Keys, stochastic and
  deterministic (the deterministic cubics take the staged decode);
- Gaussian FIS and discrete 4x4 sampling (sigma 0.3 / 0.5 / 0.8) on the same
  set and frame, and the two Gaussian means;
- EWA over the full MIP pyramid of a 4096^2 RGBA8 texture for the frame's
  8,294,400 queries with derivatives, max anisotropy 8 and 64;
- the neural texture at 4096^2 x 8 with 1024^2 x 8 latents and 16,777,216
  uv queries, bilinear and bicubic, stochastic and deterministic.

The oracle recomputes 65,536 sampled queries of each batch as members of the
whole batch (a draw depends on the query's index).  Bars as in the small
tests: taps exact (Gaussian FIS and EWA: except within 1e-9 of a decision
boundary of the binary64 transcendental step), values within 1e-6 of the
oracle relative to their absolute scale (DCT: the scale of the decoded
texel's coefficient terms), neural values within 1e-2 of the bfloat16-
emulating oracle."""
import numpy as np
import pytest
import torch
from scipy import fft

import oracle
import paper_2305_05810_amd as stf
import synth

pytestmark = pytest.mark.gpu

SIZE, C = 4096, 9
NSAMPLE = 1 << 16
REL = 1e-6
ZZ = [(0, 0), (0, 1), (1, 0), (2, 0), (1, 1), (0, 2)]


def _sample(n, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, NSAMPLE, replace=False)).astype(np.int64)


@pytest.fixture(scope="module")
def texset():
    return synth.texture_set_u8(SIZE, seed=51)


@pytest.fixture(scope="module")
def frame():
    return synth.screen_uv_queries(3840, 2160, seed=53)


@pytest.fixture(scope="module")
def dct(texset):
    words = stf.stf_dct_encode(texset)
    t = stf.stf_create_dct_texture2d(SIZE, SIZE, C, words)
    yield words, t
    t.destroy()


def _basis():
    out = []
    for v, u in ZZ:
        e = np.zeros((8, 8))
        e[v, u] = 1.0
        out.append(np.abs(fft.idctn(e, type=2, norm="ortho")))   # [y, x]
    return out


BASIS = _basis()


def _abs_terms_at(words, x, y):
    """A(x, y, c) = sum_k |dequantised coefficient k| |basis_k(x mod 8, y mod 8)|
    of the texels (x, y) (clamped coordinates), shape (m, C): the absolute
    scale of a binary32 decode."""
    basis = BASIS
    w = words[y // 8, x // 8].astype(np.int64)                      # (m, C)
    deq = [(w & 127) * 8 / 127] + [(((w >> (7 + 5 * (k - 1))) & 31) - 16) * 2 / 15 for k in range(1, 6)]
    out = np.zeros(w.shape)
    for k in range(6):
        out += np.abs(deq[k]) * basis[k][y % 8, x % 8][:, None]
    return out


def _raster(uv):
    x = (uv[:, 0] * np.float32(SIZE) - np.float32(0.5)).astype(np.float32)
    y = (uv[:, 1] * np.float32(SIZE) - np.float32(0.5)).astype(np.float32)
    return x, y


def _det_scale(words, uv, of):
    """sum over the taps of |w| A(tap) for the deterministic filters."""
    x, y = _raster(uv)
    ix, iy = np.floor(x).astype(np.int64), np.floor(y).astype(np.int64)
    tx, ty = x.astype(np.float64) - ix, y.astype(np.float64) - iy
    nt, base = (2, 0) if of == oracle.LINEAR else (4, -1)
    scale = np.zeros((uv.shape[0], C))
    wx = np.array([oracle.axis_weights(of, t) for t in tx])
    wy = np.array([oracle.axis_weights(of, t) for t in ty])
    for b in range(nt):
        for a in range(nt):
            sx = np.clip(ix + base + a, 0, SIZE - 1)
            sy = np.clip(iy + base + b, 0, SIZE - 1)
            scale += np.abs(wx[:, a] * wy[:, b])[:, None] * _abs_terms_at(words, sx, sy)
    return scale


DCT_FILTERS = [("linear", stf.STF_LINEAR, oracle.LINEAR), ("bspline", stf.STF_CUBIC_BSPLINE, oracle.CUBIC),
               ("keys", stf.STF_CUBIC_KEYS, oracle.KEYS)]


@pytest.mark.parametrize("fname,gf,of", DCT_FILTERS)
def test_dct_frame_full_size(dev, dct, frame, fname, gf, of):
    words, t = dct
    n = frame.shape[0]
    q = torch.from_numpy(frame).to(dev)
    qids = _sample(n, 61)
    uvs = frame[qids]
    out = torch.empty((n, C), dtype=torch.float32, device=dev)
    idx = torch.empty((n, oracle.index_width(of, 2)), dtype=torch.int32, device=dev)
    stf.stf_filter(t, q, gf, stf.STF_STOCHASTIC, 0xF00D, out, idx)
    gv = out.cpu().numpy()[qids].astype(np.float64)
    gi = idx.cpu().numpy()[qids]
    ov, oi = oracle.dct_filter2d(words, frame, of, oracle.STOCH, 0xF00D, qids=qids)
    assert np.array_equal(gi, oi), int(np.any(gi != oi, axis=1).sum())
    scale = _abs_terms_at(words, oi[:, 0].astype(np.int64), oi[:, 1].astype(np.int64))
    if of in oracle.POSITIVIZED:
        x, y = _raster(uvs)
        masses = np.array([oracle.positivized_masses(of, [float(x[k]) - float(np.floor(x[k])),
                                                          float(y[k]) - float(np.floor(y[k]))])
                           for k in range(NSAMPLE)])
        scale *= masses[:, :1]
        neg = oi[:, 2] != oracle.BAD_INDEX
        scale[neg] += masses[neg, 1:] * _abs_terms_at(words, oi[neg, 2].astype(np.int64), oi[neg, 3].astype(np.int64))
    assert np.all(np.abs(gv - ov) <= REL * scale), np.max(np.abs(gv - ov) / np.maximum(scale, 1e-30))
    stf.stf_stage_counting(True)
    stf.stf_filter(t, q, gf, stf.STF_DETERMINISTIC, 0, out)
    staged, blocks = stf.stf_stage_counts()
    stf.stf_stage_counting(False)
    if gf != stf.STF_LINEAR:   # the frame's blocks decode their tap boxes once (bilinear: per tap)
        assert blocks == (n + 255) // 256 and staged > blocks // 2, (staged, blocks)
    gd = out.cpu().numpy()[qids].astype(np.float64)
    od, _ = oracle.dct_filter2d(words, frame, of, oracle.DET, qids=qids)
    dscale = _det_scale(words, uvs, of)
    err = np.abs(gd - od)
    assert np.all(err <= REL * dscale), np.max(err / np.maximum(dscale, 1e-30))


@pytest.mark.parametrize("sigma", [0.3, 0.5, 0.8])
def test_gaussian_frame_full_size(dev, dct, frame, sigma):
    sigma = float(np.float32(sigma))   # the call takes binary32 sigma: the oracle gets the same value
    words, t = dct
    n = frame.shape[0]
    q = torch.from_numpy(frame).to(dev)
    qids = _sample(n, 62)
    uvs = frame[qids]
    out = torch.empty((n, C), dtype=torch.float32, device=dev)
    idx = torch.empty((n, 2), dtype=torch.int32, device=dev)
    # FIS: taps equal except within 1e-9 of a texel edge, values the decoded texel
    stf.stf_filter_gaussian(t, q, sigma, stf.STF_GAUSS_FIS, 91, out, idx)
    gi = idx.cpu().numpy()[qids]
    gv = out.cpu().numpy()[qids].astype(np.float64)
    ov, oi = oracle.dct_gauss_filter2d(words, frame, sigma, oracle.G_FIS, 91, qids=qids)
    pos = oracle.gauss_fis_positions(SIZE, SIZE, frame, sigma, 91, qids=qids)
    near = np.any((np.abs(pos - (np.floor(pos + 0.5) - 0.5)) < 1e-9) |
                  (np.abs(pos - (np.floor(pos + 0.5) + 0.5)) < 1e-9), axis=1)
    diff = np.any(gi != oi, axis=1)
    assert not np.any(diff & ~near), int(diff.sum())
    same = ~diff
    A = _abs_terms_at(words, oi[:, 0].astype(np.int64), oi[:, 1].astype(np.int64))
    assert np.all(np.abs(gv - ov)[same] <= REL * A[same])
    # discrete 4x4 sampling: taps exact
    stf.stf_filter_gaussian(t, q, sigma, stf.STF_GAUSS_DISCRETE, 92, out, idx)
    _, oi = oracle.dct_gauss_filter2d(words, frame, sigma, oracle.G_DISCRETE, 92, qids=qids)
    assert np.array_equal(idx.cpu().numpy()[qids], oi)
    # the means: within 1e-6 of the largest absolute scale A in the window
    # (the weights are non-negative and sum to at most 1, so sum w A <= max A)
    x, y = _raster(uvs)
    ix, iy = np.floor(x).astype(np.int64), np.floor(y).astype(np.int64)
    for gm, om, R in ((stf.STF_GAUSS_DISCRETE_MEAN, oracle.G_DISCRETE_MEAN, None),
                      (stf.STF_GAUSS_FIS_MEAN, oracle.G_FIS_MEAN, oracle.lib().orc_gauss_radius(sigma))):
        stf.stf_filter_gaussian(t, q, sigma, gm, 0, out)
        gd = out.cpu().numpy()[qids].astype(np.float64)
        od, _ = oracle.dct_gauss_filter2d(words, frame, sigma, om, qids=qids)
        # discrete: the 4x4 window; FIS mean: the oracle sums |k - floor(x)| <= R,
        # the kernel one more column and row (weights below 2e-9 of the total)
        offs = range(-1, 3) if R is None else range(-R - 1, R + 2)
        amax = np.zeros((NSAMPLE, C))
        for b in offs:
            for a in offs:
                sx, sy = np.clip(ix + a, 0, SIZE - 1), np.clip(iy + b, 0, SIZE - 1)
                amax = np.maximum(amax, _abs_terms_at(words, sx, sy))
        err = np.abs(gd - od)
        assert np.all(err <= REL * amax), (gm, np.max(err / np.maximum(amax, 1e-30)))


@pytest.fixture(scope="module")
def ewa_inputs(texset):
    rgba = np.ascontiguousarray(texset[:, :, :4])
    lv = synth.mip_levels(rgba)
    t = stf.stf_create_texture2d(SIZE, SIZE, 4, stf.STF_FMT_U8, lv)
    q = synth.screen_ewa_queries(3840, 2160, seed=53)
    yield lv, t, q
    t.destroy()


@pytest.mark.parametrize("aniso", [8.0, 64.0])
def test_ewa_frame_full_size(dev, ewa_inputs, aniso):
    lv, t, qn = ewa_inputs
    n = qn.shape[0]
    qids = _sample(n, 63)
    q = torch.from_numpy(qn).to(dev)
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    idx = torch.empty((n, 3), dtype=torch.int32, device=dev)
    stf.stf_filter_ewa(t, q, aniso, stf.STF_STOCHASTIC, 9, out, idx)
    gi = idx.cpu().numpy()[qids]
    gv = out.cpu().numpy()[qids]
    ov, oi = oracle.ewa_filter2d(lv, oracle.U8, qn, aniso, oracle.STOCH, seed=9, qids=qids)
    lod = oracle.ewa_lods(qn[qids], len(lv), aniso)
    edge = np.abs(lod - np.round(lod)) < 1e-9
    diff = np.any(gi != oi, axis=1)
    assert not np.any(diff & ~edge), int(diff.sum())
    assert np.array_equal(gv[~diff], ov[~diff].astype(np.float32))
    stf.stf_filter_ewa(t, q, aniso, stf.STF_DETERMINISTIC, 0, out)
    gd = out.cpu().numpy()[qids].astype(np.float64)
    od, _ = oracle.ewa_filter2d(lv, oracle.U8, qn, aniso, oracle.DET, qids=qids)
    err = np.abs(gd - od)
    assert np.all(err <= REL * np.abs(od) + 1e-12), np.max(err / np.maximum(np.abs(od), 1e-30))


def _f16(x):
    return np.asarray(x, np.float32).astype(np.float16).astype(np.float64)


@pytest.fixture(scope="module")
def neural_inputs(dev):
    lat, mlp = synth.neural_init(SIZE // 4, seed=42)
    rng = np.random.default_rng(44)
    for a, b in ((512, 576), (4672, 4736), (5248, 5256)):   # biases b1, b2, b3: non-zero
        mlp[a:b] = rng.normal(0.0, 0.1, b - a).astype(np.float32)
    nt = stf.stf_ntex_create(SIZE, SIZE, lat, mlp)
    stf.stf_ntex_prepare_inference(nt)
    glat, gmlp = stf.stf_ntex_get_params(nt)
    on = oracle.NeuralTexture(_f16(glat), gmlp, SIZE, SIZE)
    uv = synth.neural_queries(1 << 24, seed=43)
    yield nt, on, uv
    nt.destroy()


@pytest.mark.parametrize("fname,gf,of", [("linear", stf.STF_LINEAR, oracle.LINEAR),
                                         ("cubic", stf.STF_CUBIC_BSPLINE, oracle.CUBIC)])
def test_neural_full_size(dev, neural_inputs, fname, gf, of):
    nt, on, uv = neural_inputs
    n = uv.shape[0]
    qids = _sample(n, 64)
    q = torch.from_numpy(uv).to(dev)
    out = torch.empty((n, 8), dtype=torch.float32, device=dev)
    idx = torch.empty((n, 2), dtype=torch.int32, device=dev)
    stf.stf_ntex_filter(nt, q, gf, stf.STF_STOCHASTIC, 3, out, idx)
    gi = idx.cpu().numpy()[qids]
    g = out.cpu().numpy()[qids].astype(np.float64)
    ov, oi = on.filter(uv, of, oracle.STOCH, seed=3, qids=qids, emulate=True)
    assert np.array_equal(gi, oi)
    err = np.abs(g - ov)
    print(f"neural {fname} stochastic at 16M: max abs {err.max():.3g}")
    assert err.max() < 1e-2
    stf.stf_ntex_filter(nt, q, gf, stf.STF_DETERMINISTIC, 0, out)
    g = out.cpu().numpy()[qids].astype(np.float64)
    od, _ = on.filter(uv, of, oracle.DET, qids=qids, emulate=True)
    err = np.abs(g - od)
    print(f"neural {fname} deterministic at 16M: max abs {err.max():.3g}")
    assert err.max() < 1e-2
