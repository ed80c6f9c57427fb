"""Edge cases of the filtering entry points on the GPU, through the C ABI:

- batch sizes that leave ragged tails in the kernels that give several
  queries to a thread (and a partial last block), with results equal to the
  oracle's and nothing written past the first n rows of the outputs;
- an empty batch for every entry point (a no-op that writes nothing);
- the binding's refusal of buffers of the wrong element type or size (the
  library sees raw pointers).

Bars as in the parity tests: stochastic indices exact and single-texel values
exact; deterministic values within 1e-6 of the oracle relative to
sum_k |w_k t_k|; positivized values within 1e-6 of S+|t(j+)| + S-|t(j-)|."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_05810_amd as stf
import synth
from tests.test_gpu_dct import _abs_terms

pytestmark = pytest.mark.gpu

RAGGED = [1, 2, 3, 5, 7, 255, 1021, 1027, 4099]
FILL = -7.25
GRID_FILTERS = [("linear", stf.STF_LINEAR, oracle.LINEAR), ("cubic", stf.STF_CUBIC_BSPLINE, oracle.CUBIC),
                ("keys", stf.STF_CUBIC_KEYS, oracle.KEYS), ("mitchell", stf.STF_CUBIC_MITCHELL, oracle.MITCHELL)]


def _padded(n, width, dtype, dev, fill):
    """A buffer of n + 16 rows filled with `fill`, and the view of its first n rows."""
    buf = torch.full((n + 16, width), fill, dtype=dtype, device=dev)
    return buf, buf[:n]


def _tail_ok(buf, n, fill):
    return bool(torch.all(buf[n:] == fill))


def _exact(gv, ov):
    ref = np.asarray(ov, np.float64).astype(np.float32)
    gv = gv.reshape(ref.shape)
    return np.all((gv == ref) | (np.isnan(gv) & np.isnan(ref)))


def _within(gv, ov, scale, rel=1e-6):
    ov = np.asarray(ov, np.float64)
    gv = gv.reshape(ov.shape).astype(np.float64)
    scale = np.asarray(scale, np.float64).reshape(ov.shape)
    both_nan = np.isnan(gv) & np.isnan(ov)
    return np.all(both_nan | (np.abs(gv - ov) <= rel * scale))


# ----------------------------------------------------------------------------
# 3D sparse grid
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def grid(dev):
    g = synth.fbm_grid((64, 64, 64), base_period=16.0, seed=21)
    t = stf.stf_create_sparse_grid3d(g.dims, stf.STF_FMT_F32, g.origins, g.values)
    og = oracle.Grid(g.dims, oracle.F32, g.origins, g.values)
    rng = np.random.default_rng(22)
    leaf, vz, vy, vx = np.nonzero(g.values > 0)
    pick = rng.integers(0, leaf.size, 4099)
    vox = g.origins[leaf[pick]] + np.stack([vx[pick], vy[pick], vz[pick]], axis=1)
    p = (vox + rng.random((4099, 3)) * 3.0 - 1.5).astype(np.float32)   # near active voxels
    p[::97] = synth.uniform_box_queries(g.dims, p[::97].shape[0], seed=23, margin=3.0)
    p[5] = [np.nan, 1.0, 1.0]
    yield g, t, og, p
    t.destroy()


def _grid_positivized_scale(og, of, p, oi):
    scale = np.zeros(p.shape[0])
    for k in range(p.shape[0]):
        if oi[k, 0] == oracle.BAD_INDEX:
            continue
        x = p[k].astype(np.float64)
        sp, sn = oracle.positivized_masses(of, list(x - np.floor(x)))
        s = sp * abs(og.texel(*oi[k, :3]))
        if oi[k, 3] != oracle.BAD_INDEX:
            s += sn * abs(og.texel(*oi[k, 3:]))
        scale[k] = s
    return scale


@pytest.mark.parametrize("n", RAGGED)
@pytest.mark.parametrize("fname,gf,of", GRID_FILTERS)
def test_grid_ragged_batches(dev, grid, n, fname, gf, of):
    g, t, og, p = grid
    pn = np.ascontiguousarray(p[:n])
    q = torch.from_numpy(pn).to(dev)
    iw = stf.index_width(gf, 3)
    seed = 0xE06E + n
    # stochastic
    ob, out = _padded(n, 1, torch.float32, dev, FILL)
    ib, idx = _padded(n, iw, torch.int32, dev, -99)
    stf.stf_filter(t, q, gf, stf.STF_STOCHASTIC, seed, out, idx)
    ov, oi = og.filter(pn, of, oracle.STOCH, seed)
    gi, gv = idx.cpu().numpy(), out.cpu().numpy()
    assert np.array_equal(gi, oi), f"{fname} n={n}: index mismatch"
    if of in oracle.POSITIVIZED:
        assert _within(gv, ov, _grid_positivized_scale(og, of, pn, oi)), f"{fname} n={n}: value"
    else:
        assert _exact(gv, ov), f"{fname} n={n}: value"
    assert _tail_ok(ob, n, FILL) and _tail_ok(ib, n, -99), f"{fname} n={n}: wrote past n"
    # deterministic
    ob, out = _padded(n, 1, torch.float32, dev, FILL)
    stf.stf_filter(t, q, gf, stf.STF_DETERMINISTIC, 0, out)
    od, _ = og.filter(pn, of, oracle.DET)
    scale, _ = og.filter(pn, of, oracle.DET_ABS)
    assert _within(out.cpu().numpy(), od, scale), f"{fname} n={n}: deterministic value"
    assert _tail_ok(ob, n, FILL)
    # filter importance sampling (B-spline family only)
    if of in (oracle.LINEAR, oracle.CUBIC):
        ob, out = _padded(n, 1, torch.float32, dev, FILL)
        ib, idx = _padded(n, 3, torch.int32, dev, -99)
        stf.stf_filter(t, q, gf, stf.STF_STOCHASTIC_FIS, seed, out, idx)
        fv, fi = og.filter(pn, of, oracle.STOCH_FIS, seed)
        assert np.array_equal(idx.cpu().numpy(), fi) and _exact(out.cpu().numpy(), fv), f"{fname} n={n}: FIS"
        assert _tail_ok(ob, n, FILL) and _tail_ok(ib, n, -99)


# ----------------------------------------------------------------------------
# 2D textures: three channels (results are not 16-byte rows), binary32
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def tex3c(dev):
    tex = synth.texture2d(40, 24, 3, seed=31)
    t = stf.stf_create_texture2d(40, 24, 3, stf.STF_FMT_F32, [tex])
    uv = synth.uv_queries(4099, seed=32) * np.float32(1.2) - np.float32(0.1)
    uv[3] = [np.inf, 0.5]
    yield tex, t, uv
    t.destroy()


def _tex_positivized_scale(tex, of, uv, oi):
    H, W, _ = tex.shape
    scale = np.zeros((uv.shape[0], tex.shape[2]))
    for k in range(uv.shape[0]):
        if oi[k, 0] == oracle.BAD_INDEX:
            continue
        x = np.float32(np.float32(uv[k, 0]) * np.float32(W)) - np.float32(0.5)
        y = np.float32(np.float32(uv[k, 1]) * np.float32(H)) - np.float32(0.5)
        tx, ty = float(x) - np.floor(float(x)), float(y) - np.floor(float(y))
        sp, sn = oracle.positivized_masses(of, [tx, ty])
        s = sp * np.abs(tex[oi[k, 1], oi[k, 0]].astype(np.float64))
        if oi[k, 2] != oracle.BAD_INDEX:
            s = s + sn * np.abs(tex[oi[k, 3], oi[k, 2]].astype(np.float64))
        scale[k] = s
    return scale


TEX_FILTERS = [("linear", stf.STF_LINEAR, oracle.LINEAR), ("cubic", stf.STF_CUBIC_BSPLINE, oracle.CUBIC),
               ("keys", stf.STF_CUBIC_KEYS, oracle.KEYS)]


@pytest.mark.parametrize("n", RAGGED)
@pytest.mark.parametrize("fname,gf,of", TEX_FILTERS)
def test_2d_ragged_batches(dev, tex3c, n, fname, gf, of):
    tex, t, uv = tex3c
    un = np.ascontiguousarray(uv[:n])
    q = torch.from_numpy(un).to(dev)
    iw = stf.index_width(gf, 2)
    seed = 0x2D + n
    ob, out = _padded(n, 3, torch.float32, dev, FILL)
    ib, idx = _padded(n, iw, torch.int32, dev, -99)
    stf.stf_filter(t, q, gf, stf.STF_STOCHASTIC, seed, out, idx)
    ov, oi = oracle.filter2d(tex, oracle.F32, un, of, oracle.STOCH, seed)
    assert np.array_equal(idx.cpu().numpy(), oi), f"{fname} n={n}: index mismatch"
    if of in oracle.POSITIVIZED:
        assert _within(out.cpu().numpy(), ov, _tex_positivized_scale(tex, of, un, oi)), f"{fname} n={n}: value"
    else:
        assert _exact(out.cpu().numpy(), ov), f"{fname} n={n}: value"
    assert _tail_ok(ob, n, FILL) and _tail_ok(ib, n, -99), f"{fname} n={n}: wrote past n"
    ob, out = _padded(n, 3, torch.float32, dev, FILL)
    stf.stf_filter(t, q, gf, stf.STF_DETERMINISTIC, 0, out)
    od, _ = oracle.filter2d(tex, oracle.F32, un, of, oracle.DET)
    scale, _ = oracle.filter2d(tex, oracle.F32, un, of, oracle.DET_ABS)
    assert _within(out.cpu().numpy(), od, scale), f"{fname} n={n}: deterministic value"
    assert _tail_ok(ob, n, FILL)


# ----------------------------------------------------------------------------
# DCT texture, nine channels; Gaussian and EWA entry points
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 3, 5, 1027])
def test_dct_gauss_ewa_ragged_batches(dev, n):
    rng = np.random.default_rng(41)
    u8 = rng.integers(0, 256, (40, 48, 9), dtype=np.uint8)
    words = stf.stf_dct_encode(u8)
    t = stf.stf_create_dct_texture2d(48, 40, 9, words)
    uv = np.ascontiguousarray(synth.uv_queries(n, seed=42))
    q = torch.from_numpy(uv).to(dev)
    ob, out = _padded(n, 9, torch.float32, dev, FILL)
    ib, idx = _padded(n, 2, torch.int32, dev, -99)
    stf.stf_filter(t, q, stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 5, out, idx)
    ov, oi = oracle.dct_filter2d(words, uv, oracle.CUBIC, oracle.STOCH, 5)
    assert np.array_equal(idx.cpu().numpy(), oi)
    A = _abs_terms(words)   # the decoded texel's absolute scale
    assert _within(out.cpu().numpy(), ov, A[oi[:, 1], oi[:, 0]])
    assert _tail_ok(ob, n, FILL) and _tail_ok(ib, n, -99)
    ob, out = _padded(n, 9, torch.float32, dev, FILL)
    ib, idx = _padded(n, 2, torch.int32, dev, -99)
    stf.stf_filter_gaussian(t, q, 0.5, stf.STF_GAUSS_DISCRETE, 6, out, idx)
    _, gi = oracle.dct_gauss_filter2d(words, uv, 0.5, oracle.G_DISCRETE, seed=6)
    assert np.array_equal(idx.cpu().numpy(), gi)
    assert _tail_ok(ob, n, FILL) and _tail_ok(ib, n, -99)
    t.destroy()
    # EWA over a small RGBA8 pyramid
    base = rng.integers(0, 256, (32, 48, 4), dtype=np.uint8)
    lv = synth.mip_levels(base)
    te = stf.stf_create_texture2d(48, 32, 4, stf.STF_FMT_U8, lv)
    qe = np.concatenate([rng.random((n, 2)), rng.normal(0, 0.03, (n, 4))], axis=1).astype(np.float32)
    qd = torch.from_numpy(qe).to(dev)
    ob, out = _padded(n, 4, torch.float32, dev, FILL)
    ib, idx = _padded(n, 3, torch.int32, dev, -99)
    stf.stf_filter_ewa(te, qd, 8.0, stf.STF_STOCHASTIC, 7, out, idx)
    ev, ei = oracle.ewa_filter2d(lv, oracle.U8, qe, 8.0, oracle.STOCH, seed=7)
    lod = oracle.ewa_lods(qe, len(lv), 8.0)
    with np.errstate(invalid="ignore"):
        edge = np.abs(lod - np.round(lod)) < 1e-9
    assert not np.any(np.any(idx.cpu().numpy() != ei, axis=1) & ~edge)
    assert _tail_ok(ob, n, FILL) and _tail_ok(ib, n, -99)
    te.destroy()


# ----------------------------------------------------------------------------
# empty batches
# ----------------------------------------------------------------------------
def test_empty_batches_are_no_ops(dev, grid, tex3c):
    _, tg, _, _ = grid
    _, t2, _ = tex3c
    q3 = torch.empty((0, 3), dtype=torch.float32, device=dev)
    q2 = torch.empty((0, 2), dtype=torch.float32, device=dev)
    for t, q, c in ((tg, q3, 1), (t2, q2, 3)):
        for gf in (stf.STF_LINEAR, stf.STF_CUBIC_BSPLINE, stf.STF_CUBIC_KEYS):
            for mode in (stf.STF_STOCHASTIC, stf.STF_DETERMINISTIC):
                ob, out = _padded(0, c, torch.float32, dev, FILL)
                stf.stf_filter(t, q, gf, mode, 1, out)
                assert _tail_ok(ob, 0, FILL)
        s1, s1v = _padded(0, 1, torch.float64, dev, FILL)
        s2, s2v = _padded(0, 1, torch.float64, dev, FILL)
        stf.stf_filter_moments(t, q, stf.STF_CUBIC_BSPLINE, 0, 16, s1v, s2v)
        assert _tail_ok(s1, 0, FILL) and _tail_ok(s2, 0, FILL)
    ob, out = _padded(0, 3, torch.float32, dev, FILL)
    stf.stf_filter_gaussian(t2, q2, 0.5, stf.STF_GAUSS_FIS, 1, out)
    assert _tail_ok(ob, 0, FILL)
    lv = synth.mip_levels(np.zeros((16, 16, 4), np.uint8))
    te = stf.stf_create_texture2d(16, 16, 4, stf.STF_FMT_U8, lv)
    ob, out = _padded(0, 4, torch.float32, dev, FILL)
    stf.stf_filter_ewa(te, torch.empty((0, 6), dtype=torch.float32, device=dev), 8.0, stf.STF_STOCHASTIC, 1, out)
    assert _tail_ok(ob, 0, FILL)
    te.destroy()
    sq, order = stf.sort_queries(tg, q3)
    assert sq.shape[0] == 0 and order.shape[0] == 0


# ----------------------------------------------------------------------------
# the binding refuses buffers the library would overrun
# ----------------------------------------------------------------------------
def test_binding_refuses_wrong_buffers(dev, grid):
    _, t, _, p = grid
    q = torch.from_numpy(np.ascontiguousarray(p[:64])).to(dev)
    ok = torch.empty((64, 1), dtype=torch.float32, device=dev)
    with pytest.raises(ValueError, match="float32"):
        stf.stf_filter(t, q, stf.STF_LINEAR, stf.STF_STOCHASTIC, 0, torch.empty((64, 1), dtype=torch.float16,
                                                                                device=dev))
    with pytest.raises(ValueError, match="int32"):
        stf.stf_filter(t, q, stf.STF_LINEAR, stf.STF_STOCHASTIC, 0, ok,
                       torch.empty((64, 3), dtype=torch.int64, device=dev))
    with pytest.raises(ValueError, match="needed"):
        stf.stf_filter(t, q, stf.STF_LINEAR, stf.STF_STOCHASTIC, 0, torch.empty((63, 1), device=dev))
    with pytest.raises(ValueError, match="needed"):
        stf.stf_filter(t, q, stf.STF_CUBIC_KEYS, stf.STF_STOCHASTIC, 0, ok,
                       torch.empty((64, 3), dtype=torch.int32, device=dev))   # positivized: 6 per query
    with pytest.raises(ValueError, match="per query"):
        stf.stf_filter(t, q[:, :2].contiguous(), stf.STF_LINEAR, stf.STF_STOCHASTIC, 0, ok)
    with pytest.raises(ValueError, match="float64"):
        stf.stf_filter_moments(t, q, stf.STF_LINEAR, 0, 4, torch.empty(64, dtype=torch.float32, device=dev),
                               torch.empty(64, dtype=torch.float64, device=dev))
    with pytest.raises(ValueError, match="contiguous"):
        stf.stf_filter(t, q, stf.STF_LINEAR, stf.STF_STOCHASTIC, 0, torch.empty((64, 2), device=dev)[:, :1])


# ----------------------------------------------------------------------------
# neural texture: batches that fill part of a 64-decode pair of MFMA batches
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 3, 31, 33, 65, 1027])
def test_neural_ragged_batches(dev, n):
    lat, mlp = synth.neural_init(16, seed=71)
    nt = stf.stf_ntex_create(64, 64, lat, mlp)
    stf.stf_ntex_prepare_inference(nt)
    on = oracle.NeuralTexture(np.asarray(lat, np.float32).astype(np.float16).astype(np.float64), mlp, 64, 64)
    uv = np.ascontiguousarray(synth.uv_queries(n, seed=72))
    q = torch.from_numpy(uv).to(dev)
    for gf, of in ((stf.STF_LINEAR, oracle.LINEAR), (stf.STF_CUBIC_BSPLINE, oracle.CUBIC)):
        ob, out = _padded(n, 8, torch.float32, dev, FILL)
        ib, idx = _padded(n, 2, torch.int32, dev, -99)
        stf.stf_ntex_filter(nt, q, gf, stf.STF_STOCHASTIC, 3, out, idx)
        ov, oi = on.filter(uv, of, oracle.STOCH, seed=3, emulate=True)
        assert np.array_equal(idx.cpu().numpy(), oi)
        assert np.abs(out.cpu().numpy() - ov).max() < 1e-2   # the bf16 inference bar of the neural parity test
        assert _tail_ok(ob, n, FILL) and _tail_ok(ib, n, -99)
        ob, out = _padded(n, 8, torch.float32, dev, FILL)
        stf.stf_ntex_filter(nt, q, gf, stf.STF_DETERMINISTIC, 0, out)
        od, _ = on.filter(uv, of, oracle.DET, emulate=True)
        assert np.abs(out.cpu().numpy() - od).max() < 1e-2
        assert _tail_ok(ob, n, FILL)
    nt.destroy()


def test_binding_launches_on_the_current_stream(dev, grid):
    # The binding reads torch's current stream as a raw handle; it must be the
    # stream torch itself reports, also inside a stream context, and a batch
    # launched there must be complete once that stream is synchronised.
    _, t, _, p = grid
    q = torch.from_numpy(np.ascontiguousarray(p[:4096])).to(dev)
    assert stf._stream(None) == torch.cuda.current_stream().cuda_stream
    ref = torch.empty((4096, 1), dtype=torch.float32, device=dev)
    stf.stf_filter(t, q, stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 5, ref)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    out = torch.full((4096, 1), -1.0, dtype=torch.float32, device=dev)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        assert stf._stream(None) == side.cuda_stream
        stf.stf_filter(t, q, stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 5, out)
    side.synchronize()
    assert torch.equal(torch.nan_to_num(out, nan=-7.0), torch.nan_to_num(ref, nan=-7.0))   # NaN for the fixture's non-finite queries
