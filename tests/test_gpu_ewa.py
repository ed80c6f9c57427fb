"""GPU parity of EWA filtering over a MIP pyramid through the C ABI against
the FP64 oracle.

Bar: stochastic -- (x, y, level) equal to the oracle's for every query
(the ellipse and the tap draw are pinned binary32; the level decision goes
through log2 in binary64, so a query whose binary64 lod lies within 1e-9 of
an integer, or whose level uniform lies within 1e-9 of the fractional part,
may differ -- none does in practice) and the value is the texel; deterministic
-- within 1e-6 of the oracle relative to the value (weights and texels are
non-negative here)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_05810_amd as stf
import synth

pytestmark = pytest.mark.gpu


def _queries(n, seed, res):
    rng = np.random.default_rng(seed)
    st = rng.random((n, 2))
    ang = rng.random(n) * np.pi
    a = 2.0 ** rng.uniform(-2, 4, n) / res
    r = 2.0 ** rng.uniform(0, 4, n)
    d0 = np.stack([a * r * np.cos(ang), a * r * np.sin(ang)], axis=1)
    d1 = np.stack([-a * np.sin(ang), a * np.cos(ang)], axis=1)
    q = np.concatenate([st, d0, d1], axis=1).astype(np.float32)
    q[:4, 2:] = 0.0                                   # degenerate footprints
    q[4] = [np.nan, 0.5, 0.01, 0, 0, 0.01]
    q[5] = [0.5, 0.5, 1e6, 0, 0, 0.01]
    return q


@pytest.mark.parametrize("fmt", ["f32", "u8"])
@pytest.mark.parametrize("aniso", [1.0, 8.0, 64.0])
def test_ewa_parity(dev, fmt, aniso):
    rng = np.random.default_rng(1)
    base = rng.random((128, 96, 4)).astype(np.float32)
    tex = synth.encode(base, fmt)
    lv = synth.mip_levels(tex)
    t = stf.stf_create_texture2d(96, 128, 4, stf.FORMATS[fmt], lv)
    ofmt = {"f32": oracle.F32, "u8": oracle.U8}[fmt]
    q = _queries(20000, 2, 96.0)
    qd = torch.from_numpy(q).to(dev)
    n = q.shape[0]
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    idx = torch.empty((n, 3), dtype=torch.int32, device=dev)
    stf.stf_filter_ewa(t, qd, aniso, stf.STF_STOCHASTIC, 7, out, idx)
    ov, oi = oracle.ewa_filter2d(lv, ofmt, q, aniso, oracle.STOCH, seed=7)
    gi = idx.cpu().numpy()
    lod = oracle.ewa_lods(q, len(lv), aniso)
    with np.errstate(invalid="ignore"):
        edge = np.abs(lod - np.round(lod)) < 1e-9
    diff = np.any(gi != oi, axis=1)
    assert not np.any(diff & ~edge), int(diff.sum())
    gv = out.cpu().numpy()
    same = ~diff
    assert np.array_equal(np.nan_to_num(gv[same], nan=-1), np.nan_to_num(ov[same].astype(np.float32), nan=-1))
    stf.stf_filter_ewa(t, qd, aniso, stf.STF_DETERMINISTIC, 0, out)
    od, _ = oracle.ewa_filter2d(lv, ofmt, q, aniso, oracle.DET)
    gd = out.cpu().numpy().astype(np.float64)
    err = np.abs(gd - od)
    ok = (np.isnan(gd) & np.isnan(od)) | (err <= 1e-6 * np.abs(od) + 1e-12)
    assert ok.all(), np.nanmax(err / np.maximum(np.abs(od), 1e-30))
    t.destroy()


def test_ewa_argument_errors(dev):
    lv = synth.mip_levels(np.zeros((8, 8, 1), np.float32))
    t = stf.stf_create_texture2d(8, 8, 1, stf.STF_FMT_F32, lv)
    q = torch.zeros((4, 6), dtype=torch.float32, device=dev)
    out = torch.empty((4, 1), dtype=torch.float32, device=dev)
    idx = torch.empty((4, 3), dtype=torch.int32, device=dev)
    L = stf.lib()
    assert L.stf_filter_ewa(t.handle, q.data_ptr(), 4, 8.0, 0, 0, out.data_ptr(), None, None) == stf.STF_OK
    assert L.stf_filter_ewa(t.handle, q.data_ptr(), 4, 0.5, 0, 0, out.data_ptr(), None, None) == stf.STF_E_INVALID
    assert L.stf_filter_ewa(t.handle, q.data_ptr(), 4, 65.0, 0, 0, out.data_ptr(), None, None) == stf.STF_E_INVALID
    assert L.stf_filter_ewa(t.handle, q.data_ptr(), 4, 8.0, 0, 0, out.data_ptr(), idx.data_ptr(), None) == stf.STF_E_INVALID
    assert L.stf_filter_ewa(t.handle, q.data_ptr(), 4, 8.0, 5, 0, out.data_ptr(), None, None) == stf.STF_E_INVALID
    host = np.zeros((4, 6), np.float32)
    assert L.stf_filter_ewa(t.handle, host.ctypes.data, 4, 8.0, 0, 0, out.data_ptr(), None, None) == stf.STF_E_INVALID
    torch.cuda.synchronize()
    t.destroy()
    # a pyramid that stops before 1x1 is refused
    short = stf.stf_create_texture2d(8, 8, 1, stf.STF_FMT_F32, lv[:2])
    assert L.stf_filter_ewa(short.handle, q.data_ptr(), 4, 8.0, 0, 0, out.data_ptr(), None, None) == stf.STF_E_INVALID
    short.destroy()


@pytest.mark.parametrize("mode", ["stoch", "det"])
def test_ewa_footprints_larger_than_the_texture(dev, mode):
    # Derivatives up to 1e4 texture widths select the last level (one texel),
    # which is read directly: the work per query stays bounded and the result
    # equals the oracle's (the coarsest texel; index (0, 0, last level)).
    rng = np.random.default_rng(5)
    base = rng.integers(0, 256, (64, 64, 4), dtype=np.uint8)
    lv = synth.mip_levels(base)
    t = stf.stf_create_texture2d(64, 64, 4, stf.STF_FMT_U8, lv)
    n = 4096
    q = np.zeros((n, 6), np.float32)
    q[:, :2] = rng.random((n, 2))
    scale = 10.0 ** rng.uniform(-0.5, 4.0, n)             # 0.3 .. 1e4 texture widths
    ang = rng.random(n) * np.pi
    q[:, 2], q[:, 3] = scale * np.cos(ang), scale * np.sin(ang)
    q[:, 4], q[:, 5] = -0.5 * scale * np.sin(ang), 0.5 * scale * np.cos(ang)
    qd = torch.from_numpy(q).to(dev)
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    L = len(lv)
    if mode == "stoch":
        idx = torch.empty((n, 3), dtype=torch.int32, device=dev)
        stf.stf_filter_ewa(t, qd, 8.0, stf.STF_STOCHASTIC, 3, out, idx)
        ov, oi = oracle.ewa_filter2d(lv, oracle.U8, q, 8.0, oracle.STOCH, seed=3)
        gi = idx.cpu().numpy()
        assert np.array_equal(gi, oi)
        assert np.all(gi[scale >= 2.0] == [0, 0, L - 1])     # shorter axis = scale / 2 >= 1: lod >= L - 1
        assert np.array_equal(out.cpu().numpy(), ov.astype(np.float32))
    else:
        stf.stf_filter_ewa(t, qd, 8.0, stf.STF_DETERMINISTIC, 0, out)
        od, _ = oracle.ewa_filter2d(lv, oracle.U8, q, 8.0, oracle.DET)
        gd = out.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(gd - od) <= 1e-6 * np.abs(od) + 1e-12)
        top = lv[-1][0, 0].astype(np.float32) / np.float32(255)
        assert np.array_equal(out.cpu().numpy()[scale >= 2.0], np.broadcast_to(top, (int((scale >= 2.0).sum()), 4)))
    t.destroy()


@pytest.mark.parametrize("mode", ["stoch", "det"])
def test_ewa_raster_bound(dev, mode):
    # Records around the level-0 raster bound 2^24 (s up to +-40000 on a
    # 512-wide level 0, zero and small footprints, plus s spread over
    # 32000..33000 where the bound falls): NaN and the bad index beyond it,
    # the oracle's values and indices inside it.
    rng = np.random.default_rng(8)
    base = rng.integers(0, 256, (64, 512, 4), dtype=np.uint8)
    lv = synth.mip_levels(base)
    t = stf.stf_create_texture2d(512, 64, 4, stf.STF_FMT_U8, lv)
    rows = []
    for s in (32768.0, 32767.998046875, 40000.0, 30000.0):
        for sign in (1.0, -1.0):
            rows.append([sign * s, 0.25, 0.0, 0.0, 0.0, 0.0])
            rows.append([sign * s, 0.25, 3.0 / 512, 1.0 / 512, -0.5 / 512, 1.5 / 512])
    m = 2048
    far = np.zeros((m, 6), np.float32)
    far[:, 0] = rng.uniform(32000.0, 33000.0, m) * rng.choice([-1.0, 1.0], m)
    far[:, 1] = rng.random(m)
    far[:, 2:] = rng.normal(0.0, 2.0 / 512, (m, 4)) * (rng.random((m, 1)) < 0.75)
    q = np.concatenate([np.array(rows, np.float32), far.astype(np.float32)])
    n = q.shape[0]
    x0 = q[:, 0] * np.float32(512) - np.float32(0.5)
    beyond = np.abs(x0) >= np.float32(2.0 ** 24)
    assert 100 < beyond.sum() < n - 100
    qd = torch.from_numpy(q).to(dev)
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    if mode == "stoch":
        idx = torch.empty((n, 3), dtype=torch.int32, device=dev)
        stf.stf_filter_ewa(t, qd, 8.0, stf.STF_STOCHASTIC, 6, out, idx)
        ov, oi = oracle.ewa_filter2d(lv, oracle.U8, q, 8.0, oracle.STOCH, seed=6)
        gi = idx.cpu().numpy()
        assert np.array_equal(gi, oi)
        assert np.all(gi[beyond] == oracle.BAD_INDEX)
        gv = out.cpu().numpy()
        assert np.array_equal(np.isnan(gv), np.isnan(ov)) and np.all(np.isnan(gv[beyond]))
        assert np.array_equal(gv[~beyond], ov[~beyond].astype(np.float32))
    else:
        stf.stf_filter_ewa(t, qd, 8.0, stf.STF_DETERMINISTIC, 0, out)
        od, _ = oracle.ewa_filter2d(lv, oracle.U8, q, 8.0, oracle.DET)
        gd = out.cpu().numpy().astype(np.float64)
        assert np.array_equal(np.isnan(gd), np.isnan(od)) and np.all(np.isnan(gd[beyond]))
        assert np.all(np.abs(gd[~beyond] - od[~beyond]) <= 1e-6 * np.abs(od[~beyond]) + 1e-12)
    t.destroy()
