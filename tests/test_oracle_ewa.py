"""Pins of the oracle's EWA filtering over a MIP pyramid (section "B-Spline
and Anisotropic Filters": stochastic level choice, then one tap drawn in
proportion to the EWA weights; supplement, "Stochastic sampling of the EWA
kernel").

What fixes the answers: closed forms of the level of detail (powers of two,
the anisotropy clamp), normalisation (constant textures), the degenerate
footprint reducing to the already-pinned bilinear filter, the level-choice
frequency, and Monte Carlo agreement of the stochastic estimate with the
deterministic EWA (two independent code paths over the same weights)."""
import math

import numpy as np
import pytest

import oracle
import synth


def _q(n, s, t, d0, d1):
    q = np.zeros((n, 6), np.float32)
    q[:, 0], q[:, 1] = s, t
    q[:, 2:4] = d0
    q[:, 4:6] = d1
    return q


def test_lut():
    lut = np.array([oracle.ewa_lut(i) for i in range(128)])
    assert lut[0] == np.float32(1.0 - math.exp(-2.0)) and lut[127] == 0.0
    assert np.all(np.diff(lut) < 0)


def test_level_of_detail_closed_forms():
    L, W0 = 8, 128
    for j in range(L):
        q = _q(1, 0.3, 0.6, (2.0 ** j / W0, 0.0), (0.0, 2.0 ** j / W0))
        assert oracle.ewa_lods(q, L, 8.0)[0] == (j if j <= L - 1 else L - 1)
    # anisotropy clamp: the shorter axis is raised to longer / max_aniso
    q = _q(1, 0.5, 0.5, (32.0 / W0, 0.0), (0.0, 0.5 / W0))
    assert oracle.ewa_lods(q, L, 8.0)[0] == pytest.approx((L - 1) + math.log2(4.0 / W0), abs=1e-12)
    q = _q(1, 0.5, 0.5, (0.25 / W0, 0.0), (0.0, 0.25 / W0))   # below level 0
    assert oracle.ewa_lods(q, L, 8.0)[0] == 0.0


@pytest.fixture(scope="module")
def pyramid():
    rng = np.random.default_rng(1)
    tex = rng.random((64, 64, 2)).astype(np.float32)
    return synth.mip_levels(tex)


def test_constant_texture_is_reproduced():
    lv = synth.mip_levels(np.full((32, 32, 1), 0.37, np.float32))
    rng = np.random.default_rng(2)
    q = np.concatenate([rng.random((300, 2)), rng.normal(0, 0.02, (300, 4))], axis=1).astype(np.float32)
    d, _ = oracle.ewa_filter2d(lv, oracle.F32, q, 8.0, oracle.DET)
    assert np.allclose(d, np.float32(0.37), rtol=0, atol=1e-7)   # the levels hold fl32(0.37) exactly
    v, idx = oracle.ewa_filter2d(lv, oracle.F32, q, 8.0, oracle.STOCH, seed=3)
    assert np.all(v == np.float32(0.37))
    assert np.all((idx[:, 2] >= 0) & (idx[:, 2] < len(lv)))


def test_integer_lod_picks_that_level(pyramid):
    j = 2
    q = _q(400, 0.41, 0.23, (2.0 ** j / 64, 0.0), (0.0, 2.0 ** j / 64))
    q[:, 0:2] = np.random.default_rng(4).random((400, 2))
    _, idx = oracle.ewa_filter2d(pyramid, oracle.F32, q, 8.0, oracle.STOCH, seed=5)
    assert np.all(idx[:, 2] == j)


def test_level_choice_frequency(pyramid):
    f = 0.3
    shorter = 2.0 ** (1 + f) / 64
    n = 20000
    q = _q(n, 0.5, 0.5, (shorter, 0.0), (0.0, shorter))
    lod = oracle.ewa_lods(q[:1], len(pyramid), 8.0)[0]
    assert lod == pytest.approx(1 + f, abs=1e-6)
    _, idx = oracle.ewa_filter2d(pyramid, oracle.F32, q, 8.0, oracle.STOCH, seed=6)
    p = (idx[:, 2] == 2).mean()
    assert set(np.unique(idx[:, 2])) <= {1, 2}
    frac = lod - 1
    assert abs(p - frac) <= 5 * math.sqrt(frac * (1 - frac) / n)


def test_stochastic_ewa_is_unbiased(pyramid):
    rng = np.random.default_rng(7)
    K = 20000
    for _ in range(6):
        s, t = rng.random(2)
        ang = rng.random() * math.pi
        a = 2.0 ** rng.uniform(-1, 3) / 64
        r = rng.uniform(1, 10)
        d0 = (a * r * math.cos(ang), a * r * math.sin(ang))
        d1 = (-a * math.sin(ang), a * math.cos(ang))
        q = _q(K, s, t, d0, d1)
        det, _ = oracle.ewa_filter2d(pyramid, oracle.F32, q[:1], 8.0, oracle.DET)
        v, _ = oracle.ewa_filter2d(pyramid, oracle.F32, q, 8.0, oracle.STOCH, seed=8)
        sd = v.std(axis=0)
        assert np.all(np.abs(v.mean(axis=0) - det[0]) <= 5 * sd / math.sqrt(K) + 1e-12), (d0, d1)


def test_degenerate_footprint_is_bilinear(pyramid):
    rng = np.random.default_rng(9)
    uv = rng.random((200, 2)).astype(np.float32)
    q = np.concatenate([uv, np.zeros((200, 4), np.float32)], axis=1)
    d, _ = oracle.ewa_filter2d(pyramid, oracle.F32, q, 8.0, oracle.DET)
    ref, _ = oracle.filter2d(pyramid[0], oracle.F32, uv, oracle.LINEAR, oracle.DET)
    assert np.allclose(d, ref, rtol=0, atol=1e-15)
    v, idx = oracle.ewa_filter2d(pyramid, oracle.F32, q, 8.0, oracle.STOCH, seed=2)
    assert np.all(idx[:, 2] == 0)


def test_argument_checks(pyramid):
    q = np.zeros((1, 6), np.float32)
    with pytest.raises(ValueError):
        oracle.ewa_filter2d(pyramid, oracle.F32, q, 0.5, oracle.DET)   # max anisotropy below 1
    q[0, 0] = np.nan
    v, idx = oracle.ewa_filter2d(pyramid, oracle.F32, q, 8.0, oracle.STOCH)
    assert np.all(np.isnan(v)) and np.all(idx == oracle.BAD_INDEX)


def _far_records():
    """EWA records on a 512-texel-wide level 0 around the raster bound 2^24:
    s = 32768 gives s W0 - 1/2 = 2^24 - 1/2, which binary32 rounds (to even)
    to 2^24 itself, so the record is out; the next float below, 32767.998046875,
    gives 16777214.5 -> 16777214, which is in, while its mirror gives
    -16777215.5 -> -2^24 (ties to even), which is out.  Each s comes with a
    zero footprint and with a small ellipse, and mirrored to -s."""
    rows = []
    for s in (32768.0, 32767.998046875, 40000.0, 30000.0):
        for sign in (1.0, -1.0):
            rows.append([sign * s, 0.25, 0.0, 0.0, 0.0, 0.0])
            rows.append([sign * s, 0.25, 3.0 / 512, 1.0 / 512, -0.5 / 512, 1.5 / 512])
    q = np.array(rows, np.float32)
    x0 = q[:, 0] * np.float32(512) - np.float32(0.5)          # binary32, as the filters form it
    return q, np.abs(x0) >= np.float32(2.0 ** 24)


def test_raster_bound_on_level_zero():
    # A record whose level-0 raster position is 2^24 or more in magnitude has
    # no integer cell (the rule of every 2D filter) and yields NaN with the
    # bad index, whichever level it would draw; positions just inside the
    # bound filter normally (on a constant texture: the constant; the taps
    # clamp to the edge column of their level).
    lv = synth.mip_levels(np.full((16, 512, 1), 0.625, np.float32))
    q, out = _far_records()
    assert out.tolist() == [True] * 4 + [False] * 2 + [True] * 6 + [False] * 4
    for mode in (oracle.DET, oracle.STOCH):
        v, idx = oracle.ewa_filter2d(lv, oracle.F32, q, 8.0, mode, seed=4)
        assert np.all(np.isnan(v[out])) and not np.any(np.isnan(v[~out]))
        assert np.all(v[~out] == 0.625)
        if mode == oracle.STOCH:
            assert np.all(idx[out] == oracle.BAD_INDEX)
            ok = idx[~out]
            w_l = np.array([max(1, 512 >> int(l)) for l in ok[:, 2]])
            right = q[~out, 0] > 0
            assert np.all(ok[right, 0] == w_l[right] - 1) and np.all(ok[~right, 0] == 0)
