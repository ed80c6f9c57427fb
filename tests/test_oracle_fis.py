"""Pins of the oracle's filter importance sampling (section "Filter
Importance Sampling") and Gaussian filters (section "Results", magnification;
supplement, "Real-time discrete and filter importance sampling").

What fixes the answers: the Cox-de Boor identity (jittering by a B-spline of
degree n-1 and reading the nearest texel samples the degree-n B-spline; the
taps' frequencies are tested against the cubic B-spline weights of the
already-pinned oracle), the normal distribution of the Box-Muller offsets
(Kolmogorov-Smirnov), Monte Carlo agreement of each stochastic mode with the
independently computed mean it estimates, and limiting cases of the discrete
Gaussian (sigma -> 0 reads the nearest texel, sigma -> infinity the 4x4 box
average)."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle


def _freq(taps, lo, n_bins):
    return np.bincount(taps - lo, minlength=n_bins)


@pytest.mark.parametrize("t", [0.0, 0.13, 0.5, 0.77, 0.999])
def test_fis_cubic_taps_follow_bspline_weights(t):
    x = np.float32(40 + t)
    n = 60000
    taps = np.array([oracle.fis_tap(oracle.CUBIC, float(x), 9, q, 0) for q in range(n)])
    i = 40
    assert taps.min() >= i - 1 and taps.max() <= i + 2
    w = oracle.axis_weights(oracle.CUBIC, float(x) - i)
    f = _freq(taps, i - 1, 4)
    live = w > 0
    assert np.all(f[~live] == 0)
    assert stats.chisquare(f[live], w[live] / w[live].sum() * n).pvalue > 1e-4


@pytest.mark.parametrize("t", [0.0, 0.3, 0.8])
def test_fis_linear_is_jittered_nearest(t):
    x = np.float32(7 + t)
    n = 40000
    taps = np.array([oracle.fis_tap(oracle.LINEAR, float(x), 2, q, 1) for q in range(n)])
    assert set(np.unique(taps)) <= {7, 8}
    up = (taps == 8).mean()
    assert abs(up - t) <= 5 * math.sqrt(max(t * (1 - t), 1e-12) / n) + 1e-12
    # exact form: tap = floor(x + u) with the axis-1 uniform
    for q in range(50):
        assert oracle.fis_tap(oracle.LINEAR, float(x), 2, q, 1) == math.floor(float(x) + oracle.uniform(2, q, 1))


@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC])
def test_fis_filters_are_unbiased(filt):
    rng = np.random.default_rng(3)
    tex = rng.random((12, 12, 1)).astype(np.float32)
    K = 20000
    for uvq in rng.random((5, 2)).astype(np.float32):
        uv = np.repeat(uvq[None], K, axis=0)
        v, idx = oracle.filter2d(tex, oracle.F32, uv, filt, oracle.STOCH_FIS, seed=4)
        mean, var = oracle.moments2d(tex, oracle.F32, uvq[None], filt)
        assert abs(v[:, 0].mean() - mean[0, 0]) <= 5 * math.sqrt(var[0, 0] / K) + 1e-12
    g = oracle.Grid((16, 16, 16), oracle.F32, *_dense(rng))
    p = rng.uniform(2, 13, (3, 3)).astype(np.float32)
    for pq in p:
        v, _ = g.filter(np.repeat(pq[None], K, axis=0), filt, oracle.STOCH_FIS, seed=5)
        mean, var = g.moments(pq[None], filt)
        assert abs(v.mean() - mean[0]) <= 5 * math.sqrt(var[0] / K) + 1e-12


def _dense(rng):
    from tests._util import leaves_from_dense
    o, v = leaves_from_dense(rng.random((16, 16, 16)).astype(np.float32))
    return o, v


def test_box_muller_offsets_are_standard_normal():
    uv = np.full((50000, 2), 0.5, np.float32)
    pos = oracle.gauss_fis_positions(64, 64, uv, 0.8, seed=6)
    z = (pos - 31.5) / 0.8
    assert stats.kstest(z[:, 0], "norm").pvalue > 1e-4
    assert stats.kstest(z[:, 1], "norm").pvalue > 1e-4
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 0.02


@pytest.mark.parametrize("sigma", [0.3, 0.5, 0.8, 2.0])
def test_gaussian_fis_estimates_the_box_convolved_gaussian(sigma):
    rng = np.random.default_rng(7)
    tex = rng.random((24, 24, 1)).astype(np.float32)
    K = 20000
    for uvq in rng.random((4, 2)).astype(np.float32):
        uv = np.repeat(uvq[None], K, axis=0)
        v, _ = oracle.gauss_filter2d(tex, oracle.F32, uv, sigma, oracle.G_FIS, seed=8)
        m, _ = oracle.gauss_filter2d(tex, oracle.F32, uvq[None], sigma, oracle.G_FIS_MEAN)
        sd = v[:, 0].std()
        assert abs(v[:, 0].mean() - m[0, 0]) <= 5 * sd / math.sqrt(K) + 1e-12
    ones = np.ones((24, 24, 1), np.float32)
    m, _ = oracle.gauss_filter2d(ones, oracle.F32, rng.random((50, 2)).astype(np.float32), sigma, oracle.G_FIS_MEAN)
    assert np.all(np.abs(m - 1.0) < 2e-9)   # mass outside the window


@pytest.mark.parametrize("sigma", [0.3, 0.5, 0.8])
def test_discrete_gaussian_sampler_estimates_its_mean(sigma):
    rng = np.random.default_rng(9)
    tex = rng.random((16, 16, 1)).astype(np.float32)
    K = 20000
    for uvq in rng.random((4, 2)).astype(np.float32):
        uv = np.repeat(uvq[None], K, axis=0)
        v, idx = oracle.gauss_filter2d(tex, oracle.F32, uv, sigma, oracle.G_DISCRETE, seed=10)
        m, _ = oracle.gauss_filter2d(tex, oracle.F32, uvq[None], sigma, oracle.G_DISCRETE_MEAN)
        x = uvq * np.float32(16) - np.float32(0.5)
        i = np.floor(x).astype(int)
        assert np.all(idx >= np.clip(i - 1, 0, 15)) and np.all(idx <= np.clip(i + 2, 0, 15))
        sd = v[:, 0].std()
        assert abs(v[:, 0].mean() - m[0, 0]) <= 5 * sd / math.sqrt(K) + 1e-12


def test_discrete_gaussian_limits():
    rng = np.random.default_rng(11)
    tex = rng.random((16, 16, 2)).astype(np.float32)
    uv = rng.uniform(0.2, 0.8, (600, 2)).astype(np.float32)
    x = uv * np.float32(16) - np.float32(0.5)
    frac = x - np.floor(x)
    keep = np.all(np.abs(frac - 0.5) > 0.2, axis=1)   # away from the half-way point between texels
    uv, x = uv[keep][:200], x[keep][:200]
    near = np.floor(x + 0.5).astype(int)
    tiny, _ = oracle.gauss_filter2d(tex, oracle.F32, uv, 0.02, oracle.G_DISCRETE_MEAN)
    assert np.allclose(tiny, tex[near[:, 1], near[:, 0]], atol=1e-12)
    wide, _ = oracle.gauss_filter2d(tex, oracle.F32, uv, 16.0, oracle.G_DISCRETE_MEAN)
    i = np.floor(x).astype(int)
    box = np.array([tex[i[k, 1] - 1:i[k, 1] + 3, i[k, 0] - 1:i[k, 0] + 3].mean(axis=(0, 1)) for k in range(200)])
    assert np.allclose(wide, box, atol=3e-3)   # sigma = 16: weights within 0.5% of uniform over 4 texels
    # FIS mean with a tiny sigma reads the nearest texel too
    fm, _ = oracle.gauss_filter2d(tex, oracle.F32, uv, 0.02, oracle.G_FIS_MEAN)
    assert np.allclose(fm, tex[near[:, 1], near[:, 0]], atol=1e-9)


def test_argument_checks():
    tex = np.zeros((8, 8, 1), np.float32)
    uv = np.zeros((1, 2), np.float32)
    with pytest.raises(ValueError):
        oracle.gauss_filter2d(tex, oracle.F32, uv, 0.0, oracle.G_FIS)
    with pytest.raises(ValueError):
        oracle.filter2d(tex, oracle.F32, uv, oracle.KEYS, oracle.STOCH_FIS)
