"""Pins of the oracle's random numbers and its per-axis tap choice.

The uniforms must be uniform and independent across queries and axes; the tap
choice must realise the filter weights as probabilities (chi-square), never
pick a tap of zero weight, and reduce to the obvious answer at the ends of
[0, 1) -- the properties that the sampling rules of section "Sampling
Techniques" (Eq. stochastic-sum, "sampling arrays") state."""
import numpy as np
import pytest
from scipy import stats

import oracle


def _uniforms(seed, n, axis):
    return np.array([oracle.uniform(seed, q, axis) for q in range(n)], np.float64)


def test_uniform_grid_and_range():
    u = _uniforms(7, 4096, 0)
    assert np.all(u >= 0.0) and np.all(u < 1.0)
    assert np.all(u * 2 ** 24 == np.floor(u * 2 ** 24))   # on the 2^-24 grid


def test_uniform_distribution_chi_square():
    u = _uniforms(11, 1 << 16, 1)
    counts = np.bincount((u * 64).astype(int), minlength=64)
    assert stats.chisquare(counts).pvalue > 1e-4
    assert stats.kstest(u, "uniform").pvalue > 1e-4


def test_uniform_axes_and_seeds_independent():
    n = 1 << 14
    a, b = _uniforms(3, n, 0), _uniforms(3, n, 1)
    c = _uniforms(4, n, 0)
    d = _uniforms(3 + (1 << 32), n, 0)           # the seed's high word matters
    for x, y in ((a, b), (a, c), (a, d)):
        r = np.corrcoef(x, y)[0, 1]
        assert abs(r) < 5.0 / np.sqrt(n)
    # successive queries are not correlated either
    assert abs(np.corrcoef(a[:-1], a[1:])[0, 1]) < 5.0 / np.sqrt(n)


def test_pcg_is_injective_on_a_range():
    v = [oracle.pcg(x) for x in range(1 << 16)]
    assert len(set(v)) == len(v)


@pytest.mark.parametrize("t", [0.0, 0.125, 0.3, 0.5, 0.77, 0.999])
@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC])
def test_tap_frequencies_match_weights(t, filt):
    # sampling arrays: tap j is chosen with probability w_j
    n = 40000
    rng = np.random.default_rng(5)
    us = (rng.integers(0, 1 << 24, n) * 2.0 ** -24).astype(np.float32)
    offs = np.array([oracle.select(filt, t, u) for u in us])
    w = oracle.axis_weights(filt, np.float32(t))
    if filt == oracle.CUBIC:
        counts = np.bincount(offs + 1, minlength=4)
        probs = w
    else:
        counts = np.bincount(offs, minlength=2)[:2]
        probs = w[:2]
    nz = probs > 0
    assert counts[~nz].sum() == 0                 # zero-weight taps never chosen
    exp = probs[nz] * n
    if nz.sum() > 1:
        assert stats.chisquare(counts[nz], exp).pvalue > 1e-4


def test_select_end_points():
    # u = 0 takes the first tap of the cumulative order: the upper tap for the
    # lerp rule (u < t), tap i-1 for the cubic one
    assert oracle.select(oracle.LINEAR, 0.3, 0.0) == 1
    assert oracle.select(oracle.LINEAR, 0.0, 0.0) == 0        # t = 0: upper tap has weight 0
    assert oracle.select(oracle.CUBIC, 0.3, 0.0) == -1
    umax = 1.0 - 2.0 ** -24
    assert oracle.select(oracle.LINEAR, 0.3, umax) == 0
    assert oracle.select(oracle.CUBIC, 0.3, umax) == 2
    assert oracle.select(oracle.CUBIC, 0.0, umax) == 1        # tap i+2 has weight 0 at t = 0
    # tie at u == t: the strict comparison of the bilinear listing keeps the lower tap
    assert oracle.select(oracle.LINEAR, 0.5, 0.5) == 0


def test_select_breakpoints_are_cumulative_weights():
    # the cubic choice flips exactly at the (binary32) cumulative weights
    for t in [0.1, 0.37, 0.5, 0.81]:
        w = oracle.axis_weights(oracle.CUBIC, np.float32(t))
        cum = np.cumsum(w)[:3]
        for k, c in enumerate(cum):
            below = np.float32(c) - np.float32(4e-7)
            above = np.float32(c) + np.float32(4e-7)
            assert oracle.select(oracle.CUBIC, t, below) == k - 1
            assert oracle.select(oracle.CUBIC, t, above) == k


def test_cubic_breakpoints_ordered_for_every_binary32_t():
    # the chosen tap is the first whose cumulative weight exceeds u only if
    # the breakpoints are ordered; checked for all 2^30 binary32 t in [0, 1)
    assert oracle.cubic_breakpoints_disorder() == 0


def test_cubic_breakpoints_close_to_exact_cumulative_weights():
    for t in np.linspace(0.0, 1.0, 1001, endpoint=False).astype(np.float32):
        w = oracle.axis_weights(oracle.CUBIC, float(t))
        c = oracle.cubic_breakpoints(t).astype(np.float64)
        assert np.allclose(c, np.cumsum(w)[:3], rtol=0, atol=2e-7)
