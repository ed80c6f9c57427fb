"""Pins of the oracle's interpolating cubics (negative lobes) and their
positivized stochastic estimator (section "Sampling Techniques", paragraph
on positivization; supplement, "Filter Kernels" and "The interpolating
(negative lobe) bicubic filter").

What fixes the answers here: the Catmull-Rom spline in its textbook Hermite
form, polynomial reproduction and continuity of the kernels, brute force over
the tap window, exact masses, chi-square tests of the tap frequencies against
the weights, the paper's own two-reservoir sampler, and 5-sigma unbiasedness.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from tests._util import leaves_from_dense

FILTERS = [pytest.param(oracle.KEYS, id="keys"), pytest.param(oracle.MITCHELL, id="mitchell")]
SCALE = {oracle.KEYS: 2.0, oracle.MITCHELL: 18.0}
TS = np.concatenate([[0.0, 2.0 ** -24, 1e-6, 1 / 7, 0.25, 0.5, 6 / 7, 1 - 2.0 ** -24],
                     np.random.default_rng(0).random(200)]).astype(np.float32)


# ----------------------------------------------------------------------------
# the kernels
# ----------------------------------------------------------------------------
def test_keys_is_the_catmull_rom_spline():
    """K_3 with a = -1/2 interpolates like the Catmull-Rom spline: Hermite
    basis with tangents (p[i+1] - p[i-1]) / 2."""
    rng = np.random.default_rng(1)
    for t in rng.random(50):
        p = rng.standard_normal(4)
        w = oracle.axis_weights(oracle.KEYS, t)
        h00, h10 = 2 * t ** 3 - 3 * t ** 2 + 1, t ** 3 - 2 * t ** 2 + t
        h01, h11 = -2 * t ** 3 + 3 * t ** 2, t ** 3 - t ** 2
        m1, m2 = (p[2] - p[0]) / 2, (p[3] - p[1]) / 2
        ref = h00 * p[1] + h10 * m1 + h01 * p[2] + h11 * m2
        assert abs(w @ p - ref) <= 1e-14 * (1 + np.abs(p).sum())


@pytest.mark.parametrize("f", FILTERS)
def test_kernel_values_and_c1_continuity(f):
    K = lambda d: oracle.kernel(f, d)
    if f == oracle.KEYS:
        assert (K(0.0), K(1.0), K(2.0), K(-1.0)) == (1.0, 0.0, 0.0, 0.0)   # interpolating
    else:
        assert math.isclose(K(0.0), 8 / 9, rel_tol=1e-14) and math.isclose(K(1.0), 1 / 18, rel_tol=1e-13)
        assert K(2.0) == 0.0
    h = 1e-6
    for d in (1.0, 2.0):
        assert abs(K(d - 1e-12) - K(d + 1e-12)) < 1e-10
        left = (K(d - h) - K(d - 2 * h)) / h
        right = (K(d + 2 * h) - K(d + h)) / h
        assert abs(left - right) < 1e-4, (d, left, right)
    assert K(2.5) == 0.0 and K(-3.0) == 0.0
    for d in np.linspace(0, 2.5, 26):
        assert K(d) == K(-d)


@pytest.mark.parametrize("f", FILTERS)
def test_polynomial_reproduction(f):
    """Sum w = 1 and sum w (k-1) = t for both; sum w (k-1)^2 = t^2 for Keys
    (quadratics are reproduced) and t^2 + B/3 = t^2 + 1/9 for Mitchell."""
    k = np.arange(4) - 1.0
    for t in TS.astype(np.float64):
        w = oracle.axis_weights(f, t)
        assert abs(w.sum() - 1.0) < 1e-14
        assert abs(w @ k - t) < 1e-14
        extra = 0.0 if f == oracle.KEYS else 1.0 / 9.0
        assert abs(w @ k ** 2 - (t * t + extra)) < 1e-14


# ----------------------------------------------------------------------------
# pinned binary32 weights and the cumulative rule
# ----------------------------------------------------------------------------
def _exact_weights(f, t):
    """The four weights at the exact binary32 t, in rational arithmetic from
    the kernels' definitions (K_3 with a = -1/2; Mitchell-Netravali with
    B = C = 1/3)."""
    from fractions import Fraction as Fr

    def k(d):
        d = abs(d)
        if f == oracle.KEYS:
            a = Fr(-1, 2)
            if d < 1:
                return (a + 2) * d ** 3 - (a + 3) * d ** 2 + 1
            return a * d ** 3 - 5 * a * d ** 2 + 8 * a * d - 4 * a if d < 2 else Fr(0)
        B = C = Fr(1, 3)
        if d < 1:
            return ((12 - 9 * B - 6 * C) * d ** 3 + (-18 + 12 * B + 6 * C) * d ** 2 + (6 - 2 * B)) / 6
        if d < 2:
            return ((-B - 6 * C) * d ** 3 + (6 * B + 30 * C) * d ** 2 + (-12 * B - 48 * C) * d + (8 * B + 24 * C)) / 6
        return Fr(0)

    t = Fr(float(t))
    return [k(t + 1), k(t), k(1 - t), k(2 - t)]


@pytest.mark.parametrize("f", FILTERS)
def test_binary32_weights_track_the_kernel(f):
    """The factored binary32 forms agree with the exact kernel weight by
    weight to a few ulps of the weight itself (no cancellation near zeros),
    with the same sign; the binary64 weights agree to 4e-15 absolute."""
    rng = np.random.default_rng(2)
    ts = np.concatenate([TS, rng.random(3000).astype(np.float32),
                         (np.float32(1 / 7) + np.arange(-30, 30, dtype=np.float32) * np.float32(2 ** -26)),
                         (np.float32(6 / 7) + np.arange(-30, 30, dtype=np.float32) * np.float32(2 ** -26))])
    worst = 0.0
    for t in ts:
        ex = _exact_weights(f, t)
        w32 = oracle.interp_weights32(f, t).astype(np.float64) / SCALE[f]
        w64 = oracle.axis_weights(f, float(t))
        for k in range(4):
            assert np.sign(w32[k]) == np.sign(float(ex[k])), (t, k, w32, ex)
            assert abs(w64[k] - float(ex[k])) < 4e-15
            if ex[k] != 0:
                worst = max(worst, float(abs((type(ex[k])(float(w32[k])) - ex[k]) / ex[k])))
    assert worst < 8 * 2.0 ** -24, worst


def test_cumulative_choice_brute_force():
    """On the 2^-24 grid of u, each mass is chosen for a share of the grid
    equal to its share of the total (to a few grid points), zero masses never."""
    rng = np.random.default_rng(3)
    us = np.arange(0, 1 << 24, 97, dtype=np.float64) * 2.0 ** -24
    for trial in range(30):
        m = rng.random(4).astype(np.float32)
        m[rng.random(4) < 0.35] = 0
        if m.sum() == 0:
            m[2] = 0.5
        got = np.array([oracle.cumulative_choice(m, u) for u in us])
        assert np.all(m[got] > 0)
        share = np.bincount(got, minlength=4) / us.size
        assert np.allclose(share, m / m.sum(), atol=3e-4), (m, share)
    assert oracle.cumulative_choice(np.float32([0, 1, 1, 0]), 0.0) == 1
    assert oracle.cumulative_choice(np.float32([0, 1, 1, 0]), 1 - 2 ** -24) == 2
    assert oracle.cumulative_choice(np.float32([1e-40, 0, 0, 0]), 1 - 2 ** -24) == 0   # subnormal total


# ----------------------------------------------------------------------------
# the positivized draw
# ----------------------------------------------------------------------------
def _tensor(f, t):
    w = [oracle.axis_weights(f, float(x)) for x in t]
    out = w[0]
    for wa in w[1:]:
        out = np.multiply.outer(wa, out)   # index order (..., y, x)
    return out


def _draws(f, t, n, seed=11):
    D = len(t)
    pos = np.zeros((n, D), np.int32)
    neg = np.zeros((n, D), np.int32)
    has = np.zeros(n, bool)
    for q in range(n):
        pos[q], neg[q], has[q] = oracle.positivized_taps(f, t, seed, q)
    return pos, neg, has


def _chi2_ok(taps, w, p_min=1e-4):
    """taps (n, D) offsets -1..2 vs weights w (4,)*D in (..., y, x) order."""
    D = taps.shape[1]
    flat = np.zeros(w.size)
    key = np.zeros(taps.shape[0], np.int64)
    for a in range(D):
        key += (taps[:, a] + 1) * 4 ** a
    np.add.at(flat, key, 1)
    wf = np.zeros(w.size)
    for k in range(w.size):
        idx = tuple(((k // 4 ** a) % 4) for a in reversed(range(D)))
        wf[k] = w[idx]
    assert np.all(flat[wf == 0] == 0)
    live = wf > 0
    exp = wf[live] / wf[live].sum() * taps.shape[0]
    return stats.chisquare(flat[live], exp).pvalue > p_min


@pytest.mark.parametrize("f", FILTERS)
@pytest.mark.parametrize("t", [(0.3, 0.6), (0.05, 0.93), (0.5, 0.5, 0.2), (0.8, 0.1, 0.45)])
def test_draws_follow_positive_and_negative_weights(f, t):
    w = _tensor(f, t)
    pos, neg, has = _draws(f, t, 40000)
    assert has.all()
    assert _chi2_ok(pos, np.where(w > 0, w, 0))
    assert _chi2_ok(neg, np.where(w < 0, -w, 0))


@pytest.mark.parametrize("f", FILTERS)
def test_texel_centre_has_no_negative_tap(f):
    pos, neg, has = _draws(f, (0.0, 0.0), 500)
    if f == oracle.KEYS:
        assert not has.any() and np.all(pos == 0)   # all weight on the centre tap
    else:
        assert not has.any()                         # Mitchell at t = 0 has no negative weight
    sp, sn = oracle.positivized_masses(f, [0.0, 0.0])
    assert sn == 0.0 and abs(sp - 1.0) < 1e-15


@pytest.mark.parametrize("f", FILTERS)
def test_masses_are_exact(f):
    """S+ - S- = 1 (normalised filter) and S+ + S- = (P_x + N_x)(P_y + N_y)
    per-axis absolute sums, for the binary64 masses."""
    for t in [(0.3, 0.6), (0.7, 0.01), (0.25, 0.5, 0.125)]:
        sp, sn = oracle.positivized_masses(f, list(t))
        ab = 1.0
        for x in t:
            ab *= np.abs(oracle.axis_weights(f, x)).sum()
        assert abs(sp - sn - 1.0) < 1e-14 and abs(sp + sn - ab) < 1e-14


@pytest.mark.parametrize("f", FILTERS)
def test_paper_two_reservoir_sampler_has_the_same_marginals(f):
    """The paper's single-uniform two-reservoir sampler and the pinned draw
    both follow w+/S+ and w-/S- (the pinned one is tested above)."""
    t = (0.37, 0.71)
    w = _tensor(f, t)
    n = 40000
    rng = np.random.default_rng(5)
    pos = np.zeros((n, 2), np.int32)
    neg = np.zeros((n, 2), np.int32)
    for q in range(n):
        pos[q], neg[q], _ = oracle.positivized_wrs2d(f, t[0], t[1], rng.random())
    assert _chi2_ok(pos, np.where(w > 0, w, 0))
    assert _chi2_ok(neg, np.where(w < 0, -w, 0))


# ----------------------------------------------------------------------------
# filters: deterministic against brute force, stochastic unbiased
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("f", FILTERS)
def test_2d_separable_equals_brute_force(f):
    rng = np.random.default_rng(6)
    tex = rng.random((16, 16, 3)).astype(np.float32)
    uv = rng.random((500, 2)).astype(np.float32)
    det, _ = oracle.filter2d(tex, oracle.F32, uv, f, oracle.DET)
    bru = oracle.filter2d_brute(tex, oracle.F32, uv, f)
    assert np.allclose(det, bru, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("f", FILTERS)
def test_3d_separable_equals_brute_force_and_reproduces_polynomials(f):
    n = 16
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    rng = np.random.default_rng(7)
    field = rng.random((n, n, n)).astype(np.float32)
    o, v = leaves_from_dense(field)
    g = oracle.Grid((n, n, n), oracle.F32, o, v)
    p = rng.uniform(-1, n + 1, (400, 3)).astype(np.float32)
    det, _ = g.filter(p, f, oracle.DET)
    assert np.allclose(det, g.filter_brute(p, f), rtol=1e-12, atol=1e-13)
    # polynomial fields, interior queries: Keys reproduces (x^2)(y)(1), Mitchell x^2 + 1/9
    quad = (x.astype(np.float64) ** 2 * (1 + 0.5 * y) + z).astype(np.float32)   # exact in binary32
    o, v = leaves_from_dense(quad)
    g2 = oracle.Grid((n, n, n), oracle.F32, o, v)
    pi = rng.uniform(2, n - 3, (300, 3)).astype(np.float32)
    got, _ = g2.filter(pi, f, oracle.DET)
    X, Y, Z = (pi[:, a].astype(np.float64) for a in range(3))
    extra = 0.0 if f == oracle.KEYS else 1.0 / 9.0
    ref = (X ** 2 + extra) * (1 + 0.5 * Y) + Z
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("f", FILTERS)
def test_2d_stochastic_is_unbiased_5_sigma(f):
    rng = np.random.default_rng(8)
    tex = rng.random((8, 8, 2)).astype(np.float32)
    K = 20000
    for uvq in rng.random((6, 2)).astype(np.float32):
        uv = np.repeat(uvq[None], K, axis=0)
        vals, idx = oracle.filter2d(tex, oracle.F32, uv, f, oracle.STOCH, seed=3)
        mean, var = oracle.moments2d(tex, oracle.F32, uvq[None], f)
        assert np.all(np.abs(vals.mean(0) - mean[0]) <= 5 * np.sqrt(var[0] / K))
        # sample variance vs exact variance
        assert np.all(np.abs(vals.var(0) / var[0] - 1) < 0.1)
        assert idx.shape == (K, 4)


@pytest.mark.parametrize("f", FILTERS)
def test_3d_stochastic_value_and_index(f):
    """Value = S+ t(j+) - S- t(j-) at the returned indices; moments mean equals
    the deterministic value."""
    n = 16
    rng = np.random.default_rng(9)
    field = rng.random((n, n, n)).astype(np.float32)
    o, v = leaves_from_dense(field)
    g = oracle.Grid((n, n, n), oracle.F32, o, v)
    p = rng.uniform(1, n - 2, (300, 3)).astype(np.float32)
    val, idx = g.filter(p, f, oracle.STOCH, seed=4)
    assert idx.shape == (300, 6)
    for q in range(300):
        t = [float(c) - math.floor(float(c)) for c in p[q]]
        sp, sn = oracle.positivized_masses(f, t)
        ref = sp * g.texel(*idx[q, :3])
        if idx[q, 3] != oracle.BAD_INDEX:
            ref -= sn * g.texel(*idx[q, 3:])
        assert val[q] == ref
        cell = np.floor(p[q]).astype(int)
        assert np.all((idx[q, :3] - cell >= -1) & (idx[q, :3] - cell <= 2))
    mean, var = g.moments(p, f)
    det, _ = g.filter(p, f, oracle.DET)
    assert np.allclose(mean, det, rtol=1e-12, atol=1e-13) and np.all(var >= -1e-12)


def test_reuse_sampler_is_2d_only():
    g = oracle.Grid((8, 8, 8), oracle.F32, np.zeros((1, 3), np.int32), np.zeros((1, 8, 8, 8), np.float32))
    with pytest.raises(ValueError):
        g.filter(np.zeros((1, 3), np.float32), oracle.KEYS, oracle.STOCH_REUSE)


@pytest.mark.parametrize("f", FILTERS + [pytest.param(oracle.CUBIC, id="bspline")])
def test_abs_scale_bounds_the_value(f):
    """DET_ABS = sum |w||t| >= |F|, with equality for non-negative weights
    and texels."""
    rng = np.random.default_rng(10)
    tex = (rng.random((12, 12, 2)) - 0.3).astype(np.float32)
    uv = rng.random((300, 2)).astype(np.float32)
    d, _ = oracle.filter2d(tex, oracle.F32, uv, f, oracle.DET)
    a, _ = oracle.filter2d(tex, oracle.F32, uv, f, oracle.DET_ABS)
    assert np.all(a >= np.abs(d) - 1e-15)
    pos, _ = oracle.filter2d(np.abs(tex), oracle.F32, uv, oracle.CUBIC, oracle.DET)
    apos, _ = oracle.filter2d(np.abs(tex), oracle.F32, uv, oracle.CUBIC, oracle.DET_ABS)
    assert np.allclose(pos, apos, rtol=1e-14)
