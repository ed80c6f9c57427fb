"""Independent pins of the oracle's random numbers, tap choice, GGX terms and
EWA ellipse.

Each test checks the oracle against something other than its own formula:
known-answer values worked out from the published definitions
(tests/golden/rng_select_vectors.txt), textbook identities of the GGX
microfacet model, and the closed-form second moments of an elliptical
weighted average.  tests/test_oracle_mutations.py plants a plausible mistake
in a copy of the oracle and shows that one of these tests then fails."""
import os
import time

import numpy as np
import pytest
from scipy import stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rng_select_vectors.txt")


def _golden(kind):
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            parts = line.split()
            if parts and parts[0] == kind:
                rows.append(parts[1:])
    assert rows, kind
    return rows


# ---------------------------------------------------------------------------
# random numbers and tap choice: known answers
# ---------------------------------------------------------------------------
def test_pcg_known_answers():
    for x, h in _golden("pcg"):
        assert oracle.pcg(int(x, 16)) == int(h, 16)


def test_seed_key_known_answer():
    for seed, key in _golden("key"):
        assert oracle.lib().orc_seed_key(int(seed)) == int(key, 16)


def test_uniform_known_answers():
    for seed, qid, axis, u in _golden("u"):
        got = oracle.uniform(int(seed), int(qid), int(axis))
        assert got == pytest.approx(float(u), abs=1e-9), (seed, qid, axis)
        assert got * 2 ** 24 == int(got * 2 ** 24)


def test_cubic_breakpoints_known_answers():
    for x, c1, c2, c3 in _golden("bp"):
        xf = np.float32(x)
        t = xf - np.floor(xf)
        c = oracle.cubic_breakpoints(t)
        assert np.allclose(c, [float(c1), float(c2), float(c3)], rtol=0, atol=1e-9), (x, c)


def test_tap_known_answers():
    # each vector: one 2D query of a W x W texture at (u, v) as query qid
    for W, u, v, seed, qid, filt, tx, ty in _golden("tap"):
        W, seed, qid = int(W), int(seed), int(qid)
        f = oracle.CUBIC if filt == "cubic" else oracle.LINEAR
        tex = np.zeros((W, W, 1), np.float32)
        uv = np.tile(np.array([[float(u), float(v)]], np.float32), (qid + 1, 1))
        _, idx = oracle.filter2d(tex, oracle.F32, uv, f, oracle.STOCH, seed=seed)
        assert tuple(idx[qid]) == (int(tx), int(ty)), (W, u, v, seed, qid, filt, idx[qid])


# ---------------------------------------------------------------------------
# GGX (section "Effect of Texture Filtering on Rendering": the filtered
# quantity is BSDF x cosine; the BSDF is a GGX microfacet lobe)
# ---------------------------------------------------------------------------
N = np.array([0.0, 0.0, 1.0])


def _sph(theta, phi):
    return np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])


def _h_quadrature(alpha, n_psi=240, n_phi=96):
    """Nodes and weights over the hemisphere of microfacet normals h, with
    tan(theta_h) = alpha tan(psi) so the nodes follow the peak of D."""
    psi = (np.arange(n_psi) + 0.5) / n_psi * (np.pi / 2)
    theta = np.arctan(alpha * np.tan(psi))
    dtheta = alpha / np.cos(psi) ** 2 / (1 + (alpha * np.tan(psi)) ** 2) * (np.pi / 2 / n_psi)
    phi = (np.arange(n_phi) + 0.5) / n_phi * 2 * np.pi
    for th, dth in zip(theta, dtheta):
        for ph in phi:
            yield _sph(th, ph), np.sin(th) * dth * (2 * np.pi / n_phi)


@pytest.mark.parametrize("alpha,theta_o", [(0.3, 1.0), (0.5, 1.2), (0.8, 0.7), (1.0, 1.35)])
def test_ggx_visible_normal_identity(alpha, theta_o):
    # The projected area of the visible microfacets equals that of the
    # macrosurface: G1(wo) * int max(0, wo.h) D(h) dw_h = cos(theta_o), with
    # the Smith masking G1 = 1 / (1 + Lambda(wo)) (Heitz 2014, Eq. 4 with the
    # Smith G1).  This pins Lambda against D.
    wo = _sph(theta_o, 0.4)
    lam = oracle.ggx_terms(N, wo, wo, alpha)["lambda_o"]
    acc = 0.0
    for h, dw in _h_quadrature(alpha):
        c = float(wo @ h)
        if c > 0:
            acc += oracle.ggx_D(N, h, alpha) * c * dw
    assert acc / (1.0 + lam) == pytest.approx(np.cos(theta_o), rel=2e-3)


@pytest.mark.parametrize("alpha,theta_o", [(0.1, 0.3), (0.15, 0.6), (0.2, 0.45)])
def test_shading_weak_white_furnace(alpha, theta_o):
    # Weak white furnace (Heitz 2014): with the shadowing G2 and the Fresnel
    # F replaced by the masking G1(wo) and 1, the specular lobe of shade_eval
    # integrates to 1 over wi.  Integrated over h with wi = reflect(wo, h)
    # and the reflection Jacobian dw_i = 4 |wo.h| dw_h (Walter et al. 2007).
    # The lobe is zero below the horizon; the visible microfacets that reflect
    # there carry the mass D(h) G1(wo) (wo.h) / cos_o dw_h (about 1% here:
    # the GGX tail is long), which is added back.  This pins the
    # 1/(4 cos_o cos_i) normalisation of the lobe.
    wo = _sph(theta_o, 1.1)
    mat = np.array([0.0, 0.0, 0.0, np.sqrt(alpha), 0.0, 0.0])   # black albedo, r^2 = alpha
    g1o = 1.0 / (1.0 + oracle.ggx_terms(N, wo, wo, alpha)["lambda_o"])
    acc = lost = 0.0
    for h, dw in _h_quadrature(alpha, n_psi=200, n_phi=80):
        c = float(wo @ h)
        if c <= 0:
            continue
        wi = 2.0 * c * h - wo
        if wi[2] <= 1e-6:
            lost += oracle.ggx_D(N, h, alpha) * g1o * c / wo[2] * dw
            continue
        wo32, wi32 = wo.astype(np.float32), wi.astype(np.float32)
        g = oracle.ggx_terms(N, wo32.astype(np.float64), wi32.astype(np.float64), alpha)
        fhat = oracle.shade_eval(mat, wo32, wi32)[0]   # D G2 F / (4 cos_o)
        acc += fhat / (g["G2"] * g["F"]) * g1o * 4.0 * c * dw
    assert lost < 0.05
    assert acc + lost == pytest.approx(1.0, rel=2e-3)


def test_schlick_fresnel_limits():
    # Schlick's approximation: F = F0 = 0.04 at normal incidence (wi.h = 1),
    # rising monotonically to 1 at grazing incidence (wi.h -> 0).
    assert oracle.ggx_terms(N, N, N, 0.3)["F"] == pytest.approx(0.04, abs=1e-15)
    prev = 0.0
    for th in [0.0, 0.3, 0.7, 1.0, 1.3, 1.5, 1.57, 1.5707]:
        wo, wi = _sph(th, 0.0), _sph(th, np.pi)        # h = n, wi.h = cos(th)
        F = oracle.ggx_terms(N, wo, wi, 0.3)["F"]
        assert F >= prev
        prev = F
    assert prev > 0.999


@pytest.mark.parametrize("alpha", [0.2, 0.6, 1.0])
def test_ggx_shadowing_is_height_correlated(alpha):
    # Height-correlated Smith shadowing (Heitz 2014): masking and shadowing
    # are positively correlated, so G2 lies strictly between the uncorrelated
    # product G1(wo) G1(wi) and the fully correlated min(G1(wo), G1(wi)), and
    # reduces to G1 of the other direction when one direction is the normal.
    rng = np.random.default_rng(3)
    for _ in range(50):
        wo = _sph(rng.uniform(0.2, 1.45), rng.uniform(0, 6.28))
        wi = _sph(rng.uniform(0.2, 1.45), rng.uniform(0, 6.28))
        g = oracle.ggx_terms(N, wo, wi, alpha)
        g1o, g1i = 1 / (1 + g["lambda_o"]), 1 / (1 + g["lambda_i"])
        assert g1o * g1i < g["G2"] < min(g1o, g1i)
    wi = _sph(1.1, 0.5)
    g = oracle.ggx_terms(N, N, wi, alpha)
    assert g["lambda_o"] == 0.0
    assert g["G2"] == pytest.approx(1 / (1 + g["lambda_i"]), rel=1e-15)


# ---------------------------------------------------------------------------
# EWA (section "B-Spline and Anisotropic Filters"; supplement, "Stochastic
# sampling of the EWA kernel"): the ellipse is the image of the unit circle
# under the derivative matrix J, widened by one texel (pbrt: the +1 terms),
# i.e. r^2 = p^T M^-1 p with M = J J^T + I in texels.  With a radial profile
# f(r^2), the weighted second moments are E[p p^T] = M * E[r^2] / 2, and an
# average over sub-texel offsets of the centre turns the lattice sums into
# that integral.
# ---------------------------------------------------------------------------
def _lut_mean_r2():
    L = np.array([np.exp(-2.0 * i / 127.0) - np.exp(-2.0) for i in range(128)])
    # area is uniform in rho = r^2; bin i covers rho in [i/128, (i+1)/128)
    return float((L * (2 * np.arange(128) + 1) / 256.0).sum() / L.sum())


def _ewa_second_moments(W, d0, d1, n_off=12):
    num = np.zeros((2, 2))
    den = 0.0
    c = W // 2
    for oy in range(n_off):
        for ox in range(n_off):
            fx, fy = (ox + 0.5) / n_off, (oy + 0.5) / n_off
            s = np.float32((c + 0.5 + fx) / W)
            t = np.float32((c + 0.5 + fy) / W)
            stx = np.float32(np.float32(s * np.float32(W)) - np.float32(0.5))
            sty = np.float32(np.float32(t * np.float32(W)) - np.float32(0.5))
            xy, w = oracle.ewa_weights(W, W, s, t, d0, d1)
            p = xy.astype(np.float64) - [float(stx), float(sty)]
            w = w.astype(np.float64)
            num += np.einsum("k,ki,kj->ij", w, p, p)
            den += w.sum()
    return num / den


@pytest.mark.parametrize("major,minor,angle", [
    (6.0, 1.5, 0.0), (1.5, 6.0, 0.0), (8.0, 2.0, 0.5), (8.0, 2.0, -1.1), (3.0, 3.0, 0.3), (0.5, 0.25, 0.0)])
def test_ewa_ellipse_second_moments(major, minor, angle):
    W = 1024
    ca, sa = np.cos(angle), np.sin(angle)
    d0 = np.array([major * ca, major * sa]) / W     # texture units
    d1 = np.array([-minor * sa, minor * ca]) / W
    J = np.stack([d0, d1], axis=1) * W             # columns: derivative vectors in texels
    M = J @ J.T + np.eye(2)
    S = _ewa_second_moments(W, d0.astype(np.float32), d1.astype(np.float32))
    expect = M * _lut_mean_r2() / 2.0
    assert np.allclose(S, expect, rtol=0, atol=2e-3 * np.abs(expect).max()), (S, expect)


def test_ewa_coarsest_level_is_constant_work():
    # A footprint larger than the whole texture selects the last level, a
    # single texel, which is read directly: 64 queries with derivatives of
    # 1e4 texture widths finish at once (a scan of the ellipse's bounding box
    # on that level would visit ~4e8 taps per query) and return that texel.
    rng = np.random.default_rng(9)
    sizes = [64 >> l for l in range(7)]
    lv = [rng.integers(0, 256, (s, s, 4), dtype=np.uint8) for s in sizes]
    q = np.zeros((64, 6), np.float32)
    q[:, :2] = rng.random((64, 2))
    q[:, 2] = 1e4
    q[:, 5] = 1e4
    t0 = time.time()
    det, _ = oracle.ewa_filter2d(lv, oracle.U8, q, 8.0, oracle.DET)
    sto, idx = oracle.ewa_filter2d(lv, oracle.U8, q, 8.0, oracle.STOCH, seed=4)
    assert time.time() - t0 < 2.0
    top = lv[-1][0, 0].astype(np.float64) / 255.0
    assert np.allclose(det, top, rtol=0, atol=1e-15)
    assert np.allclose(sto, top, rtol=0, atol=0)
    assert np.all(idx == [0, 0, 6])


def test_ewa_rejects_a_pyramid_that_stops_short():
    lv = [np.zeros((8, 8, 1), np.uint8), np.zeros((4, 4, 1), np.uint8)]
    q = np.zeros((1, 6), np.float32)
    with pytest.raises(ValueError):
        oracle.ewa_filter2d(lv, oracle.U8, q, 8.0, oracle.DET)


@pytest.mark.parametrize("d0,d1", [((5.0, 0.0), (0.0, 1.2)), ((3.5, 3.5), (-0.9, 0.9)), ((1.0, -0.3), (0.2, 0.8))])
def test_ewa_draws_follow_the_weights(d0, d1):
    # The stochastic EWA tap is drawn with probability w / sum w.  The row
    # rule of the oracle (reservoir over row sums, then the cumulative rule
    # within the row) and the supplement's single-uniform reservoir sampler
    # are both checked against the weights by chi-square.
    W = 256
    levels = 9
    sizes = [W >> l for l in range(levels)]
    lv = [np.zeros((s, s, 1), np.uint8) for s in sizes]
    # lod = (levels - 1) + log2(shorter) = 2 exactly: shorter = 2^-6 texture units
    a0 = np.array(d0, np.float64)
    a1 = np.array(d1, np.float64)
    if np.hypot(*a0) < np.hypot(*a1):
        a0, a1 = a1, a0
    scale = 2.0 ** -6 / np.hypot(*a1)
    d0f = (a0 * scale).astype(np.float32)
    d1f = (a1 * scale).astype(np.float32)
    K = 120000
    s, t = np.float32(0.51), np.float32(0.47)
    q = np.tile(np.array([[s, t, d0f[0], d0f[1], d1f[0], d1f[1]]], np.float32), (K, 1))
    _, idx = oracle.ewa_filter2d(lv, oracle.U8, q, 64.0, oracle.STOCH, seed=21)
    lvl = int(np.bincount(idx[:, 2]).argmax())      # lod is 2 up to rounding of the lengths
    assert lvl == 2
    idx = idx[idx[:, 2] == lvl]
    assert idx.shape[0] > K // 2
    xy, w = oracle.ewa_weights(sizes[lvl], sizes[lvl], s, t, d0f, d1f)
    assert xy.min() >= 0 and xy.max() < sizes[lvl]      # no clamping in this test
    p = w.astype(np.float64) / w.sum()
    key = {(int(x), int(y)): k for k, (x, y) in enumerate(xy)}
    lst = oracle.ewa_listing_draws(sizes[lvl], sizes[lvl], s, t, d0f, d1f, seed=22, K=K)
    for draws in (idx[:, :2], lst):
        counts = np.zeros(len(w))
        for x, y in draws:
            counts[key[(int(x), int(y))]] += 1           # a tap outside the ellipse raises KeyError
        exp = p * counts.sum()
        keep = exp >= 5
        obs = np.append(counts[keep], counts[~keep].sum())
        ex = np.append(exp[keep], exp[~keep].sum())
        if ex[-1] == 0:
            obs, ex = obs[:-1], ex[:-1]
        ex = ex * (obs.sum() / ex.sum())
        assert stats.chisquare(obs, ex).pvalue > 1e-4
