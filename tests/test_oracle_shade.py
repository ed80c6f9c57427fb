"""Pins of the shading oracle: textbook identities of the GGX microfacet
model, the affine-contribution statement of section "Effect of Texture
Filtering on Rendering", and the unbiasedness of the sampled filter-after-
shade estimator."""
import numpy as np
import pytest

import oracle
import synth


def _hemi(theta, phi):
    return np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])


@pytest.mark.parametrize("alpha", [0.05, 0.2, 0.6, 1.0])
def test_ggx_D_projected_area_is_one(alpha):
    # int D(h) (n.h) dw_h = 1 over the hemisphere (microfacet normalisation)
    n = np.array([0.0, 0.0, 1.0])
    # substitution tan(theta) = alpha * tan(psi) spreads points over the peak
    psi = (np.arange(400000) + 0.5) / 400000 * (np.pi / 2)
    theta = np.arctan(alpha * np.tan(psi))
    dtheta = alpha / np.cos(psi) ** 2 / (1 + (alpha * np.tan(psi)) ** 2) * (np.pi / 2 / 400000)
    D = np.array([oracle.ggx_D(n, _hemi(t, 0.0), alpha) for t in theta[::40]])
    integrand = D * np.cos(theta[::40]) * np.sin(theta[::40]) * dtheta[::40] * 40
    assert 2 * np.pi * integrand.sum() == pytest.approx(1.0, rel=2e-4)


@pytest.mark.parametrize("alpha", [1e-3, 0.1, 0.7])
def test_ggx_D_peak(alpha):
    n = np.array([0.0, 0.0, 1.0])
    assert oracle.ggx_D(n, n, alpha) == pytest.approx(1.0 / (np.pi * alpha * alpha), rel=1e-14)


def _mat(r, nx=0.0, ny=0.0, albedo=(0.5, 0.25, 0.75)):
    return np.array([*albedo, r, nx, ny])


def _dir(theta, phi):
    return _hemi(theta, phi).astype(np.float32)


def test_reciprocity():
    rng = np.random.default_rng(1)
    for _ in range(200):
        m = _mat(rng.random(), rng.random() * 0.4 - 0.2, rng.random() * 0.4 - 0.2)
        wo = _dir(rng.random() * 1.4, rng.random() * 6.28)
        wi = _dir(rng.random() * 1.4, rng.random() * 6.28)
        n = np.array([m[4], m[5], np.sqrt(max(0.0, 1 - m[4] ** 2 - m[5] ** 2))])
        ni, no = n @ wi.astype(np.float64), n @ wo.astype(np.float64)
        if ni <= 0 or no <= 0:
            continue
        a = oracle.shade_eval(m, wo, wi) / ni
        b = oracle.shade_eval(m, wi, wo) / no
        assert np.allclose(a, b, rtol=1e-12)


def test_albedo_enters_affinely():
    # f^(albedo) - f^(albedo') = (albedo - albedo') cos_i / pi
    wo, wi = _dir(0.4, 0.3), _dir(0.9, 2.0)
    a = oracle.shade_eval(_mat(0.3, albedo=(0.1, 0.2, 0.3)), wo, wi)
    b = oracle.shade_eval(_mat(0.3, albedo=(0.6, 0.9, 0.0)), wo, wi)
    ci = float(wi.astype(np.float64)[2])
    assert np.allclose(a - b, (np.array([0.1, 0.2, 0.3]) - [0.6, 0.9, 0.0]) * ci / np.pi, rtol=1e-12, atol=1e-15)


def test_below_horizon_is_zero():
    m = _mat(0.3)
    assert np.all(oracle.shade_eval(m, _dir(0.3, 0), _dir(1.8, 0)) == 0)
    assert np.all(oracle.shade_eval(m, _dir(1.7, 0), _dir(0.2, 0)) == 0)


@pytest.mark.parametrize("r", [0.2, 0.5, 0.9])
def test_specular_directional_albedo_bounded(r):
    # int f_spec cos_i dw_i <= 1 (G2 <= 1, F <= 1): energy is not created
    wo = _dir(0.5, 0.0)
    black = _mat(r, albedo=(0.0, 0.0, 0.0))
    nt, nphi = 200, 200
    th = (np.arange(nt) + 0.5) / nt * (np.pi / 2)
    ph = (np.arange(nphi) + 0.5) / nphi * 2 * np.pi
    tot = 0.0
    for t in th:
        for p in ph[::4]:
            tot += oracle.shade_eval(black, wo, _dir(t, p))[0] * np.sin(t)
    tot *= (np.pi / 2 / nt) * (2 * np.pi / nphi * 4)
    assert 0.0 < tot < 1.0


def test_level_rule():
    assert oracle.shade_level(0.25, 3) == 0
    assert oracle.shade_level(1.4142134, 3) == 0
    assert oracle.shade_level(1.41421356, 3) == 1
    assert oracle.shade_level(2.0, 3) == 1
    assert oracle.shade_level(2.8284271, 3) == 2
    assert oracle.shade_level(4.0, 3) == 2
    assert oracle.shade_level(4.0, 2) == 1
    assert oracle.shade_level(4.0, 1) == 0


def _material_with(albedo_var=True, other_var=True, size=16, seed=3):
    rng = np.random.default_rng(seed)
    lv = synth.material_levels(size, seed=seed, levels=3)
    for m in lv:
        if not albedo_var:
            m["albedo"] = 128
        if not other_var:
            m["rough"] = 77
            m["nx"] = np.float16(0.125)
            m["ny"] = np.float16(-0.25)
    return lv


@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC])
def test_affine_texture_filter_order_does_not_matter(filt):
    # only the albedo varies: it enters f^ affinely, so filtering before or
    # after shading gives the same result
    mat = oracle.Material(_material_with(albedo_var=True, other_var=False))
    recs = synth.shade_queries(2000, seed=5)
    a, _ = mat.shade(recs, filt, oracle.SH_AFTER_FILTER)
    b, _ = mat.shade(recs, filt, oracle.SH_FILTER_AFTER)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC])
def test_constant_material_all_modes_agree(filt):
    lv = _material_with(albedo_var=False, other_var=False)
    mat = oracle.Material(lv)
    recs = synth.shade_queries(500, seed=6)
    a, _ = mat.shade(recs, filt, oracle.SH_AFTER_FILTER)
    b, _ = mat.shade(recs, filt, oracle.SH_FILTER_AFTER)
    c, _ = mat.shade(recs, filt, oracle.SH_STOCH, seed=1)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-14)
    assert np.allclose(b, c, rtol=1e-12, atol=1e-14)


def test_nonlinear_roughness_makes_the_orders_differ():
    mat = oracle.Material(_material_with(albedo_var=False, other_var=True, seed=7))
    recs = synth.shade_queries(2000, seed=8)
    a, _ = mat.shade(recs, oracle.CUBIC, oracle.SH_AFTER_FILTER)
    b, _ = mat.shade(recs, oracle.CUBIC, oracle.SH_FILTER_AFTER)
    assert np.max(np.abs(a - b)) > 1e-3


@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC])
def test_stochastic_shading_is_unbiased(filt):
    mat = oracle.Material(_material_with(seed=9))
    recs = synth.shade_queries(12, seed=10)
    recs[:, 2] = 0.5                                    # level 0
    recs[:, 5] = np.maximum(recs[:, 5], 0.3)            # keep both directions well above the horizon
    recs[:, 8] = np.maximum(recs[:, 8], 0.3)
    mean, var = mat.moments(recs, filt)
    K = 6000
    acc = np.zeros((12, 3))
    for k in range(K):
        v, _ = mat.shade(recs, filt, oracle.SH_STOCH, seed=500 + k, want_index=False, nthreads=1)
        acc += v
    ref, _ = mat.shade(recs, filt, oracle.SH_FILTER_AFTER)
    assert np.allclose(mean, ref, rtol=1e-12, atol=1e-15)
    live = var > 1e-20
    z = (acc / K - mean)[live] / np.sqrt(var[live] / K)
    assert np.all(np.abs(z) < 5.0), np.abs(z).max()


def _decode_material_np(lv0):
    """The six channels of every texel, decoded in numpy from the field
    layout (independent of the C decoder): v / 255 and binary16 widened."""
    H, W = lv0.shape
    d = np.empty((H, W, 6), np.float64)
    d[..., 0:3] = lv0["albedo"] / 255.0
    d[..., 3] = lv0["rough"] / 255.0
    d[..., 4] = lv0["nx"].astype(np.float64)
    d[..., 5] = lv0["ny"].astype(np.float64)
    return d


@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC])
def test_material_source_stochastic_reads_the_decoded_texel(filt):
    """A sampled tap returns exactly the six decoded channels of its texel
    (channel order, texel stride and both decodings pinned)."""
    lv0 = np.ascontiguousarray(synth.material_levels(48, seed=61, levels=1)[0])
    raw = lv0.view(np.uint8).reshape(48, 48, 8)
    uv = synth.uv_queries(3000, seed=62) * np.float32(1.2) - np.float32(0.1)
    dec = _decode_material_np(lv0)
    for mode in (oracle.STOCH, oracle.STOCH_FIS):
        v, idx = oracle.material_filter2d(raw, uv.astype(np.float32), filt, mode, seed=5)
        assert np.array_equal(v, dec[idx[:, 1], idx[:, 0]])


@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC, oracle.KEYS, oracle.MITCHELL])
def test_material_source_deterministic_matches_decoded_texture(filt):
    """Deterministic filtering of the material equals filtering its decoded
    channels stored as binary32 (within the rounding of the decode)."""
    lv0 = np.ascontiguousarray(synth.material_levels(40, seed=63, levels=1)[0])
    raw = lv0.view(np.uint8).reshape(40, 40, 8)
    uv = (synth.uv_queries(2000, seed=64) * np.float32(1.2) - np.float32(0.1)).astype(np.float32)
    dec32 = _decode_material_np(lv0).astype(np.float32)
    got, _ = oracle.material_filter2d(raw, uv, filt, oracle.DET)
    ref, _ = oracle.filter2d(dec32, oracle.F32, uv, filt, oracle.DET)
    scale, _ = oracle.filter2d(np.abs(dec32), oracle.F32, uv, filt, oracle.DET_ABS)
    assert np.all(np.abs(got - ref) <= 2 ** -23 * scale + 1e-300)
