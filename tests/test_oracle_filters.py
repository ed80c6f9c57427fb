"""Pins of the oracle's 2D and 3D filters against closed forms, brute force,
exact decoding, a plain dense array and the unbiasedness of the single-tap
estimator (Eqs. filtered-texture and stochastic-sum)."""
import numpy as np
import pytest
import torch

import oracle
from tests._util import dense_masked, leaves_from_dense


# ----------------------------------------------------------------------------
# exact decoders (storage format -> binary64)
# ----------------------------------------------------------------------------
def test_decode_f16_exhaustive():
    raw = np.arange(1 << 16, dtype=np.uint16)
    ref = raw.view(np.float16).astype(np.float64)
    got = oracle.decode(oracle.F16, raw)
    fin = np.isfinite(ref)
    assert np.array_equal(got[fin], ref[fin])
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    assert np.array_equal(np.isinf(got), np.isinf(ref))


def test_decode_bf16_exhaustive():
    raw = np.arange(1 << 16, dtype=np.uint16)
    with np.errstate(invalid="ignore"):   # the signalling-NaN patterns
        ref = (raw.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    got = oracle.decode(oracle.BF16, raw)
    fin = np.isfinite(ref)
    assert np.array_equal(got[fin], ref[fin])
    assert np.array_equal(np.isnan(got), np.isnan(ref))


def test_decode_e4m3_exhaustive():
    raw = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(raw).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = oracle.decode(oracle.FP8_E4M3, raw)
    fin = np.isfinite(ref)
    assert np.array_equal(got[fin], ref[fin])
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    assert np.nanmax(got) == 448.0


def test_decode_u8():
    raw = np.arange(256, dtype=np.uint8)
    got = oracle.decode(oracle.U8, raw)
    assert np.array_equal(got, raw / 255.0)


# ----------------------------------------------------------------------------
# closed forms
# ----------------------------------------------------------------------------
def _dense_grid(field, fmt=oracle.F32):
    o, v = leaves_from_dense(field)
    return oracle.Grid((field.shape[2], field.shape[1], field.shape[0]), fmt, o, v.astype(np.float32))


def _coords(n):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC])
def test_3d_reproduces_products_of_affine_functions(filt):
    n = 32
    X, Y, Z = _coords(n)
    f = lambda x, y, z: (0.5 + 0.25 * x) * (2.0 - 0.03125 * y) * (1.0 + 0.125 * z)
    g = _dense_grid(f(X, Y, Z).astype(np.float32))
    rng = np.random.default_rng(1)
    p = (2.0 + rng.random((500, 3)) * (n - 5.0)).astype(np.float32)
    got, _ = g.filter(p, filt, oracle.DET)
    ref = f(*(p.astype(np.float64).T))
    assert np.allclose(got, ref, rtol=1e-12, atol=0)


def test_3d_cubic_quadratic_gains_one_third():
    # sum_k w_k (k-1)^2 = t^2 + 1/3: the field x^2 filters to x^2 + 1/3
    n = 32
    X, _, _ = _coords(n)
    g = _dense_grid((X * X).astype(np.float32))
    rng = np.random.default_rng(2)
    p = (2.0 + rng.random((300, 3)) * (n - 5.0)).astype(np.float32)
    got, _ = g.filter(p, oracle.CUBIC, oracle.DET)
    x = p[:, 0].astype(np.float64)
    assert np.allclose(got, x * x + 1.0 / 3.0, rtol=1e-12, atol=0)


def test_3d_linear_quadratic_gains_t_one_minus_t():
    # linear interpolation of x^2 between i and i+1 is x^2 + t (1 - t)
    n = 24
    X, _, _ = _coords(n)
    g = _dense_grid((X * X).astype(np.float32))
    rng = np.random.default_rng(3)
    p = (1.0 + rng.random((300, 3)) * (n - 3.0)).astype(np.float32)
    got, _ = g.filter(p, oracle.LINEAR, oracle.DET)
    x = p[:, 0].astype(np.float64)
    t = x - np.floor(x)
    assert np.allclose(got, x * x + t * (1 - t), rtol=1e-12, atol=0)


def test_3d_texel_centres():
    # at integer positions linear returns the voxel, cubic the [1 4 1]/6 stencil
    n = 16
    rng = np.random.default_rng(4)
    field = rng.random((n, n, n)).astype(np.float32)
    g = _dense_grid(field)
    pts = np.array([[5, 6, 7], [8, 8, 8], [3, 10, 12]], np.float32)
    lin, _ = g.filter(pts, oracle.LINEAR, oracle.DET)
    cub, _ = g.filter(pts, oracle.CUBIC, oracle.DET)
    k = np.array([1.0, 4.0, 1.0]) / 6.0
    for q, (x, y, z) in enumerate(pts.astype(int)):
        assert lin[q] == field[z, y, x]
        blk = field[z - 1:z + 2, y - 1:y + 2, x - 1:x + 2].astype(np.float64)
        ref = np.einsum("i,j,k,ijk->", k, k, k, blk)
        assert cub[q] == pytest.approx(ref, rel=1e-14)


@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC])
def test_2d_reproduces_products_of_affine_functions(filt):
    W, H = 32, 16
    xs = np.arange(W, dtype=np.float64)
    ys = np.arange(H, dtype=np.float64)
    coef = [(1.0, 0.5, 2.0, -0.0625), (0.25, 0.125, 1.0, 0.25), (3.0, -0.0625, 0.5, 0.5)]
    tex = np.stack([np.outer(c + d * ys, a + b * xs) for a, b, c, d in coef], axis=2).astype(np.float32)
    rng = np.random.default_rng(5)
    uv = np.stack([(2.0 + rng.random(400) * (W - 5.0) + 0.5) / W,
                   (2.0 + rng.random(400) * (H - 5.0) + 0.5) / H], axis=1).astype(np.float32)
    got, _ = oracle.filter2d(tex, oracle.F32, uv, filt, oracle.DET)
    # the raster position the filter sees: binary32 uv*W - 0.5
    x = (uv[:, 0] * np.float32(W) - np.float32(0.5)).astype(np.float64)
    y = (uv[:, 1] * np.float32(H) - np.float32(0.5)).astype(np.float64)
    for c, (a, b, cc, d) in enumerate(coef):
        assert np.allclose(got[:, c], (a + b * x) * (cc + d * y), rtol=1e-12, atol=0)


# ----------------------------------------------------------------------------
# brute force: every texel weighted by the kernel at its distance
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC])
def test_2d_separable_equals_brute_force(filt):
    rng = np.random.default_rng(6)
    tex = rng.random((8, 8, 3)).astype(np.float32)
    uv = (rng.random((2000, 2)) * 1.6 - 0.3).astype(np.float32)   # includes clamped borders
    sep, _ = oracle.filter2d(tex, oracle.F32, uv, filt, oracle.DET)
    bru = oracle.filter2d_brute(tex, oracle.F32, uv, filt)
    assert np.allclose(sep, bru, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC])
def test_3d_separable_equals_brute_force(filt):
    rng = np.random.default_rng(7)
    field = rng.random((24, 24, 24)).astype(np.float32)
    keep = rng.random((3, 3, 3)) < 0.6
    o, v = leaves_from_dense(field, keep)
    g = oracle.Grid((24, 24, 24), oracle.F32, o, v, background=0.0)
    p = (rng.random((1500, 3)) * 30.0 - 3.0).astype(np.float32)   # includes outside the domain
    sep, _ = g.filter(p, filt, oracle.DET)
    bru = g.filter_brute(p, filt)
    assert np.allclose(sep, bru, rtol=1e-14, atol=1e-15)


# ----------------------------------------------------------------------------
# the sparse grid is the dense array of the same field
# ----------------------------------------------------------------------------
def test_sparse_grid_texels_equal_dense_array():
    rng = np.random.default_rng(8)
    field = rng.random((16, 24, 32)).astype(np.float32)     # z, y, x
    keep = rng.random((2, 3, 4)) < 0.5
    o, v = leaves_from_dense(field, keep)
    g = oracle.Grid((32, 24, 16), oracle.F32, o, v, background=0.25)
    dense = dense_masked(field, keep)
    for _ in range(3000):
        x, y, z = rng.integers(-3, 35), rng.integers(-3, 27), rng.integers(-3, 19)
        inside = 0 <= x < 32 and 0 <= y < 24 and 0 <= z < 16
        if inside and keep[z // 8, y // 8, x // 8]:
            assert g.texel(x, y, z) == dense[z, y, x]
        else:
            assert g.texel(x, y, z) == 0.25


@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC])
def test_sparse_filter_equals_dense_filter(filt):
    rng = np.random.default_rng(9)
    field = rng.random((24, 24, 24)).astype(np.float32)
    keep = rng.random((3, 3, 3)) < 0.5
    o, v = leaves_from_dense(field, keep)
    sparse = oracle.Grid((24, 24, 24), oracle.F32, o, v)
    full = _dense_grid(dense_masked(field, keep))
    p = (rng.random((2000, 3)) * 28.0 - 2.0).astype(np.float32)
    a, _ = sparse.filter(p, filt, oracle.DET)
    b, _ = full.filter(p, filt, oracle.DET)
    assert np.array_equal(a, b)
    sa, ia = sparse.filter(p, filt, oracle.STOCH, seed=3)
    sb, ib = full.filter(p, filt, oracle.STOCH, seed=3)
    assert np.array_equal(ia, ib) and np.array_equal(sa, sb)


def test_grid_rejects_bad_leaves():
    v = np.zeros((2, 8, 8, 8), np.float32)
    with pytest.raises(ValueError):
        oracle.Grid((16, 16, 16), oracle.F32, np.array([[0, 0, 0], [0, 0, 0]]), v)     # duplicate
    with pytest.raises(ValueError):
        oracle.Grid((16, 16, 16), oracle.F32, np.array([[0, 0, 0], [4, 0, 0]]), v)     # not a multiple of 8
    with pytest.raises(ValueError):
        oracle.Grid((16, 16, 16), oracle.F32, np.array([[0, 0, 0], [16, 0, 0]]), v)    # outside


# ----------------------------------------------------------------------------
# stochastic filter: one real tap of positive weight, exact value
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC])
def test_3d_stochastic_returns_a_tap_of_positive_weight(filt):
    rng = np.random.default_rng(10)
    field = rng.random((16, 16, 16)).astype(np.float32)
    g = _dense_grid(field)
    p = (rng.random((3000, 3)) * 18.0 - 1.0).astype(np.float32)
    p[:200] = np.round(p[:200])                   # texel centres: t = 0
    val, idx = g.filter(p, filt, oracle.STOCH, seed=5)
    lo = np.floor(p).astype(int)
    for q in range(p.shape[0]):
        w = 1.0
        for a in range(3):
            off = idx[q, a] - lo[q, a]
            t = float(p[q, a]) - lo[q, a]
            wa = oracle.axis_weights(filt, t)
            k = off + (1 if filt == oracle.CUBIC else 0)
            assert 0 <= k < (4 if filt == oracle.CUBIC else 2)
            w *= wa[k]
        assert w > 0.0
        assert val[q] == g.texel(*idx[q])


def test_nonfinite_queries():
    g = _dense_grid(np.ones((8, 8, 8), np.float32))
    p = np.array([[np.nan, 1, 1], [1, np.inf, 1], [1, 1, 2.0 ** 24], [1, 1, -2.0 ** 25], [3, 3, 3]], np.float32)
    for filt in (oracle.LINEAR, oracle.CUBIC):
        v, idx = g.filter(p, filt, oracle.STOCH, seed=1)
        assert np.all(np.isnan(v[:4])) and np.all(idx[:4] == oracle.BAD_INDEX) and v[4] == 1.0
        d, _ = g.filter(p, filt, oracle.DET)
        assert np.all(np.isnan(d[:4])) and d[4] == pytest.approx(1.0)


# ----------------------------------------------------------------------------
# unbiasedness (Eq. stochastic-sum): mean over seeds -> deterministic value
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [oracle.STOCH, oracle.STOCH_REUSE])
@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC])
def test_3d_unbiased_within_5_sigma(filt, mode):
    rng = np.random.default_rng(11)
    field = rng.random((16, 16, 16)).astype(np.float32)
    g = _dense_grid(field)
    p = (2.0 + rng.random((16, 3)) * 11.0).astype(np.float32)
    K = 6000
    s1 = np.zeros(16)
    for k in range(K):
        v, _ = g.filter(p, filt, mode, seed=1000 + k, want_index=False, nthreads=1)   # 16 queries: one thread
        s1 += v
    mean, var = g.moments(p, filt)
    det, _ = g.filter(p, filt, oracle.DET)
    assert np.allclose(mean, det, rtol=1e-13)
    assert np.all(var > 0)
    z = (s1 / K - mean) / np.sqrt(var / K)
    assert np.all(np.abs(z) < 5.0), z


def test_2d_stochastic_clamps_and_is_exact():
    rng = np.random.default_rng(12)
    tex = rng.random((8, 8, 4)).astype(np.float32)
    uv = (rng.random((3000, 2)) * 1.6 - 0.3).astype(np.float32)
    for filt in (oracle.LINEAR, oracle.CUBIC):
        v, idx = oracle.filter2d(tex, oracle.F32, uv, filt, oracle.STOCH, seed=9)
        assert idx.min() >= 0 and idx.max() <= 7
        assert np.array_equal(v, tex[idx[:, 1], idx[:, 0]].astype(np.float64))
