"""Pins of the neural-texture oracle: its analytic gradient against central
finite differences, its reduction to plain bilinear interpolation when the
MLP is the identity on positive inputs (checked against scipy's own linear
interpolation), bfloat16 rounding against torch's conversion, and the
unbiasedness of decoding one sampled texel per lookup."""
import numpy as np
import pytest
import torch
from scipy import ndimage

import oracle


def _small(seed=1, LW=4, W=16, scale=0.3):
    rng = np.random.default_rng(seed)
    lat = rng.normal(0.0, 0.5, (LW, LW, 8))
    mlp = rng.normal(0.0, scale, oracle.NTEX_PARAMS)
    return oracle.NeuralTexture(lat, mlp, W, W), rng


def test_gradient_matches_finite_differences():
    nt, rng = _small()
    target = rng.random((16, 16, 8)).astype(np.float32)
    pos = rng.integers(0, 16, (24, 2)).astype(np.int32)
    loss, gl, gm = nt.loss_grad(target, pos)
    h = 1e-6
    for k in rng.choice(oracle.NTEX_PARAMS, 60, replace=False):
        m0 = nt.mlp[k]
        nt.mlp[k] = m0 + h
        lp, _, _ = nt.loss_grad(target, pos, want_grad=False)
        nt.mlp[k] = m0 - h
        lm, _, _ = nt.loss_grad(target, pos, want_grad=False)
        nt.mlp[k] = m0
        fd = (lp - lm) / (2 * h)
        assert fd == pytest.approx(gm[k], rel=1e-5, abs=1e-10)
    flat = nt.lat.reshape(-1)
    for k in rng.choice(flat.size, 60, replace=False):
        v0 = flat[k]
        flat[k] = v0 + h
        lp, _, _ = nt.loss_grad(target, pos, want_grad=False)
        flat[k] = v0 - h
        lm, _, _ = nt.loss_grad(target, pos, want_grad=False)
        flat[k] = v0
        fd = (lp - lm) / (2 * h)
        assert fd == pytest.approx(gl.reshape(-1)[k], rel=1e-5, abs=1e-10)


def _identity_mlp():
    mlp = np.zeros(oracle.NTEX_PARAMS)
    w1 = np.zeros((64, 8)); w1[:8, :8] = np.eye(8)
    w2 = np.zeros((64, 64)); w2[:8, :8] = np.eye(8)
    w3 = np.zeros((8, 64)); w3[:8, :8] = np.eye(8)
    mlp[0:512] = w1.ravel()
    mlp[576:4672] = w2.ravel()
    mlp[4736:5248] = w3.ravel()
    return mlp


def test_identity_mlp_reduces_to_bilinear_interpolation():
    rng = np.random.default_rng(2)
    LW, W = 8, 32
    lat = rng.random((LW, LW, 8)) + 0.1            # positive: the ReLUs pass it through
    nt = oracle.NeuralTexture(lat, _identity_mlp(), W, W)
    dec = nt.decode_all()
    # texel (i, j) samples the latent grid at (i + 1/2) LW/W - 1/2, edges clamped
    coords = (np.arange(W) + 0.5) * LW / W - 0.5
    yy, xx = np.meshgrid(coords, coords, indexing="ij")
    for c in range(8):
        ref = ndimage.map_coordinates(lat[:, :, c], [yy.ravel(), xx.ravel()], order=1, mode="nearest")
        assert np.allclose(dec[:, :, c].ravel(), ref, rtol=1e-13, atol=1e-15)


def test_round_bf16_matches_torch():
    rng = np.random.default_rng(3)
    x = (rng.normal(0, 1, 4000) * 10.0 ** rng.integers(-20, 20, 4000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([oracle.round_bf16(float(v)) for v in x])
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC])
def test_deterministic_filter_is_filter_of_decoded_texture(filt):
    nt, rng = _small(seed=4, LW=8, W=32)
    dec = nt.decode_all().astype(np.float64)
    uv = rng.random((500, 2)).astype(np.float32)
    got, _ = nt.filter(uv, filt, oracle.DET)
    lo, _ = oracle.filter2d(dec[:, :, :4].astype(np.float32), oracle.F32, uv, filt, oracle.DET)
    hi, _ = oracle.filter2d(dec[:, :, 4:].astype(np.float32), oracle.F32, uv, filt, oracle.DET)
    # the 2D oracle reads binary32 texels: compare at that precision
    assert np.allclose(got, np.concatenate([lo, hi], axis=1), rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC])
def test_one_decode_per_lookup_is_unbiased(filt):
    nt, rng = _small(seed=5, LW=8, W=32, scale=0.2)
    uv = (0.1 + 0.8 * rng.random((8, 2))).astype(np.float32)
    det, _ = nt.filter(uv, filt, oracle.DET)
    K = 4000
    s1 = np.zeros_like(det)
    s2 = np.zeros_like(det)
    for k in range(K):
        v, _ = nt.filter(uv, filt, oracle.STOCH, seed=900 + k, nthreads=1)
        s1 += v
        s2 += v * v
    mean = s1 / K
    var = np.maximum(s2 / K - mean ** 2, 1e-30)
    z = (mean - det) / np.sqrt(var / K)
    assert np.all(np.abs(z) < 5.0), np.abs(z).max()


def test_emulated_bf16_decode_is_close():
    nt, _ = _small(seed=6, LW=8, W=32, scale=0.2)
    for i, j in [(0, 0), (5, 17), (31, 31)]:
        a = nt.decode(i, j)
        b = nt.decode(i, j, emulate=True)
        assert np.max(np.abs(a - b)) < 0.05 * (np.max(np.abs(a)) + 1e-3)
