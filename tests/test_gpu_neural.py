"""GPU neural texture: training gradients against the FP64 oracle, training
progress, BF16-MFMA inference against the oracle that rounds at the same
points, unbiasedness of one decode per lookup, and what the trained network
gains over an untrained one and over a plain texture of equal memory."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_05810_amd as stf
import synth

pytestmark = pytest.mark.gpu

FILTERS = [("linear", stf.STF_LINEAR, oracle.LINEAR), ("cubic", stf.STF_CUBIC_BSPLINE, oracle.CUBIC)]
# BF16 inference against the oracle that rounds at the same points but sums in
# binary64: binary32 accumulation order and the binary32 latent interpolation
# before its bfloat16 rounding can move a hidden activation by one bfloat16 ulp
# (2^-8 relative); the worst measured output difference is 2.6e-3
INFER_ABS = 1e-2


def _f16(x):
    return np.asarray(x, np.float32).astype(np.float16).astype(np.float64)


@pytest.fixture(scope="module")
def small():
    target = synth.neural_target(64, seed=51)
    lat, mlp = synth.neural_init(16, seed=52)
    return target, lat, mlp


def test_gradients_match_oracle(dev, small):
    target, lat, mlp = small
    nt = stf.stf_ntex_create(64, 64, lat, mlp)
    rng = np.random.default_rng(1)
    pos = rng.integers(0, 64, (3000, 2)).astype(np.int32)
    gl = torch.empty((16, 16, 8), dtype=torch.float32, device=dev)
    gm = torch.empty(stf.stf_ntex_param_count(), dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    stf.stf_ntex_gradients(nt, torch.from_numpy(target).to(dev), torch.from_numpy(pos).to(dev), gl, gm, loss)
    on = oracle.NeuralTexture(lat, mlp, 64, 64)
    ol, ogl, ogm = on.loss_grad(target, pos)
    assert loss.item() == pytest.approx(ol, rel=1e-5)
    g_m, g_l = gm.cpu().numpy().astype(np.float64), gl.cpu().numpy().astype(np.float64)
    assert np.allclose(g_m, ogm, rtol=1e-4, atol=1e-4 * np.abs(ogm).max())
    assert np.allclose(g_l, ogl, rtol=1e-4, atol=1e-4 * np.abs(ogl).max())
    # the parameters are unchanged by a gradient evaluation
    l2, m2 = stf.stf_ntex_get_params(nt)
    assert np.array_equal(l2, lat) and np.array_equal(m2, mlp)
    nt.destroy()


def _psnr(a, b):
    mse = np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2)
    return 10 * np.log10(1.0 / mse)


def _decode_all(nt, dev):
    """Decoded texels through the MFMA filter at texel centres (bilinear at
    t = 0 returns the texel)."""
    js, is_ = np.meshgrid(np.arange(nt.H), np.arange(nt.W), indexing="ij")
    uv = np.stack([(is_ + 0.5) / nt.W, (js + 0.5) / nt.H], axis=-1).reshape(-1, 2).astype(np.float32)
    q = torch.from_numpy(uv).to(dev)
    out = torch.empty((uv.shape[0], 8), dtype=torch.float32, device=dev)
    stf.stf_ntex_filter(nt, q, stf.STF_LINEAR, stf.STF_DETERMINISTIC, 0, out)
    return out.cpu().numpy().reshape(nt.H, nt.W, 8)


@pytest.fixture(scope="module")
def trained(dev):
    size, lsize = 256, 64
    target = synth.neural_target(size, seed=61)
    lat, mlp = synth.neural_init(lsize, seed=62)
    nt = stf.stf_ntex_create(size, size, lat, mlp)
    stf.stf_ntex_prepare_inference(nt)
    untrained = _decode_all(nt, dev)
    tgt = torch.from_numpy(target).to(dev)
    steps = 600
    loss = torch.empty(steps, dtype=torch.float32, device=dev)
    stf.stf_ntex_train(nt, tgt, steps, 1 << 14, 1e-2, 1e-3, 7, loss)
    stf.stf_ntex_prepare_inference(nt)
    return nt, target, untrained, loss.cpu().numpy()


def test_training_lowers_the_loss(trained):
    nt, target, untrained, loss = trained
    assert np.all(np.isfinite(loss))
    assert loss[-20:].mean() < 0.1 * loss[:5].mean()


def test_trained_network_beats_untrained_and_equal_memory_texture(dev, trained):
    nt, target, untrained, loss = trained
    dec = _decode_all(nt, dev)
    p_trained, p_untrained = _psnr(dec, target), _psnr(untrained, target)
    # a plain texture of the same memory as the latents: 4x fewer texels per
    # axis (box average), reconstructed bilinearly at full resolution
    small = target.reshape(64, 4, 64, 4, 8).mean(axis=(1, 3)).astype(np.float32)
    uv = np.stack(np.meshgrid((np.arange(256) + 0.5) / 256, (np.arange(256) + 0.5) / 256, indexing="xy"),
                  axis=-1).reshape(-1, 2).astype(np.float32)
    lo, _ = oracle.filter2d(np.ascontiguousarray(small[:, :, :4]), oracle.F32, uv, oracle.LINEAR, oracle.DET)
    hi, _ = oracle.filter2d(np.ascontiguousarray(small[:, :, 4:]), oracle.F32, uv, oracle.LINEAR, oracle.DET)
    base = np.concatenate([lo, hi], axis=1).reshape(256, 256, 8)
    p_base = _psnr(base, target)
    print(f"PSNR trained {p_trained:.2f} dB, untrained {p_untrained:.2f} dB, equal-memory bilinear {p_base:.2f} dB")
    assert p_trained > p_untrained + 10.0
    assert p_trained > p_base


@pytest.mark.parametrize("fname,gf,of", FILTERS)
def test_inference_matches_bf16_oracle(dev, trained, fname, gf, of):
    nt, target, _, _ = trained
    lat, mlp = stf.stf_ntex_get_params(nt)
    on = oracle.NeuralTexture(_f16(lat), mlp, nt.W, nt.H)
    rng = np.random.default_rng(5)
    uv = rng.random((4096, 2)).astype(np.float32)
    uv[:4] = [[0, 0], [1 - 2 ** -24, 0.5], [np.nan, 0.5], [0.5, 0.5]]
    q = torch.from_numpy(uv).to(dev)
    out = torch.empty((4096, 8), dtype=torch.float32, device=dev)
    idx = torch.empty((4096, 2), dtype=torch.int32, device=dev)
    stf.stf_ntex_filter(nt, q, gf, stf.STF_STOCHASTIC, 9, out, idx)
    ov, oi = on.filter(uv, of, oracle.STOCH, seed=9, emulate=True)
    assert np.array_equal(idx.cpu().numpy(), oi)
    g = out.cpu().numpy().astype(np.float64)
    fin = ~np.isnan(ov)
    assert np.array_equal(np.isnan(g), ~fin)
    err = np.abs(g[fin] - ov[fin])
    print(f"{fname} stochastic: max abs {err.max():.3g}, p99.9 {np.percentile(err, 99.9):.3g}")
    assert err.max() < INFER_ABS
    stf.stf_ntex_filter(nt, q, gf, stf.STF_DETERMINISTIC, 0, out)
    od, _ = on.filter(uv, of, oracle.DET, emulate=True)
    g = out.cpu().numpy().astype(np.float64)
    err = np.abs(g[fin] - od[fin])
    print(f"{fname} deterministic: max abs {err.max():.3g}, p99.9 {np.percentile(err, 99.9):.3g}")
    assert err.max() < INFER_ABS


def _tap_distribution(uv, W, H, cubic):
    """The taps a stochastic lookup draws from and their probabilities (the
    per-axis linear or cubic B-spline weights, in binary64): (n, T, 2) texel
    coordinates (clamped) and (n, T) probabilities."""
    def axis(x, size):
        c = np.floor(x)
        t = x - c
        if cubic:
            offs = np.array([-1, 0, 1, 2])
            w = np.stack([(1 - t) ** 3, 3 * t ** 3 - 6 * t ** 2 + 4, -3 * t ** 3 + 3 * t ** 2 + 3 * t + 1, t ** 3],
                         axis=1) / 6.0
        else:
            offs = np.array([0, 1])
            w = np.stack([1 - t, t], axis=1)
        return np.clip(c[:, None].astype(np.int64) + offs[None, :], 0, size - 1), w
    x = uv[:, 0].astype(np.float64) * W - 0.5
    y = uv[:, 1].astype(np.float64) * H - 0.5
    ix, wx = axis(x, W)
    iy, wy = axis(y, H)
    k = ix.shape[1]
    taps = np.stack([np.tile(ix, (1, k)), np.repeat(iy, k, axis=1)], axis=-1)   # tap t = (x t mod k, y t div k)
    p = np.tile(wx, (1, k)) * np.repeat(wy, k, axis=1)
    return taps, p


@pytest.mark.parametrize("fname,gf,of", FILTERS)
def test_one_decode_per_lookup_is_unbiased(dev, trained, fname, gf, of):
    # The mean of K one-decode lookups against the deterministic filter.  The
    # bound is Bernstein's for a bounded variable, with the exact variance
    # and range of the estimator: each tap's decoded value (the deterministic
    # filter at that texel's centre, where the bilinear weights are 1 and 0)
    # and probability (its weight) give them.  Neighbouring texels whose
    # bfloat16 latents coincide decode alike, so a query's estimator is often
    # a rare tap against a constant: a sample variance would then read 0
    # whenever the rare tap was not drawn, where the exact one does not.
    nt, _, _, _ = trained
    rng = np.random.default_rng(11)
    n = 64
    uv = (0.05 + 0.9 * rng.random((n, 2))).astype(np.float32)
    q = torch.from_numpy(uv).to(dev)
    det = torch.empty((n, 8), dtype=torch.float32, device=dev)
    stf.stf_ntex_filter(nt, q, gf, stf.STF_DETERMINISTIC, 0, det)
    taps, p = _tap_distribution(uv, nt.W, nt.H, gf == stf.STF_CUBIC_BSPLINE)
    T = taps.shape[1]
    centres = ((taps.reshape(-1, 2) + 0.5) / np.array([nt.W, nt.H])).astype(np.float32)
    vt = torch.empty((n * T, 8), dtype=torch.float32, device=dev)
    stf.stf_ntex_filter(nt, torch.from_numpy(centres).to(dev), stf.STF_LINEAR, stf.STF_DETERMINISTIC, 0, vt)
    v = vt.cpu().numpy().astype(np.float64).reshape(n, T, 8)
    mu = np.einsum("nt,ntc->nc", p, v)
    var = np.einsum("nt,ntc->nc", p, (v - mu[:, None, :]) ** 2)
    rng_t = np.max(np.abs(v - mu[:, None, :]), axis=1)
    d = det.cpu().numpy().astype(np.float64)
    scale = np.max(np.abs(v), axis=1)
    # the deterministic filter is the weighted sum of the same decodes, in binary32
    assert np.all(np.abs(d - mu) <= 1e-5 * scale + 1e-12), np.max(np.abs(d - mu) / np.maximum(scale, 1e-30))
    K = 3000
    out = torch.empty((n, 8), dtype=torch.float32, device=dev)
    s1 = torch.zeros((n, 8), dtype=torch.float64, device=dev)
    for k in range(K):
        stf.stf_ntex_filter(nt, q, gf, stf.STF_STOCHASTIC, 100 + k, out)
        s1 += out.double()
    mean = (s1 / K).cpu().numpy()
    L = np.log(2.0 / 1e-9)   # each bound fails with probability below 1e-9
    bound = np.sqrt(2.0 * var * L / K) + 2.0 * rng_t * L / (3.0 * K) + 1e-5 * scale + 1e-12
    err = np.abs(mean - d)
    print(f"{fname}: largest |mean - deterministic| / bound {(err / bound).max():.3f}")
    assert np.all(err <= bound), (err / bound).max()


def test_neural_argument_errors(dev, small):
    target, lat, mlp = small
    with pytest.raises(stf.STFError) as e:
        stf.stf_ntex_create(60, 64, lat, mlp)
    assert e.value.status == stf.STF_E_UNSUPPORTED
    nt = stf.stf_ntex_create(64, 64, lat, mlp)
    q = torch.zeros((4, 2), dtype=torch.float32, device=dev)
    out = torch.empty((4, 8), dtype=torch.float32, device=dev)
    with pytest.raises(stf.STFError):   # not prepared for inference yet
        stf.stf_ntex_filter(nt, q, stf.STF_LINEAR, stf.STF_STOCHASTIC, 0, out)
    stf.stf_ntex_prepare_inference(nt)
    with pytest.raises(stf.STFError):
        stf.stf_ntex_filter(nt, q, stf.STF_LINEAR, stf.STF_DETERMINISTIC, 0, out,
                            torch.empty((4, 2), dtype=torch.int32, device=dev))
    nt.destroy()
