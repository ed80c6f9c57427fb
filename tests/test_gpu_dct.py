"""GPU parity of DCT-compressed textures (single-texel decode in binary32)
through the C ABI against the FP64 oracle on identical blocks.

Bar: stochastic -- the drawn taps equal the oracle's for every query; every
value is within 1e-6 of the oracle relative to its absolute scale: A(t) =
sum_k |c_k b_k(t)| for a decoded texel t (the six dequantised coefficient
terms), sum |w| A over the taps for deterministic filters, and S+ A(j+) +
S- A(j-) for the positivized cubics."""
import numpy as np
import pytest
import torch
from scipy import fft

import oracle
import paper_2305_05810_amd as stf
import synth

pytestmark = pytest.mark.gpu

ZZ = [(0, 0), (0, 1), (1, 0), (2, 0), (1, 1), (0, 2)]
FILTERS = [("linear", stf.STF_LINEAR, oracle.LINEAR), ("bspline", stf.STF_CUBIC_BSPLINE, oracle.CUBIC),
           ("keys", stf.STF_CUBIC_KEYS, oracle.KEYS), ("mitchell", stf.STF_CUBIC_MITCHELL, oracle.MITCHELL)]
REL = 1e-6


def _staged(fn):
    """(blocks that staged their taps in LDS, blocks) of the staged kernels
    during fn()."""
    stf.stf_stage_counting(True)
    try:
        fn()
        return stf.stf_stage_counts()
    finally:
        stf.stf_stage_counting(False)


def _abs_terms(words):
    """A(x, y, c) = sum_k |dequant_k * basis_k(x, y)| for every texel."""
    BH, BW, Ch = words.shape
    basis = []
    for v, u in ZZ:
        e = np.zeros((8, 8))
        e[v, u] = 1.0
        basis.append(np.abs(fft.idctn(e, type=2, norm="ortho")))   # [y, x]
    out = np.zeros((BH * 8, BW * 8, Ch))
    w = words.astype(np.int64)
    deq = [(w & 127) * 8 / 127] + [(((w >> (7 + 5 * (k - 1))) & 31) - 16) * 2 / 15 for k in range(1, 6)]
    for k in range(6):
        out += np.abs(np.repeat(np.repeat(deq[k], 8, 0), 8, 1)) * np.tile(basis[k], (BH, BW))[:, :, None]
    return out


def _texture(H, W, C, seed):
    """Smooth 8-bit texels plus noise: the kind of content block DCT codes."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:H, 0:W]
    base = np.stack([np.sin(xx / (5.0 + c) + c) * np.cos(yy / (7.0 + 2 * c)) for c in range(C)], axis=-1)
    tex = 127.5 + 100 * base + rng.normal(0, 12, (H, W, C))
    return np.clip(np.round(tex), 0, 255).astype(np.uint8)


@pytest.fixture(scope="module", params=[(96, 80, 9), (64, 40, 3), (40, 48, 16)], ids=["c9", "c3", "c16"])
def dct_inputs(request):
    W, H, C = request.param
    tex = _texture(H, W, C, seed=W + C)
    words = stf.stf_dct_encode(tex)
    uv = synth.uv_queries(20000, seed=C) * np.float32(1.1) - np.float32(0.05)
    uv[:8] = [[np.nan, 0.5], [0.5, np.inf], [1e30, 0.5], [-0.7, 1.4], [0, 0], [1, 1], [0.5, 0.5], [0.25, 0.75]]
    return W, H, C, words, uv.astype(np.float32)


@pytest.mark.parametrize("fname,gf,of", FILTERS)
def test_dct_parity(dev, dct_inputs, fname, gf, of):
    W, H, C, words, uv = dct_inputs
    t = stf.stf_create_dct_texture2d(W, H, C, words)
    assert stf.stf_texture_bytes(t) == (W // 8) * (H // 8) * ((C + 3) // 4 * 4) * 4
    q = torch.from_numpy(uv).to(dev)
    A = _abs_terms(words).astype(np.float32)
    seed = 0xD0C7
    gv, gi = stf.filter(t, q, gf, stf.STF_STOCHASTIC, seed, want_index=True)
    gv, gi = gv.cpu().numpy().astype(np.float64), gi.cpu().numpy()
    ov, oi = oracle.dct_filter2d(words, uv, of, oracle.STOCH, seed)
    assert np.array_equal(gi, oi), f"{fname}: {np.sum(np.any(gi != oi, axis=1))} index mismatches"
    fin = oi[:, 0] != oracle.BAD_INDEX
    scale = np.zeros_like(ov)
    if of in oracle.POSITIVIZED:
        x = uv[:, 0].astype(np.float32) * np.float32(W) - np.float32(0.5)
        y = uv[:, 1].astype(np.float32) * np.float32(H) - np.float32(0.5)
        for k in np.nonzero(fin)[0]:
            tt = [float(x[k]) - float(np.floor(x[k])), float(y[k]) - float(np.floor(y[k]))]
            sp, sn = oracle.positivized_masses(of, tt)
            scale[k] = sp * A[oi[k, 1], oi[k, 0]]
            if oi[k, 2] != oracle.BAD_INDEX:
                scale[k] += sn * A[oi[k, 3], oi[k, 2]]
    else:
        scale[fin] = A[oi[fin, 1], oi[fin, 0]]
    err = np.abs(gv - ov)
    ok = (np.isnan(gv) & np.isnan(ov)) | (err <= REL * scale)
    worst = np.nanmax(np.where(scale > 0, err / np.where(scale > 0, scale, 1), 0))
    assert ok.all(), f"{fname} stoch: {np.sum(~ok)} outside (worst {worst:.3g})"
    gd, _ = stf.filter(t, q, gf, stf.STF_DETERMINISTIC, 0)
    gd = gd.cpu().numpy().astype(np.float64)
    od, _ = oracle.dct_filter2d(words, uv, of, oracle.DET)
    dscale, _ = oracle.filter2d(A, oracle.F32, uv, of, oracle.DET_ABS)
    err = np.abs(gd - od)
    ok = (np.isnan(gd) & np.isnan(od)) | (err <= REL * dscale)
    dworst = np.nanmax(np.where(dscale > 0, err / np.where(dscale > 0, dscale, 1), 0))
    assert ok.all(), f"{fname} det: {np.sum(~ok)} outside (worst {dworst:.3g})"
    print(f"dct c{C} {fname}: worst rel stoch {worst:.3g} det {dworst:.3g}")
    t.destroy()


@pytest.mark.parametrize("fname,gf,of", [FILTERS[1], FILTERS[2]])
def test_dct_moments_unbiased_5_sigma(dev, fname, gf, of):
    tex = _texture(64, 64, 4, seed=3)
    words = stf.stf_dct_encode(tex)
    t = stf.stf_create_dct_texture2d(64, 64, 4, words)
    uv = synth.uv_queries(512, seed=9)
    q = torch.from_numpy(uv).to(dev)
    K = 8192
    s1 = torch.empty(512, dtype=torch.float64, device=dev)
    s2 = torch.empty_like(s1)
    stf.stf_filter_moments(t, q, gf, 31, K, s1, s2)
    mean, var = oracle.dct_moments2d(words, uv, of)
    mean, var = mean[:, 0], var[:, 0]
    live = var > 1e-12
    z = (s1.cpu().numpy() / K - mean)[live] / np.sqrt(var[live] / K)
    assert live.sum() > 400 and np.all(np.abs(z) < 5.0), np.abs(z).max()
    t.destroy()


def test_dct_ordered_stream_and_errors(dev):
    tex = _texture(64, 64, 9, seed=4)
    words = stf.stf_dct_encode(tex)
    t = stf.stf_create_dct_texture2d(64, 64, 9, words)
    uv = synth.uv_queries(5000, seed=10)
    q = torch.from_numpy(uv).to(dev)
    a, ia = stf.filter(t, q, stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 3, want_index=True)
    sq, order = stf.sort_queries(t, q)
    out = torch.empty_like(a)
    idx = torch.empty_like(ia)
    stf.stf_filter_ordered(t, sq, order, stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 3, out, idx, stf.STF_ORDER_SCATTER)
    assert torch.equal(idx, ia) and torch.equal(out, a)
    with pytest.raises(stf.STFError):
        stf.stf_create_dct_texture2d(60, 64, 9, np.zeros((8, 7, 9), np.uint32))   # width not a multiple of 8
    L = stf.lib()
    sq9 = torch.zeros((4, 9), dtype=torch.float32, device=dev)
    rgb = torch.empty((4, 3), dtype=torch.float32, device=dev)
    assert L.stf_shade_filter(t.handle, sq9.data_ptr(), 4, 1, 0, 0, rgb.data_ptr(), None, None) == stf.STF_E_INVALID
    t.destroy()


@pytest.mark.parametrize("fname,gf,of", FILTERS)
@pytest.mark.parametrize("W,H,C", [(96, 80, 9), (64, 48, 16)])
def test_dct_sorted_stream_staged_decode(dev, fname, gf, of, W, H, C):
    """A Morton-sorted stream: deterministic bicubic blocks decode the texels
    of their taps once into LDS (blocks whose taps span too many texels decode
    per tap).  Values within the bar of the oracle, and bit for bit those of
    the unsorted call (uniform uv: its blocks' boxes are too large to stage,
    so every tap is decoded on its own)."""
    tex = _texture(H, W, C, seed=W + 7)
    words = stf.stf_dct_encode(tex)
    t = stf.stf_create_dct_texture2d(W, H, C, words)
    uv = synth.uv_queries(30000, seed=W) * np.float32(1.1) - np.float32(0.05)
    q = torch.from_numpy(uv).to(dev)
    res = {}
    staged, blocks = _staged(lambda: res.update(ref=stf.filter(t, q, gf, stf.STF_DETERMINISTIC, 0)[0]))
    ref = res["ref"]
    nblocks = 0 if gf == stf.STF_LINEAR else (uv.shape[0] + 255) // 256   # bilinear: never the staged kernel
    assert blocks == nblocks and staged == 0                       # uniform uv: no block box fits
    sq, order = stf.sort_queries(t, q)
    out = torch.empty_like(ref)
    staged, blocks = _staged(lambda: stf.stf_filter_ordered(t, sq, order, gf, stf.STF_DETERMINISTIC, 0, out, None,
                                                            stf.STF_ORDER_SCATTER))
    assert blocks == nblocks and (gf == stf.STF_LINEAR or staged > blocks // 2), (staged, blocks)   # sorted
    assert torch.equal(out.nan_to_num(-7), ref.nan_to_num(-7)), fname
    gd = out.cpu().numpy().astype(np.float64)
    od, _ = oracle.dct_filter2d(words, uv, of, oracle.DET)
    A = _abs_terms(words).astype(np.float32)
    dscale, _ = oracle.filter2d(A, oracle.F32, uv, of, oracle.DET_ABS)
    assert np.all((np.isnan(gd) & np.isnan(od)) | (np.abs(gd - od) <= REL * dscale)), fname
    t.destroy()


@pytest.mark.parametrize("fname,gf,of", FILTERS[1:])
def test_dct_frame_order_staged_decode(dev, fname, gf, of):
    """A frame in pixel order magnifying the texture: each block's 256 pixels
    cover a small texel box, so deterministic bicubic / Keys / Mitchell blocks
    decode that box once into LDS.  The same queries shuffled (no block box
    fits, every tap decoded on its own) give the same bits, and both meet the
    oracle's bar."""
    W, H, C = 96, 80, 9
    tex = _texture(H, W, C, seed=W + 11)
    words = stf.stf_dct_encode(tex)
    t = stf.stf_create_dct_texture2d(W, H, C, words)
    fw, fh = 4 * W, 4 * H
    ys, xs = np.mgrid[0:fh, 0:fw]
    uv = np.stack([(xs + 0.37) / fw, (ys + 0.61) / fh], axis=-1).reshape(-1, 2).astype(np.float32)
    perm = np.random.default_rng(12).permutation(uv.shape[0])
    res = {}
    staged, blocks = _staged(lambda: res.update(f=stf.filter(t, torch.from_numpy(uv).to(dev), gf,
                                                             stf.STF_DETERMINISTIC, 0)[0]))
    assert staged == blocks == uv.shape[0] // 256, (staged, blocks)   # every block of the frame stages
    staged, blocks = _staged(lambda: res.update(s=stf.filter(t, torch.from_numpy(uv[perm]).to(dev), gf,
                                                             stf.STF_DETERMINISTIC, 0)[0]))
    assert staged == 0 and blocks == uv.shape[0] // 256, (staged, blocks)
    framed, shuffled = res["f"], res["s"]
    back = torch.empty_like(shuffled)
    back[torch.from_numpy(perm).to(dev)] = shuffled
    assert torch.equal(framed, back), fname
    gd = framed.cpu().numpy().astype(np.float64)
    od, _ = oracle.dct_filter2d(words, uv, of, oracle.DET)
    A = _abs_terms(words).astype(np.float32)
    dscale, _ = oracle.filter2d(A, oracle.F32, uv, of, oracle.DET_ABS)
    assert np.all(np.abs(gd - od) <= REL * dscale), fname
    t.destroy()


@pytest.mark.parametrize("sigma", [0.3, 0.8])
def test_dct_gaussian_discrete_mean_staged(dev, sigma):
    """The discrete Gaussian mean (normalised 4x4 window) of a DCT texture over
    a frame in pixel order: every block decodes its taps' box once into LDS;
    shuffled, no block stages; both give the same bits and meet the oracle's
    bar (1e-6 of sum |w| A over the window; the weights are positive)."""
    sigma = float(np.float32(sigma))
    W, H, C = 96, 80, 9
    tex = _texture(H, W, C, seed=W + 13)
    words = stf.stf_dct_encode(tex)
    t = stf.stf_create_dct_texture2d(W, H, C, words)
    fw, fh = 4 * W, 4 * H
    ys, xs = np.mgrid[0:fh, 0:fw]
    uv = np.stack([(xs + 0.29) / fw, (ys + 0.53) / fh], axis=-1).reshape(-1, 2).astype(np.float32)
    perm = np.random.default_rng(14).permutation(uv.shape[0])
    n = uv.shape[0]
    res = {}

    def run(key, u):
        o = torch.empty((n, C), dtype=torch.float32, device=dev)
        stf.stf_filter_gaussian(t, torch.from_numpy(u).to(dev), sigma, stf.STF_GAUSS_DISCRETE_MEAN, 0, o)
        res[key] = o

    staged, blocks = _staged(lambda: run("f", uv))
    assert staged == blocks == n // 256, (staged, blocks)
    staged, blocks = _staged(lambda: run("s", uv[perm]))
    assert staged == 0 and blocks == n // 256, (staged, blocks)
    back = torch.empty_like(res["s"])
    back[torch.from_numpy(perm).to(dev)] = res["s"]
    assert torch.equal(res["f"], back)
    gd = res["f"].cpu().numpy().astype(np.float64)
    od, _ = oracle.dct_gauss_filter2d(words, uv, sigma, oracle.G_DISCRETE_MEAN)
    A = _abs_terms(words).astype(np.float32)
    dscale, _ = oracle.gauss_filter2d(A, oracle.F32, uv, sigma, oracle.G_DISCRETE_MEAN)
    assert np.all(np.abs(gd - od) <= REL * dscale + 1e-12)
    t.destroy()
