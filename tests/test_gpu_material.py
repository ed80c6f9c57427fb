"""GPU parity of material textures filtered as six-channel 2D textures
(albedo RGB, roughness, normal x, y): the material is filtered before
shading (Eq. traditional-lighting-integral) with every filter and mode of
stf_filter and stf_filter_gaussian, through a sorted stream and through the
server, against the FP64 oracle reading the same 8-byte texels.

Bar: stochastic -- taps equal to the oracle's and values the decoded texel
exactly (both decodes are exact in binary32); deterministic and the Gaussian
means -- within 1e-6 of the oracle relative to sum |w| |t| over the taps."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_05810_amd as stf
import synth

pytestmark = pytest.mark.gpu

FILTERS = [("linear", stf.STF_LINEAR, oracle.LINEAR), ("bspline", stf.STF_CUBIC_BSPLINE, oracle.CUBIC),
           ("keys", stf.STF_CUBIC_KEYS, oracle.KEYS), ("mitchell", stf.STF_CUBIC_MITCHELL, oracle.MITCHELL)]
REL = 1e-6


def _abs_decoded(lv0):
    """|decoded channel| of every texel, (H, W, 6) binary32 (the tolerance scale)."""
    H, W = lv0.shape
    a = np.empty((H, W, 6), np.float32)
    a[..., 0:3] = lv0["albedo"] / np.float32(255.0)
    a[..., 3] = lv0["rough"] / np.float32(255.0)
    a[..., 4] = np.abs(lv0["nx"].astype(np.float32))
    a[..., 5] = np.abs(lv0["ny"].astype(np.float32))
    return a


@pytest.fixture(scope="module")
def material():
    lv = synth.material_levels(96, seed=51, levels=1)
    lv0 = np.ascontiguousarray(lv[0])
    raw = lv0.view(np.uint8).reshape(96, 96, 8)
    uv = synth.uv_queries(30000, seed=52) * np.float32(1.1) - np.float32(0.05)
    uv[:6] = [[np.nan, 0.5], [0.5, np.inf], [1e30, 0.5], [-0.7, 1.4], [0, 0], [1, 1]]
    mat = stf.stf_create_material2d(96, 96, [lv0])
    yield mat, lv0, raw, uv.astype(np.float32)
    mat.destroy()


def _check_det(gd, od, scale, label):
    gd = gd.astype(np.float64)
    err = np.abs(gd - od)
    ok = (np.isnan(gd) & np.isnan(od)) | (err <= REL * scale)
    worst = np.nanmax(np.where(scale > 0, err / np.where(scale > 0, scale, 1), 0))
    assert ok.all(), f"{label}: {np.sum(~ok)} outside (worst {worst:.3g})"


@pytest.mark.parametrize("fname,gf,of", FILTERS)
def test_material_filter_parity(dev, material, fname, gf, of):
    mat, lv0, raw, uv = material
    assert mat.channels == 6
    q = torch.from_numpy(uv).to(dev)
    gv, gi = stf.filter(mat, q, gf, stf.STF_STOCHASTIC, 0x3A7, want_index=True)
    ov, oi = oracle.material_filter2d(raw, uv, of, oracle.STOCH, 0x3A7)
    assert np.array_equal(gi.cpu().numpy(), oi), fname
    gv = gv.cpu().numpy()
    if of in oracle.POSITIVIZED:
        # S+ t+ - S- t-: binary32 arithmetic on exact texels; scale S+|t+| + S-|t-|
        A = _abs_decoded(lv0)
        x = uv[:, 0] * np.float32(96) - np.float32(0.5)
        y = uv[:, 1] * np.float32(96) - np.float32(0.5)
        scale = np.zeros_like(ov)
        for k in np.nonzero(oi[:, 0] != oracle.BAD_INDEX)[0]:
            sp, sn = oracle.positivized_masses(of, [float(x[k]) - float(np.floor(x[k])),
                                                    float(y[k]) - float(np.floor(y[k]))])
            scale[k] = sp * A[oi[k, 1], oi[k, 0]]
            if oi[k, 2] != oracle.BAD_INDEX:
                scale[k] += sn * A[oi[k, 3], oi[k, 2]]
        _check_det(gv, ov, scale, f"{fname} stoch")
    else:
        assert np.array_equal(np.nan_to_num(gv, nan=-7), np.nan_to_num(ov.astype(np.float32), nan=-7)), fname
    gd, _ = stf.filter(mat, q, gf, stf.STF_DETERMINISTIC, 0)
    od, _ = oracle.material_filter2d(raw, uv, of, oracle.DET)
    scale, _ = oracle.filter2d(_abs_decoded(lv0), oracle.F32, uv, of, oracle.DET_ABS)
    _check_det(gd.cpu().numpy(), od, scale, f"{fname} det")
    if gf in (stf.STF_LINEAR, stf.STF_CUBIC_BSPLINE):
        gv, gi = stf.filter(mat, q, gf, stf.STF_STOCHASTIC_FIS, 0x3A8, want_index=True)
        ov, oi = oracle.material_filter2d(raw, uv, of, oracle.STOCH_FIS, 0x3A8)
        assert np.array_equal(gi.cpu().numpy(), oi), fname
        assert np.array_equal(np.nan_to_num(gv.cpu().numpy(), nan=-7), np.nan_to_num(ov.astype(np.float32), nan=-7))


@pytest.mark.parametrize("fname,gf,of", FILTERS)
def test_material_sorted_stream(dev, material, fname, gf, of):
    """Morton-sorted queries: the same bits as the unsorted call."""
    mat, lv0, raw, uv = material
    q = torch.from_numpy(uv).to(dev)
    sq, order = stf.sort_queries(mat, q)
    for mode in (stf.STF_STOCHASTIC, stf.STF_DETERMINISTIC):
        ref, ridx = stf.filter(mat, q, gf, mode, 11, want_index=True)
        out = torch.empty_like(ref)
        idx = None if ridx is None else torch.empty_like(ridx)
        stf.stf_filter_ordered(mat, sq, order, gf, mode, 11, out, idx, stf.STF_ORDER_SCATTER)
        assert torch.equal(out.nan_to_num(-7), ref.nan_to_num(-7)), (fname, mode)
        if idx is not None:
            assert torch.equal(idx, ridx)


@pytest.mark.parametrize("sigma", [0.3, 1.5])
def test_material_gaussian(dev, material, sigma):
    mat, lv0, raw, uv = material
    sigma = float(np.float32(sigma))
    q = torch.from_numpy(uv).to(dev)
    n = uv.shape[0]
    out = torch.empty((n, 6), dtype=torch.float32, device=dev)
    idx = torch.empty((n, 2), dtype=torch.int32, device=dev)
    stf.stf_filter_gaussian(mat, q, sigma, stf.STF_GAUSS_DISCRETE, 93, out, idx)
    ov, oi = oracle.material_gauss_filter2d(raw, uv, sigma, oracle.G_DISCRETE, 93)
    assert np.array_equal(idx.cpu().numpy(), oi)
    assert np.array_equal(np.nan_to_num(out.cpu().numpy(), nan=-7), np.nan_to_num(ov.astype(np.float32), nan=-7))
    stf.stf_filter_gaussian(mat, q, sigma, stf.STF_GAUSS_DISCRETE_MEAN, 0, out)
    od, _ = oracle.material_gauss_filter2d(raw, uv, sigma, oracle.G_DISCRETE_MEAN)
    scale, _ = oracle.gauss_filter2d(_abs_decoded(lv0), oracle.F32, uv, sigma, oracle.G_DISCRETE_MEAN)
    _check_det(out.cpu().numpy(), od, scale, f"gauss mean {sigma}")


def test_material_served_with_other_textures(dev, material):
    """Material requests mixed with RGBA requests in one server: each result
    bit-identical to stf_filter alone."""
    mat, lv0, raw, uv = material
    tex = synth.texture2d(64, 48, 4, seed=53)
    t4 = stf.stf_create_texture2d(64, 48, 4, stf.STF_FMT_F16, [synth.encode(tex, "f16")])
    rng = np.random.default_rng(54)
    srv = stf.stf_server_create(8 << 20, 16, 2048)
    reqs, tickets = [], []
    for k in range(60):
        t = mat if k % 2 == 0 else t4
        n = int(rng.integers(100, 9000))
        qk = rng.random((n, 2), dtype=np.float32)
        filt = stf.STF_CUBIC_BSPLINE if rng.random() < 0.5 else stf.STF_LINEAR
        out = np.empty((n, t.channels), np.float32)
        idx = np.empty((n, 2), np.int32)
        seed = int(rng.integers(1 << 62))
        tickets.append(stf.stf_server_submit(srv, t, qk, filt, seed, out, idx))
        reqs.append((t, qk, filt, seed, out, idx))
    for tk in tickets:
        stf.stf_server_wait(srv, tk)
    for t, qk, filt, seed, out, idx in reqs:
        ref, ridx = stf.filter(t, torch.from_numpy(qk).to(dev), filt, stf.STF_STOCHASTIC, seed, want_index=True)
        assert np.array_equal(idx, ridx.cpu().numpy())
        assert np.array_equal(out, ref.cpu().numpy())
    srv.destroy()
    t4.destroy()
