"""GPU parity of filtering with shading (stf_shade_filter) against the FP64
oracle.  The sampled tap (x, y, level) must equal the oracle's for every
query.  Shaded values are binary32 GGX evaluations compared with binary64
ones; the bound is stated relative to the value (see SHADE_REL)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_05810_amd as stf
import synth

pytestmark = pytest.mark.gpu

# binary32 GGX against binary64: |gpu - oracle| <= SHADE_REL * |oracle| + SHADE_ABS.
# Near the specular peak the GGX lobe's log-derivative with respect to the
# half-vector angle is up to 2/alpha (alpha >= 1e-3), so the binary32 rounding
# of the half vector (a few 1e-8 rad) alone allows relative errors of order
# 1e-4; the worst case measured on these inputs is 1.5e-5 (shading with the
# hardware reciprocal, square root and reciprocal square root).
SHADE_REL = 1e-4
SHADE_ABS = 1e-6

MODES = [("after_filter", stf.STF_SHADE_AFTER_FILTER, oracle.SH_AFTER_FILTER),
         ("filter_after", stf.STF_FILTER_AFTER_SHADE, oracle.SH_FILTER_AFTER),
         ("stochastic", stf.STF_SHADE_STOCHASTIC, oracle.SH_STOCH)]
FILTERS = [("linear", stf.STF_LINEAR, oracle.LINEAR), ("cubic", stf.STF_CUBIC_BSPLINE, oracle.CUBIC)]


def _err_stats(g, o):
    err = np.abs(g - o)
    rel = err / np.maximum(np.abs(o), 1e-30)
    big = np.abs(o) > 1e-3
    return dict(max_abs=float(err.max()), max_rel_big=float(rel[big].max()) if big.any() else 0.0,
                p9999_rel_big=float(np.percentile(rel[big], 99.99)) if big.any() else 0.0)


def _check(g, o, label):
    both_nan = np.isnan(g) & np.isnan(o)
    ok = both_nan | (np.abs(g - o) <= SHADE_REL * np.abs(o) + SHADE_ABS)
    print(label, _err_stats(np.nan_to_num(g), np.nan_to_num(o)))
    assert ok.all(), f"{label}: {np.sum(~ok)} values outside the bound"


@pytest.fixture(scope="module")
def small_material():
    lv = synth.material_levels(256, seed=31, levels=3)
    recs = synth.shade_queries(100000, seed=32)
    recs[:8, 0:2] = [[0, 0], [1 - 2 ** -24, 1 - 2 ** -24], [0.5, 0.5], [np.nan, 0.3], [0.2, np.inf],
                     [-0.3, 1.7], [0.25, 0.75], [0.9, 0.1]]
    recs[8:12, 2] = [1.41421354, 1.4142134, 2.82842708, 2.828427]   # level thresholds
    return lv, recs


@pytest.mark.parametrize("mname,gm,om", MODES)
@pytest.mark.parametrize("fname,gf,of", FILTERS)
def test_shade_parity(dev, small_material, mname, gm, om, fname, gf, of):
    lv, recs = small_material
    mat = stf.stf_create_material2d(lv[0].shape[1], lv[0].shape[0], lv)
    om_ = oracle.Material(lv)
    q = torch.from_numpy(recs).to(dev)
    n = recs.shape[0]
    out = torch.empty((n, 3), dtype=torch.float32, device=dev)
    idx = torch.empty((n, 3), dtype=torch.int32, device=dev) if gm == stf.STF_SHADE_STOCHASTIC else None
    seed = 77
    stf.stf_shade_filter(mat, q, gf, gm, seed, out, idx)
    ov, oi = om_.shade(recs, of, om, seed)
    if idx is not None:
        assert np.array_equal(idx.cpu().numpy(), oi)
    _check(out.cpu().numpy().astype(np.float64), ov, f"shade {mname} {fname}")
    mat.destroy()


def test_shade_full_size_sampled(dev):
    lv = synth.material_levels(4096, seed=21, levels=3)
    recs = synth.shade_queries(1 << 23, seed=22)
    mat = stf.stf_create_material2d(4096, 4096, lv)
    om_ = oracle.Material(lv)
    q = torch.from_numpy(recs).to(dev)
    n = recs.shape[0]
    rng = np.random.default_rng(3)
    qids = np.sort(rng.choice(n, 1 << 15, replace=False))
    out = torch.empty((n, 3), dtype=torch.float32, device=dev)
    idx = torch.empty((n, 3), dtype=torch.int32, device=dev)
    for mname, gm, om in MODES:
        stf.stf_shade_filter(mat, q, stf.STF_CUBIC_BSPLINE, gm, 5, out, idx if gm == stf.STF_SHADE_STOCHASTIC else None)
        g = out.cpu().numpy()[qids].astype(np.float64)
        ov, oi = om_.shade_at(recs, qids, oracle.CUBIC, om, 5)
        if gm == stf.STF_SHADE_STOCHASTIC:
            assert np.array_equal(idx.cpu().numpy()[qids], oi)
        _check(g, ov, f"full {mname}")
    mat.destroy()


def test_shade_material_errors(dev):
    with pytest.raises(stf.STFError):
        stf.stf_create_material2d(0, 4, [np.zeros(0, np.uint8)])
    lv = synth.material_levels(16, seed=1, levels=1)
    mat = stf.stf_create_material2d(16, 16, lv)
    q = torch.zeros((4, 9), dtype=torch.float32, device=dev)
    out = torch.empty((4, 3), dtype=torch.float32, device=dev)
    idx = torch.empty((4, 3), dtype=torch.int32, device=dev)
    with pytest.raises(stf.STFError):
        stf.stf_shade_filter(mat, q, stf.STF_CUBIC_BSPLINE, stf.STF_FILTER_AFTER_SHADE, 0, out, idx)
    with pytest.raises(stf.STFError):
        stf.stf_shade_filter(mat, q, stf.STF_CUBIC_BSPLINE, 7, 0, out)
    g = synth.fbm_grid((16, 16, 16), base_period=8.0, seed=1)
    grid = stf.stf_create_sparse_grid3d(g.dims, stf.STF_FMT_F32, g.origins, g.values)
    with pytest.raises(stf.STFError):
        stf.stf_shade_filter(grid, q, stf.STF_CUBIC_BSPLINE, stf.STF_SHADE_STOCHASTIC, 0, out)
    grid.destroy()
    mat.destroy()


@pytest.mark.parametrize("W,H", [(37, 29), (5, 3), (1, 1)], ids=["37x29", "5x3", "1x1"])
def test_shade_ragged_material(dev, W, H):
    # level sizes that are not multiples of the 4x4 storage tile (padded on
    # the device): every tap, including clamped ones at the ragged edges, reads
    # the texel the oracle reads from the row-major levels
    big = synth.material_levels(64, seed=33, levels=3)
    lv = [np.ascontiguousarray(big[l][:max(H >> l, 1), :max(W >> l, 1)]) for l in range(3)]
    mat = stf.stf_create_material2d(W, H, lv)
    om_ = oracle.Material(lv)
    recs = synth.shade_queries(20000, seed=34)
    recs[:, 0:2] = recs[:, 0:2] * np.float32(1.2) - np.float32(0.1)
    q = torch.from_numpy(recs).to(dev)
    n = recs.shape[0]
    for gm, om in ((stf.STF_SHADE_STOCHASTIC, oracle.SH_STOCH), (stf.STF_SHADE_AFTER_FILTER, oracle.SH_AFTER_FILTER),
                   (stf.STF_FILTER_AFTER_SHADE, oracle.SH_FILTER_AFTER)):
        out = torch.empty((n, 3), dtype=torch.float32, device=dev)
        idx = torch.empty((n, 3), dtype=torch.int32, device=dev) if gm == stf.STF_SHADE_STOCHASTIC else None
        stf.stf_shade_filter(mat, q, stf.STF_CUBIC_BSPLINE, gm, 5, out, idx)
        ov, oi = om_.shade(recs, oracle.CUBIC, om, 5)
        if idx is not None:
            assert np.array_equal(idx.cpu().numpy(), oi)
        _check(out.cpu().numpy().astype(np.float64), ov, f"ragged {W}x{H} mode {gm}")
    # the same level through the 2D filters (six channels)
    raw = lv[0].view(np.uint8).reshape(H, W, 8)
    uv = (synth.uv_queries(20000, seed=35) * np.float32(1.2) - np.float32(0.1)).astype(np.float32)
    gv, gi = stf.filter(mat, torch.from_numpy(uv).to(dev), stf.STF_CUBIC_BSPLINE, stf.STF_STOCHASTIC, 6,
                        want_index=True)
    ov, oi = oracle.material_filter2d(raw, uv, oracle.CUBIC, oracle.STOCH, 6)
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(np.nan_to_num(gv.cpu().numpy(), nan=-7), np.nan_to_num(ov.astype(np.float32), nan=-7))
    mat.destroy()
