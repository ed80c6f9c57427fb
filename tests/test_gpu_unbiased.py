"""The unbiasedness run on the full 512^3 fBm grid (the benchmark's grid):
Q = 4,096 queries near active voxels, K = 65,536 seeds each, first and
second moments accumulated in binary64 on the device; every query's mean
must lie within 5 sigma of the oracle's exact filtered value (sigma from the
oracle's exact variance), for the single-tap filters and the positivized
interpolating cubics (Eqs. filtered-texture and stochastic-sum; the expected
number of false alarms over all queries is 4,096 x 5.7e-7 = 0.002 per
filter).  Per-axis tap frequencies of the single-tap filters are tested
against the per-axis weights with a chi-square test."""
import numpy as np
import pytest
import torch
from scipy import stats

import oracle
import paper_2305_05810_amd as stf
import synth

pytestmark = pytest.mark.gpu

DIMS = (512, 512, 512)
Q, K = 4096, 65536


@pytest.fixture(scope="module")
def setup():
    g = synth.fbm_grid(DIMS, seed=3)
    rng = np.random.default_rng(31)
    leaf, vz, vy, vx = np.nonzero(g.values > 0)
    pick = rng.integers(0, leaf.size, Q)
    vox = g.origins[leaf[pick]] + np.stack([vx[pick], vy[pick], vz[pick]], axis=1)
    p = (vox + rng.random((Q, 3)) * 2.0 - 1.0).astype(np.float32)
    return g, p


@pytest.mark.parametrize("gf,of", [(stf.STF_CUBIC_BSPLINE, oracle.CUBIC), (stf.STF_LINEAR, oracle.LINEAR),
                                   (stf.STF_CUBIC_KEYS, oracle.KEYS), (stf.STF_CUBIC_MITCHELL, oracle.MITCHELL)])
def test_unbiasedness_run(dev, setup, gf, of):
    g, p = setup
    t = stf.stf_create_sparse_grid3d(DIMS, stf.STF_FMT_F32, g.origins, g.values)
    og = oracle.Grid(DIMS, oracle.F32, g.origins, g.values)
    q = torch.from_numpy(p).to(dev)
    s1 = torch.empty(Q, dtype=torch.float64, device=dev)
    s2 = torch.empty_like(s1)
    stf.stf_filter_moments(t, q, gf, 0x51EED, K, s1, s2)
    s1, s2 = s1.cpu().numpy(), s2.cpu().numpy()
    mean, var = og.moments(p, of)
    live = var > 1e-14
    assert live.sum() > 0.9 * Q
    z = (s1 / K - mean)[live] / np.sqrt(var[live] / K)
    print(f"filter {gf}: max |z| {np.abs(z).max():.2f} over {live.sum()} queries")
    assert np.all(np.abs(z) < 5.0), np.abs(z).max()
    v_hat = s2 / K - (s1 / K) ** 2
    assert 0.97 < v_hat[live].sum() / var[live].sum() < 1.03
    t.destroy()


@pytest.mark.parametrize("gf,of", [(stf.STF_CUBIC_BSPLINE, oracle.CUBIC), (stf.STF_LINEAR, oracle.LINEAR)])
def test_per_axis_tap_frequencies(dev, setup, gf, of):
    g, p = setup
    t = stf.stf_create_sparse_grid3d(DIMS, stf.STF_FMT_F32, g.origins, g.values)
    n = 1 << 16
    out = torch.empty((n, 1), dtype=torch.float32, device=dev)
    idx = torch.empty((n, 3), dtype=torch.int32, device=dev)
    pvals = []
    for k in range(8):
        pq = p[k]
        q = torch.from_numpy(np.repeat(pq[None], n, axis=0)).to(dev)
        stf.stf_filter(t, q, gf, stf.STF_STOCHASTIC, 1000 + k, out, idx)
        ix = idx.cpu().numpy()
        for a in range(3):
            c = int(np.floor(pq[a]))
            tt = float(pq[a]) - c
            w = oracle.axis_weights(of, tt)
            lo = c - 1 if of == oracle.CUBIC else c
            cnt = np.bincount(ix[:, a] - lo, minlength=4)[:4]
            live = w > 0
            assert np.all(cnt[~live] == 0)
            pvals.append(stats.chisquare(cnt[live], w[live] / w[live].sum() * n).pvalue)
    assert min(pvals) > 1e-4 / len(pvals), min(pvals)   # Bonferroni over the 24 tests
    t.destroy()
