"""Host checks of the input generators that are more than a draw from a
distribution (no GPU)."""
import numpy as np

import synth


def test_medium_ray_queries_are_the_ray_samples_that_meet_a_leaf():
    g = synth.fbm_grid((64, 64, 64), base_period=16.0, seed=7)
    n = 3000
    m = synth.medium_ray_queries(g, n, seed=11, samples_per_ray=64)
    assert m.shape == (n, 3) and m.dtype == np.float32
    leaves = {tuple(o) for o in (g.origins // 8).tolist()}

    def meets(p):
        c = np.floor(p).astype(int) - 1
        return any((x >> 3, y >> 3, z >> 3) in leaves
                   for x in range(c[0], c[0] + 4) for y in range(c[1], c[1] + 4) for z in range(c[2], c[2] + 4))

    assert all(meets(p) for p in m[:400])
    # the kept samples are, in order, exactly the meeting samples of the ray batches
    first = synth.ray_queries(g.dims, 65536, 64, 11)
    mask = np.array([meets(p) for p in first[:20000]])
    expect = first[:20000][mask]
    k = min(expect.shape[0], n)
    assert k > 100 and np.array_equal(m[:k], expect[:k])
