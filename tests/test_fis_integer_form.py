"""The identity behind the device's filter-importance-sampling tap (no GPU
needed).  The tap is floor((x + s) + 1/2) in binary64 with x binary32 and s
= K 2^-24 - 3/2 (cubic: K the sum of three 24-bit uniform integers) or
K 2^-24 - 1/2 (tent: K one uniform integer).  For |x| >= 2^-29 the device
forms it as floor(x) - c + floor((R + K) / 2^24), c = 1 (cubic) or 0 (tent),
with R = floor(x 2^24) - floor(x) 2^24 -- all of it exact in binary32 and
integers.  This checks that the two agree on random binary32 x of every
magnitude up to 2^24, on x next to integers and next to 2^-29, and on the K
where (R + K) / 2^24 lands on or beside an integer."""
import numpy as np
import pytest


def _binary64_tap(x, K, cubic):
    s = K.astype(np.float64) * 2.0 ** -24 - (1.5 if cubic else 0.5)
    return np.floor((x.astype(np.float64) + s) + 0.5).astype(np.int64)


def _integer_tap(x, K, cubic):
    yi = np.floor(x * np.float32(2 ** 24))          # binary32, exact (a power-of-two scaling)
    h = np.floor(x)
    r = (yi.astype(np.float64) - h.astype(np.float64) * 2.0 ** 24).astype(np.int64)   # the fused multiply-add: exact
    assert np.all((r >= 0) & (r < 2 ** 24))
    return h.astype(np.int64) - (1 if cubic else 0) + ((r + K.astype(np.int64)) >> 24)


def _xs(rng, n):
    mag = np.float32(2.0) ** rng.uniform(-29, 24, n).astype(np.float32)
    x = (mag * rng.choice([-1, 1], n)).astype(np.float32)
    ints = rng.integers(-2 ** 23, 2 ** 23, n // 4).astype(np.float32)
    near = np.concatenate([ints, np.nextafter(ints, np.float32(np.inf)), np.nextafter(ints, np.float32(-np.inf))])
    edge = np.array([2.0 ** -29, -2.0 ** -29, 2.0 ** -29 * (1 + 2.0 ** -23), -2.0 ** -29 * (1 + 2.0 ** -23),
                     0.5, -0.5, 1.0, -1.0, 2.0 ** 24 - 1, -(2.0 ** 24 - 1)], np.float32)
    x = np.concatenate([x, near, edge]).astype(np.float32)
    return x[np.abs(x) >= np.float32(2.0 ** -29)]


@pytest.mark.parametrize("cubic", [True, False])
def test_integer_form_equals_binary64_tap(cubic):
    rng = np.random.default_rng(7)
    x = _xs(rng, 400_000)
    kmax = 3 * (2 ** 24 - 1) if cubic else 2 ** 24 - 1
    K = rng.integers(0, kmax + 1, x.size).astype(np.int64)
    assert np.array_equal(_binary64_tap(x, K, cubic), _integer_tap(x, K, cubic))
    # K that put (R + K) / 2^24 on, just below and just above an integer
    yi = np.floor(x * np.float32(2 ** 24)).astype(np.float64)
    R = (yi - np.floor(x).astype(np.float64) * 2.0 ** 24).astype(np.int64)
    for m in (1, 2) if cubic else (1,):
        for d in (-1, 0, 1):
            Kb = m * 2 ** 24 - R + d
            ok = (Kb >= 0) & (Kb <= kmax)
            assert np.array_equal(_binary64_tap(x[ok], Kb[ok], cubic), _integer_tap(x[ok], Kb[ok], cubic))


def test_binary64_sum_rounds_below_the_bound():
    # Below 2^-29 the binary64 sum can round x away, so the device evaluates
    # it as written there: x = -2^-60 with s + 1/2 = 1 gives floor(1) = 1 in
    # binary64, while the exact value 1 - 2^-60 has floor 0.
    x = np.array([-2.0 ** -60], np.float32)
    K = np.array([2 * 2 ** 24], np.int64)   # cubic: s + 1/2 = K 2^-24 - 1 = 1
    assert _binary64_tap(x, K, True)[0] == 1
    assert _integer_tap(x, K, True)[0] == 0   # the exact floor: the two forms part below 2^-29
