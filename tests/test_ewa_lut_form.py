"""The identities behind the device's EWA weight (no GPU needed).  The
device keeps 128 A, 128 B and 128 C, so each tap forms 128 r2 directly, and
reads a 129-entry table whose last entry is +0 at index
trunc(max(min(128 r2, 128), 0)), in place of LUT[min(floor(128 r2), 127)]
for r2 < 1 and 0 otherwise.  This checks on the host, in binary32 with each
operation rounded as on the device, that (1) the scaled quadratic form is
exactly 128 times the unscaled one for the coefficients and offsets of
scanned levels, and (2) the two weight rules agree bit for bit, NaN and
negative rounding residues included."""
import math

import numpy as np

F = np.float32


def _lut128():
    return np.array([F(math.exp(-2.0 * i / 127.0) - math.exp(-2.0)) for i in range(128)], np.float32)


def _r2(A, B, C, ss, tt):
    return (A * (ss * ss) + (B * ss) * tt) + C * (tt * tt)   # numpy float32: every operation rounded once


def test_scaled_form_is_exact():
    rng = np.random.default_rng(3)
    n = 200_000
    # coefficients of scanned levels: |A|, |C| <= 1, |B| <= 1 (A = (a + 1) / F and
    # the like with F >= a + c + 1), down to 1 / (1 + 128^2 + ...) for the longest axes
    A = (10.0 ** rng.uniform(-5, 0, n)).astype(np.float32)
    C = (10.0 ** rng.uniform(-5, 0, n)).astype(np.float32)
    B = (rng.uniform(-1, 1, n) * 2.0 * np.sqrt(A.astype(np.float64) * C)).astype(np.float32)
    # centres of every magnitude (fine fractional offsets near 0, whole ones near 2^23)
    stx = (rng.choice([-1.0, 1.0], n) * 2.0 ** rng.uniform(-2, 23, n)).astype(np.float32)
    sty = (rng.choice([-1.0, 1.0], n) * 2.0 ** rng.uniform(-2, 23, n)).astype(np.float32)
    ds, dt = rng.integers(-300, 300, n), rng.integers(-300, 300, n)
    ss = (np.floor(stx).astype(np.float64) + ds).astype(np.float32) - stx
    tt = (np.floor(sty).astype(np.float64) + dt).astype(np.float32) - sty
    r2 = _r2(A, B, C, ss, tt)
    r2s = _r2(A * F(128), B * F(128), C * F(128), ss, tt)
    assert np.array_equal(r2s.view(np.uint32), (r2 * F(128)).view(np.uint32))


def test_weight_rules_agree():
    lut = _lut128()
    lut129 = np.append(lut, F(0.0))
    rng = np.random.default_rng(4)
    r2 = np.concatenate([rng.uniform(-0.02, 1.5, 1_000_000).astype(np.float32),
                         np.arange(0, 129, dtype=np.float32) / F(128),                       # exact LUT boundaries
                         np.nextafter(np.arange(1, 130, dtype=np.float32) / F(128), F(0)),  # just below them
                         np.array([np.nan, -0.0, -1e-30, -1.0 / 128, np.inf, 1e30], np.float32)])
    with np.errstate(invalid="ignore"):
        old = np.where(r2 < F(1), lut[np.clip(np.nan_to_num(r2 * F(128), nan=0.0).astype(np.int64), 0, 127)], F(0))
        r2s = r2 * F(128)
        new = lut129[np.fmax(np.fmin(r2s, F(128)), F(0)).astype(np.int64)]
    assert np.array_equal(old.view(np.uint32), new.view(np.uint32))
