"""Pins of the oracle's DCT-compressed textures (section "Results", texture
compression: 8x8 blocks, six lowest-frequency DCT coefficients per channel
in 32 bits, 7-bit DC and 5-bit AC).

What fixes the answers: scipy's orthonormal DCT-II and its inverse, the
documented bit layout, closed forms for constant blocks, and the 2D filter
machinery already pinned on dense textures (same taps, decoded texels)."""
import numpy as np
import pytest
from scipy import fft

import oracle

ZZ = [(0, 0), (0, 1), (1, 0), (2, 0), (1, 1), (0, 2)]   # (v, u): vertical, horizontal frequency


def test_coefficients_are_scipy_orthonormal_dct():
    rng = np.random.default_rng(1)
    for _ in range(5):
        f = rng.random((8, 8))
        ref = fft.dctn(f, type=2, norm="ortho")        # ref[v, u]
        for v in range(8):
            for u in range(8):
                assert abs(oracle.dct_coefficient(f, u, v) - ref[v, u]) < 1e-13


def test_bit_layout_and_dequantisation():
    word = 100 | (20 << 7) | (5 << 12) | (16 << 17) | (31 << 22) | (1 << 27)
    got = [oracle.dct_dequant(word, k) for k in range(6)]
    ref = [100 * 8 / 127, 4 * 2 / 15, -11 * 2 / 15, 0.0, 15 * 2 / 15, -15 * 2 / 15]
    assert np.allclose(got, ref, rtol=0, atol=1e-15)


def test_encoder_picks_the_nearest_code():
    """Each code is the nearest quantisation level of the exact coefficient
    (scipy), saturated at the range ends."""
    rng = np.random.default_rng(2)
    tex = rng.integers(0, 256, (16, 24, 3), dtype=np.uint8)
    tex[:8, :8] = 255                         # a saturated-DC block
    tex[8:, 8:16, 0] = (np.arange(8) % 2 * 255)[None, :]   # high-contrast stripes (AC saturation)
    words = oracle.dct_encode(tex)
    assert words.shape == (2, 3, 3)
    for by in range(2):
        for bx in range(3):
            for c in range(3):
                F = fft.dctn(tex[by * 8:by * 8 + 8, bx * 8:bx * 8 + 8, c] / 255.0, type=2, norm="ortho")
                w = int(words[by, bx, c])
                for k, (v, u) in enumerate(ZZ):
                    deq = oracle.dct_dequant(w, k)
                    if k == 0:
                        step, lo, hi = 8 / 127, 0.0, 8.0
                    else:
                        step, lo, hi = 2 / 15, -2.0, 2.0
                    target = min(max(F[v, u], lo), hi)
                    assert abs(deq - target) <= step / 2 + 1e-12, (by, bx, c, k, F[v, u], deq)


def test_decoder_is_scipy_inverse_dct_of_kept_coefficients():
    rng = np.random.default_rng(3)
    tex = rng.integers(0, 256, (8, 16, 2), dtype=np.uint8)
    words = oracle.dct_encode(tex)
    dec = oracle.dct_decode_all(words)
    for bx in range(2):
        for c in range(2):
            F = np.zeros((8, 8))
            for k, (v, u) in enumerate(ZZ):
                F[v, u] = oracle.dct_dequant(int(words[0, bx, c]), k)
            ref = fft.idctn(F, type=2, norm="ortho")
            assert np.allclose(dec[:, bx * 8:bx * 8 + 8, c], ref, rtol=0, atol=1e-13)


def test_constant_block_decodes_to_nearest_1_over_127():
    for v in (0, 1, 37, 128, 254, 255):
        tex = np.full((8, 8, 1), v, np.uint8)
        words = oracle.dct_encode(tex)
        assert (int(words[0, 0, 0]) >> 7) == sum(16 << (5 * k) for k in range(5))   # five zero AC codes
        dec = oracle.dct_decode_all(words)
        assert np.allclose(dec, round(v * 127 / 255) / 127, rtol=0, atol=1e-14)


@pytest.mark.parametrize("filt", [oracle.LINEAR, oracle.CUBIC, oracle.KEYS, oracle.MITCHELL])
def test_filters_read_decoded_texels(filt):
    """Deterministic: sum of weights times decoded texels (brute force with
    scipy-decoded texels); stochastic: the dense texture's taps for the same
    queries and seed, valued at the decoded texels."""
    rng = np.random.default_rng(4)
    tex = rng.integers(0, 256, (16, 24, 3), dtype=np.uint8)
    words = oracle.dct_encode(tex)
    dec = np.zeros((16, 24, 3))
    for by in range(2):
        for bx in range(3):
            for c in range(3):
                F = np.zeros((8, 8))
                for k, (v, u) in enumerate(ZZ):
                    F[v, u] = oracle.dct_dequant(int(words[by, bx, c]), k)
                dec[by * 8:by * 8 + 8, bx * 8:bx * 8 + 8, c] = fft.idctn(F, type=2, norm="ortho")
    uv = (rng.random((400, 2)) * 1.2 - 0.1).astype(np.float32)
    det, _ = oracle.dct_filter2d(words, uv, filt, oracle.DET)
    x = uv[:, 0] * np.float32(24) - np.float32(0.5)
    y = uv[:, 1] * np.float32(16) - np.float32(0.5)
    for q in range(400):
        ix, iy = int(np.floor(x[q])), int(np.floor(y[q]))
        wx = oracle.axis_weights(filt, float(x[q]) - ix)
        wy = oracle.axis_weights(filt, float(y[q]) - iy)
        base, nt = (0, 2) if filt == oracle.LINEAR else (-1, 4)
        ref = np.zeros(3)
        for b in range(nt):
            for a in range(nt):
                ref += wx[a] * wy[b] * dec[np.clip(iy + base + b, 0, 15), np.clip(ix + base + a, 0, 23)]
        assert np.allclose(det[q], ref, rtol=0, atol=1e-12)
    sv, si = oracle.dct_filter2d(words, uv, filt, oracle.STOCH, seed=5)
    dv, di = oracle.filter2d(tex, oracle.U8, uv, filt, oracle.STOCH, seed=5)
    assert np.array_equal(si, di)
    if filt in oracle.POSITIVIZED:
        for q in range(400):
            t = [float(x[q]) - float(np.floor(x[q])), float(y[q]) - float(np.floor(y[q]))]   # exact offsets
            sp, sn = oracle.positivized_masses(filt, t)
            ref = sp * dec[si[q, 1], si[q, 0]]
            if si[q, 2] != oracle.BAD_INDEX:
                ref = ref - sn * dec[si[q, 3], si[q, 2]]
            assert np.allclose(sv[q], ref, rtol=0, atol=1e-12)
    else:
        assert np.allclose(sv, dec[si[:, 1], si[:, 0]], rtol=0, atol=1e-13)
    mean, var = oracle.dct_moments2d(words, uv, filt)
    assert np.allclose(mean, det, rtol=0, atol=1e-12) and np.all(var > -1e-12)


def test_argument_checks():
    with pytest.raises(ValueError):
        oracle.dct_encode(np.zeros((12, 8, 1), np.uint8))   # height not a multiple of 8
    with pytest.raises(ValueError):
        oracle.dct_encode(np.zeros((8, 8, 17), np.uint8))   # more than 16 channels
