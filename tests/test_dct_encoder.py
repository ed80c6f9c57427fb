"""The library's host-side DCT encoder against the oracle's (both binary64,
different summation orders): every code is equal, except where the exact
coefficient lies within 1e-9 of a rounding boundary, where either
neighbouring code is correct.  No GPU is needed."""
import numpy as np
import pytest
from scipy import fft

import oracle
import paper_2305_05810_amd as stf

ZZ = [(0, 0), (0, 1), (1, 0), (2, 0), (1, 1), (0, 2)]


def _field(word, k):
    return (word & 127) if k == 0 else ((word >> (7 + 5 * (k - 1))) & 31)


def test_library_encoder_matches_oracle():
    rng = np.random.default_rng(7)
    tex = rng.integers(0, 256, (64, 48, 9), dtype=np.uint8)
    tex[:8, :8] = 255
    tex[8:16, :8, 0] = (np.arange(8) % 2 * 255)[None, :]
    tex[16:24, 8:16] = 128                       # DC exactly on a rounding boundary region
    lib_words = stf.stf_dct_encode(tex)
    orc_words = oracle.dct_encode(tex)
    assert lib_words.shape == orc_words.shape == (8, 6, 9)
    diff = np.argwhere(lib_words != orc_words)
    for by, bx, c in diff:
        F = fft.dctn(tex[by * 8:by * 8 + 8, bx * 8:bx * 8 + 8, c] / 255.0, type=2, norm="ortho")
        for k, (v, u) in enumerate(ZZ):
            a, b = _field(int(lib_words[by, bx, c]), k), _field(int(orc_words[by, bx, c]), k)
            if a != b:
                scaled = F[v, u] * (127 / 8 if k == 0 else 15 / 2)
                assert abs(abs(scaled - np.floor(scaled)) - 0.5) < 1e-9 and abs(a - b) == 1
    assert diff.shape[0] <= 2


def test_encoder_argument_errors():
    with pytest.raises(stf.STFError):
        stf.stf_dct_encode(np.zeros((12, 8, 1), np.uint8))
    with pytest.raises(stf.STFError):
        stf.stf_dct_encode(np.zeros((8, 8, 17), np.uint8))
