"""Error bounds of the hardware transcendental instructions behind binary32
decisions that fall back to binary64 within a margin (the Gaussian filter
importance sampling radius and angle, the discrete Gaussian weights, the EWA
level draw).  The kernels' margins are derived from these bounds; the
program measures each bound exhaustively over the inputs the kernels can
give (every 24-bit uniform, every binary32 exponent argument in [-64, 0],
every binary32 in [2^-32, 2^32]) against binary64, so a device whose
instructions differ fails here rather than silently in a rare tap."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(__file__), "hw", "transcendental_bounds")

# bound each kernel comment states -> what the margin needs
BOUNDS = {
    "box_muller_radius_abs": 4.9e-7,   # Gaussian FIS: offset within 2e-6 sigma, margin sigma 2^-14
    "sin_turns_abs": 1.3e-7,
    "cos_turns_abs": 1.3e-7,
    "exp2_rel_neg64_0": 8.5e-8,        # discrete Gaussian: weights within 2e-5 relative, margin total 2^-12
    "log2_abs_2m32_2p32": 4.0e-6,      # EWA level: lod within 1e-5 (with the sum's rounding), margin 1e-4
}


def test_transcendental_bounds():
    if not os.path.exists(BIN):
        pytest.fail(f"{BIN} is not built: run __graft_entry__.build()")
    print("running", BIN, flush=True)
    r = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    got = {}
    for line in r.stdout.splitlines():
        name, value = line.split()
        got[name] = float(value)
    assert set(got) == set(BOUNDS), got
    print(" ".join(f"{k}={v:.3e}" for k, v in got.items()), flush=True)
    for name, bound in BOUNDS.items():
        assert 0.0 <= got[name] <= bound, (name, got[name], bound)
