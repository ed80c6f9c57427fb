"""Pins of the oracle's filter kernels and per-axis weights against facts that
do not come from the oracle itself: hand-evaluated points of Eq.
cubic-bspline, the B-spline's construction as four convolved boxes, its
moments (integral 1, variance 1/3), and the polynomial identities that follow
from them (partition of unity, affine reproduction, second moment)."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_points():
    rows = []
    for line in open(os.path.join(GOLDEN, "bspline_kernel_points.txt")):
        if line.startswith("#") or not line.strip():
            continue
        a, b, c, d = map(int, line.split())
        rows.append((Fraction(a, b), Fraction(c, d)))
    return rows


@pytest.mark.parametrize("d,k", _golden_points())
def test_bspline_hand_evaluated_points(d, k):
    # Eq. cubic-bspline evaluated by hand at rational distances
    assert oracle.kernel_bspline(float(d)) == pytest.approx(float(k), abs=1e-16, rel=1e-15)


def test_bspline_is_four_convolved_boxes():
    # The cubic B-spline is the 4-fold convolution of the unit box (the
    # Cox-de Boor recursion that section "Filter Importance Sampling" uses).
    h = 1.0 / 2000.0
    box = np.ones(2000) * h                        # unit box sampled on [-1/2, 1/2)
    k = box.copy()
    for _ in range(3):
        k = np.convolve(k, box)
    # k[j] approximates the density at x = -2 + (j + 2) h (support [-2, 2])
    x = -2.0 + (np.arange(k.size) + 2.0) * h
    ref = k / h
    got = np.array([oracle.kernel_bspline(v) for v in x[::97]])
    assert np.max(np.abs(got - ref[::97])) < 5e-3


def test_bspline_moments():
    # integral 1 and variance 4 * (1/12) = 1/3 (sum of four uniform variables)
    x = np.linspace(-2.5, 2.5, 200001)
    k = np.array([oracle.kernel_bspline(v) for v in x])
    dx = x[1] - x[0]
    assert np.trapezoid(k, dx=dx) == pytest.approx(1.0, abs=1e-9)
    assert np.trapezoid(k * x * x, dx=dx) == pytest.approx(1.0 / 3.0, abs=1e-8)
    assert np.trapezoid(k * x, dx=dx) == pytest.approx(0.0, abs=1e-12)


def test_tent_kernel():
    # K_1 of the supplement: 1 - |t| on |t| < 1; integral 1, variance 1/6
    assert oracle.kernel_tent(0.0) == 1.0
    assert oracle.kernel_tent(0.25) == 0.75
    assert oracle.kernel_tent(-0.5) == 0.5
    assert oracle.kernel_tent(1.0) == 0.0
    x = np.linspace(-1.5, 1.5, 60001)
    k = np.array([oracle.kernel_tent(v) for v in x])
    dx = x[1] - x[0]
    assert np.trapezoid(k, dx=dx) == pytest.approx(1.0, abs=1e-8)
    assert np.trapezoid(k * x * x, dx=dx) == pytest.approx(1.0 / 6.0, abs=1e-7)


T_GRID = [0.0, 2.0 ** -24, 0.1, 0.25, 0.3, 0.5, 0.7, 0.9, 1.0 - 2.0 ** -24]


@pytest.mark.parametrize("t", T_GRID)
def test_cubic_axis_weights_are_the_kernel(t):
    # weights of taps i-1..i+2 are K_bs at distances t+1, t, 1-t, 2-t
    w = oracle.axis_weights(oracle.CUBIC, t)
    ref = [oracle.kernel_bspline(t + 1.0), oracle.kernel_bspline(t), oracle.kernel_bspline(1.0 - t),
           oracle.kernel_bspline(2.0 - t)]
    assert np.allclose(w, ref, rtol=1e-12, atol=1e-17)


@pytest.mark.parametrize("t", T_GRID)
def test_cubic_weight_identities(t):
    # partition of unity, affine reproduction sum w_k (k-1) = t, and second
    # moment sum w_k (k-1)^2 = t^2 + 1/3 (the kernel's variance)
    w = oracle.axis_weights(oracle.CUBIC, t)
    k = np.arange(4) - 1.0
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert (w * k).sum() == pytest.approx(t, abs=1e-15)
    assert (w * k * k).sum() == pytest.approx(t * t + 1.0 / 3.0, abs=1e-15)
    assert np.all(w >= 0.0)


def test_cubic_weights_at_texel_centre():
    # at t = 0 the weights are (1/6, 4/6, 1/6, 0)
    w = oracle.axis_weights(oracle.CUBIC, 0.0)
    assert np.allclose(w, [1 / 6, 4 / 6, 1 / 6, 0.0], rtol=0, atol=1e-17)


@pytest.mark.parametrize("t", T_GRID)
def test_linear_axis_weights(t):
    w = oracle.axis_weights(oracle.LINEAR, t)
    assert w[0] == 1.0 - t and w[1] == t and w[2] == 0.0 and w[3] == 0.0
