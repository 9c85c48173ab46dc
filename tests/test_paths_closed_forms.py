"""Closed forms the GPU path sampler is checked against, pinned on the CPU
by numerical integration (no GPU): the form factor from a point to a
parallel square centred above it, which gives the direct illumination the
next-event estimate must average to."""
import math

import numpy as np


def corner_form_factor(a, b, c):
    """Form factor from a differential area to a parallel a x b rectangle at
    distance c whose corner lies on the element's normal (the classic
    configuration factor for parallel planes)."""
    A, B = a / c, b / c
    sa, sb = math.sqrt(1.0 + A * A), math.sqrt(1.0 + B * B)
    return (A / sa * math.atan(B / sa) + B / sb * math.atan(A / sb)) / (2.0 * math.pi)


def centred_square_form_factor(s, h):
    """Point below the centre of a square of half size s at height h: four
    corner rectangles of s x s."""
    return 4.0 * corner_form_factor(s, s, h)


def test_form_factor_against_numerical_integration():
    # F = integral over the square of cos cos' / (pi d^2), both cosines h / d
    for s, h in ((0.5, 1.0), (0.25, 2.0), (1.5, 0.7)):
        m = 2000
        x = (np.arange(m) + 0.5) / m * 2.0 * s - s
        X, Z = np.meshgrid(x, x)
        d2 = X * X + Z * Z + h * h
        num = float(np.sum(h * h / (np.pi * d2 * d2)) * (2.0 * s / m) ** 2)
        assert abs(centred_square_form_factor(s, h) - num) < 1e-6, (s, h)


def test_form_factor_limits():
    # a square much larger than its height covers the whole hemisphere
    assert abs(centred_square_form_factor(1e4, 1.0) - 1.0) < 1e-3
    # a small square: F ~ area / (pi h^2)
    s, h = 1e-3, 1.0
    assert abs(centred_square_form_factor(s, h) / ((2 * s) ** 2 / (math.pi * h * h)) - 1.0) < 1e-5
