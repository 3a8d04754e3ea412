"""Pins of the oracle's filter constants (Eq. 7-10 and the t/u tables after
Eq. 16) against the conditions that define a Daubechies-4 orthonormal wavelet.

The four conditions sum(h) = sqrt(2), sum(h^2) = 1, h0*h2 + h1*h3 = 0 and
sum((-1)^k * k * h_k) = 0 admit only D4 and its mirror image, so together with
the ordering checks they fix h without retyping its formula.
"""
import math

import numpy as np


def test_lowpass_defining_conditions(oracle):
    h = oracle.filters()["h"]
    assert abs(h.sum() - math.sqrt(2.0)) < 1e-15
    assert abs((h * h).sum() - 1.0) < 1e-15
    assert abs(h[0] * h[2] + h[1] * h[3]) < 1e-16  # orthogonal to its shift by 2
    k = np.arange(4)
    alt = (-1.0) ** k
    assert abs((alt * h).sum()) < 1e-15  # zero at Nyquist (first vanishing moment)
    assert abs((alt * k * h).sum()) < 1e-15  # second vanishing moment
    # even and odd taps each sum to 1/sqrt(2)
    assert abs(h[0] + h[2] - 1 / math.sqrt(2.0)) < 1e-15
    assert abs(h[1] + h[3] - 1 / math.sqrt(2.0)) < 1e-15
    # D4 rather than its mirror: the largest tap is h1, and h3 is the only negative one
    assert np.argmax(h) == 1 and h[3] < 0 < h[2] < h[0]


def test_lowpass_is_unique_solution_family(oracle):
    """Solve the four defining conditions numerically from two starting points
    and check the oracle's h is one of the (two) solutions."""
    from scipy.optimize import fsolve

    def eqs(v):
        k = np.arange(4)
        return [v.sum() - math.sqrt(2), (v * v).sum() - 1, v[0] * v[2] + v[1] * v[3],
                (((-1.0) ** k) * k * v).sum()]

    h = oracle.filters()["h"]
    sols = [fsolve(eqs, x0) for x0 in ([0.5, 0.8, 0.2, -0.1], [-0.1, 0.2, 0.8, 0.5])]
    assert any(np.allclose(s, h, atol=1e-12) for s in sols)


def test_highpass_reading(oracle):
    f = oracle.filters()
    h, g = f["h"], f["g"]
    k = np.arange(4)
    assert abs(g.sum()) < 1e-15
    assert abs((g * g).sum() - 1.0) < 1e-15
    assert abs((k * g).sum()) < 1e-15  # annihilates linear ramps
    assert abs((h * g).sum()) < 1e-16
    assert abs(h[2] * g[0] + h[3] * g[1]) < 1e-16  # h, g orthogonal at shift 2
    assert abs(h[0] * g[2] + h[1] * g[3]) < 1e-16
    assert abs(g[0] * g[2] + g[1] * g[3]) < 1e-16
    # quadrature mirror: g_k = (-1)^k h_{3-k}
    assert np.array_equal(g, ((-1.0) ** k) * h[::-1])


def test_printed_highpass_is_not_a_wavelet_filter():
    """Eq. 9-10 as printed: g_i = (2i + sqrt3 - 3)/(4 sqrt2), g_{i+2} = (sqrt3 - 1 - 2i)/(4 sqrt2).
    Its taps do not sum to zero and its energy is not 1, which is why the
    oracle reads Eq. 9-10 as the quadrature-mirror relation instead."""
    r3, d = math.sqrt(3), 4 * math.sqrt(2)
    printed = np.array([(2 * i + r3 - 3) / d for i in (0, 1)] + [(r3 - 1 - 2 * i) / d for i in (0, 1)])
    assert abs(printed.sum()) > 0.1
    assert abs((printed ** 2).sum() - 1.0) > 0.5


def test_synthesis_tables(oracle):
    f = oracle.filters()
    h, g, t, u = f["h"], f["g"], f["t"], f["u"]
    assert list(t) == [h[2], g[2], h[0], g[0]]
    assert list(u) == [h[3], g[3], h[1], g[1]]
