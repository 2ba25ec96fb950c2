"""Pins of the oracle's sums of absolute pair terms (Eq. 1 and the Morse pair).

These sums scale every a-priori error bound of the FP32 pair arithmetic:
E_abs is the sum over unique pairs of the magnitudes of the two terms of the
pair energy, and g_abs (per atom and component) the sum over partners of the
magnitudes of the two terms of the force component.  For Eq. (1), with
V(r) = 4 r^-12 - 4 r^-6:
    E_abs = sum_{i<j} (4 r^-12 + 4 r^-6)
    g_abs[c][i] = sum_{j!=i} (48 r^-14 + 24 r^-8) |x_i[c] - x_j[c]|
and for the Morse pair V(r) = t^2 - 2 t, t = exp(rho (1 - r)):
    E_abs = sum_{i<j} (t^2 + 2 t)
    g_abs[c][i] = sum_{j!=i} 2 rho (t^2 + t) |x_i[c] - x_j[c]| / r.
They are checked against closed forms (dimer, equilateral triangle) and an
independent i<j loop written with powers of r, so that a dropped term, a
factor of two or a sign slip in the oracle fails here.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_25938_amd.inputs import random_starts


def one(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    return np.array([0, x.shape[1]], np.int32), x


def dimer(r):
    return np.array([[0.0, r * 0.6], [0.0, -r * 0.8], [0.0, 0.0]])


def lj_abs_reference(x):
    """Independent i<j loop over powers of r (no shared sub-expressions)."""
    n = x.shape[1]
    eabs = 0.0
    gabs = np.zeros_like(x)
    for i in range(n):
        for j in range(i + 1, n):
            d = x[:, i] - x[:, j]
            r = math.sqrt(float(d @ d))
            eabs += 4.0 * r ** -12 + 4.0 * r ** -6
            mag = 48.0 * r ** -14 + 24.0 * r ** -8
            gabs[:, i] += mag * np.abs(d)
            gabs[:, j] += mag * np.abs(d)
    return eabs, gabs


def morse_abs_reference(x, rho):
    n = x.shape[1]
    eabs = 0.0
    gabs = np.zeros_like(x)
    for i in range(n):
        for j in range(i + 1, n):
            d = x[:, i] - x[:, j]
            r = math.sqrt(float(d @ d))
            t = math.exp(rho * (1.0 - r))
            eabs += t * t + 2.0 * t
            mag = 2.0 * rho * (t * t + t) / r
            gabs[:, i] += mag * np.abs(d)
            gabs[:, j] += mag * np.abs(d)
    return eabs, gabs


@pytest.mark.parametrize("r", [0.8, 1.0, 2.0 ** (1 / 6), 1.5, 2.5])
def test_lj_dimer_closed_form(r):
    off, x = one(dimer(r))
    ea, ga = O.abs_sums(off, x)
    assert ea[0] == pytest.approx(4.0 * (r ** -12 + r ** -6), rel=1e-14)
    mag = 48.0 * r ** -14 + 24.0 * r ** -8
    for c, dc in enumerate([0.6 * r, 0.8 * r, 0.0]):
        assert ga[c, 0] == pytest.approx(mag * dc, rel=1e-14, abs=0.0)
        assert ga[c, 1] == pytest.approx(mag * dc, rel=1e-14, abs=0.0)


def test_lj_abs_bounds_the_signed_terms():
    # at the dimer minimum the signed energy is -1 and the gradient zero, while
    # the absolute sums are 4 (r^-12 + r^-6) = 3 and the sum of the force
    # terms' magnitudes
    r = 2.0 ** (1 / 6)
    off, x = one(dimer(r))
    ea, ga = O.abs_sums(off, x)
    E, g = O.energy_grad(off, x)
    assert ea[0] == pytest.approx(3.0, rel=1e-14)
    assert abs(E[0]) <= ea[0]
    assert np.all(np.abs(g) <= ga + 1e-15)


@pytest.mark.parametrize("a", [0.95, 2.0 ** (1 / 6), 1.4])
def test_lj_equilateral_triangle(a):
    h = a * math.sqrt(3.0) / 2.0
    x = np.array([[0.0, a, a / 2], [0.0, 0.0, h], [0.0, 0.0, 0.0]])
    off, x = one(x)
    ea, ga = O.abs_sums(off, x)
    assert ea[0] == pytest.approx(3 * 4.0 * (a ** -12 + a ** -6), rel=1e-14)
    mag = 48.0 * a ** -14 + 24.0 * a ** -8
    # atom 0 sees partners at (a, 0) and (a/2, h)
    assert ga[0, 0] == pytest.approx(mag * (a + a / 2), rel=1e-14)
    assert ga[1, 0] == pytest.approx(mag * h, rel=1e-14)
    assert ga[2, 0] == 0.0
    # atom 2 sees both partners at |dx| = a/2, |dy| = h
    assert ga[0, 2] == pytest.approx(mag * a, rel=1e-14)
    assert ga[1, 2] == pytest.approx(2 * mag * h, rel=1e-14)


def test_lj_independent_loop_ragged_batch():
    sizes = [0, 1, 2, 3, 5, 8, 7]
    off, x = random_starts(sizes, 91)
    ea, ga = O.abs_sums(off, x)
    for b, n in enumerate(sizes):
        o = off[b]
        e_ref, g_ref = lj_abs_reference(x[:, o:o + n])
        assert ea[b] == pytest.approx(e_ref, rel=1e-13, abs=0.0)
        np.testing.assert_allclose(ga[:, o:o + n], g_ref, rtol=1e-13, atol=0.0)


@pytest.mark.parametrize("rho", [3.0, 6.0, 10.0])
def test_morse_dimer_closed_form(rho):
    for r in [0.85, 1.0, 1.3, 2.0]:
        off, x = one(dimer(r))
        ea, ga = O.abs_sums(off, x, pair="morse", rho=rho)
        t = math.exp(rho * (1.0 - r))
        assert ea[0] == pytest.approx(t * t + 2.0 * t, rel=1e-14)
        mag = 2.0 * rho * (t * t + t) / r
        assert ga[0, 0] == pytest.approx(mag * 0.6 * r, rel=1e-14)
        assert ga[1, 1] == pytest.approx(mag * 0.8 * r, rel=1e-14)
        assert ga[2, 0] == 0.0


def test_morse_at_well_bottom():
    # r = 1: t = 1, so V = -1 while the absolute terms sum to 3, and the force
    # terms 2 rho t^2 and 2 rho t cancel while their magnitudes add to 4 rho
    rho = 6.0
    off, x = one(dimer(1.0))
    ea, ga = O.abs_sums(off, x, pair="morse", rho=rho)
    assert ea[0] == pytest.approx(3.0, rel=1e-15)
    assert ga[0, 0] + ga[1, 0] == pytest.approx(4.0 * rho * (0.6 + 0.8), rel=1e-14)


@pytest.mark.parametrize("rho", [3.0, 6.0])
def test_morse_independent_loop_ragged_batch(rho):
    sizes = [2, 0, 4, 8, 1, 6]
    off, x = random_starts(sizes, 92)
    ea, ga = O.abs_sums(off, x, pair="morse", rho=rho)
    for b, n in enumerate(sizes):
        o = off[b]
        e_ref, g_ref = morse_abs_reference(x[:, o:o + n], rho)
        assert ea[b] == pytest.approx(e_ref, rel=1e-13, abs=0.0)
        np.testing.assert_allclose(ga[:, o:o + n], g_ref, rtol=1e-13, atol=0.0)


def test_translation_invariance():
    off, x = random_starts([6, 8], 93)
    ea, ga = O.abs_sums(off, x)
    x2 = x + np.array([[0.25], [-0.5], [0.125]])  # exact shifts of coordinates near 1
    ea2, ga2 = O.abs_sums(off, np.ascontiguousarray(x2))
    np.testing.assert_allclose(ea2, ea, rtol=1e-12)
    np.testing.assert_allclose(ga2, ga, rtol=1e-11)
