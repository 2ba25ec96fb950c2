"""Pins of the oracle's Morse pair (the pair-potential extension).

V(r) = t (t - 2), t = exp(rho (1 - r)): well depth 1 at r = 1, range rho.
Each check is fixed by the definition or by mathematics, not by the oracle:
the value and zero of the well, its curvature 2 rho^2 (equal to the Eq. (1)
curvature in well units when rho = 6), closed forms of symmetric clusters, an
independent extended-precision i<j sum, finite differences, invariances,
Newton's third law and the unique minima of 2, 3 and 4 atoms.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_25938_amd.inputs import random_starts


def one(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    return np.array([0, x.shape[1]], np.int32), x


def eg(x, rho=6.0, pair="morse"):
    off, x = one(x)
    E, g = O.energy_grad(off, x, pair, rho)
    return E[0], g


def dimer(r):
    return np.array([[0.0, r], [0.0, 0.0], [0.0, 0.0]])


def spread_cluster(n, seed, dmin=0.8):
    rng = np.random.default_rng(seed)
    pts = []
    L = 1.2 * n ** (1 / 3) + 1.0
    while len(pts) < n:
        p = rng.uniform(-L / 2, L / 2, 3)
        if all(np.linalg.norm(p - q) > dmin for q in pts):
            pts.append(p)
    return np.ascontiguousarray(np.array(pts).T)


@pytest.mark.parametrize("rho", [3.0, 6.0, 10.0, 14.0])
def test_well_depth_zero_and_tail(rho):
    E, g = eg(dimer(1.0), rho)
    assert E == -1.0 and np.all(g == 0.0)
    r0 = 1.0 - math.log(2.0) / rho  # t = 2: V = 0
    assert abs(eg(dimer(r0), rho)[0]) < 1e-14
    assert eg(dimer(1.0 + 800.0 / rho), rho)[0] == 0.0  # beyond the exp range: exactly 0
    # repulsive inside the well, attractive outside (g_0x = dE/dx_0)
    assert eg(dimer(0.9), rho)[1][0, 0] > 0 and eg(dimer(1.1), rho)[1][0, 0] < 0


@pytest.mark.parametrize("rho", [3.0, 6.0, 10.0])
def test_curvature_at_the_well(rho):
    h = 1e-4
    c = (eg(dimer(1 + h), rho)[0] - 2 * eg(dimer(1.0), rho)[0] + eg(dimer(1 - h), rho)[0]) / h**2
    assert abs(c / (2 * rho * rho) - 1) < 1e-5


def test_rho6_matches_eq1_curvature_in_well_units():
    # Eq. (1) has its well (depth 1) at r_e = 2^(1/6); in units of r_e its
    # curvature is 72 = 2 * 6^2, the Morse curvature at rho = 6
    re, h = 2.0 ** (1 / 6), 1e-4
    lj = lambda r: eg(dimer(r * re), pair="lj")[0]
    c_lj = (lj(1 + h) - 2 * lj(1.0) + lj(1 - h)) / h**2
    c_m = (eg(dimer(1 + h))[0] - 2 * eg(dimer(1.0))[0] + eg(dimer(1 - h))[0]) / h**2
    assert abs(c_lj / 72 - 1) < 1e-5 and abs(c_m / 72 - 1) < 1e-5


@pytest.mark.parametrize("rho", [3.0, 6.0])
def test_triangle_and_tetrahedron(rho):
    tri = np.array([[0.0, 1.0, 0.5], [0.0, 0.0, math.sqrt(3) / 2], [0.0, 0.0, 0.0]])
    assert abs(eg(tri, rho)[0] + 3.0) < 1e-14
    # alternate cube corners: edge 2 sqrt(2), scaled to edge 1
    tet = np.array([[1, 1, -1, -1], [1, -1, 1, -1], [1, -1, -1, 1]], float) / (2 * math.sqrt(2))
    E, g = eg(tet, rho)
    assert abs(E + 6.0) < 1e-13 and np.abs(g).max() < 1e-12


def energy_longdouble(x, rho):
    xl = x.astype(np.longdouble)
    n, E = x.shape[1], np.longdouble(0)
    for i in range(n):
        for j in range(i + 1, n):
            d = xl[:, i] - xl[:, j]
            r = np.sqrt(d @ d)
            t = np.exp(np.longdouble(rho) * (1 - r))
            E += t * (t - 2)
    return E


@pytest.mark.parametrize("n,seed,rho", [(5, 1, 6.0), (13, 2, 3.0), (20, 3, 10.0)])
def test_against_extended_precision_sum(n, seed, rho):
    x = spread_cluster(n, seed)
    E = eg(x, rho)[0]
    El = energy_longdouble(x, rho)
    assert abs(E - float(El)) <= 1e-13 * float(abs(El))


@pytest.mark.parametrize("n,seed,rho", [(4, 5, 6.0), (8, 6, 3.0), (8, 7, 14.0)])
def test_central_finite_differences(n, seed, rho):
    x = spread_cluster(n, seed)
    _, g = eg(x, rho)
    h = 1e-6
    for c in range(3):
        for i in range(n):
            xp, xm = x.copy(), x.copy()
            xp[c, i] += h
            xm[c, i] -= h
            fd = (eg(xp, rho)[0] - eg(xm, rho)[0]) / (2 * h)
            assert abs(fd - g[c, i]) <= 1e-7 * max(1.0, abs(g[c, i]))


@pytest.mark.parametrize("n,seed", [(7, 8), (16, 9)])
def test_invariances_net_force_torque(n, seed):
    x = spread_cluster(n, seed)
    E, g = eg(x)
    assert np.abs(g.sum(axis=1)).max() < 1e-12 * np.abs(g).max() * n
    torque = np.cross(x.T, g.T).sum(axis=0)
    assert np.abs(torque).max() < 1e-11 * np.abs(g).max() * n
    assert abs(eg(x + np.array([[0.3], [-1.7], [2.2]]))[0] - E) < 1e-12 * abs(E)
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    assert abs(eg(R @ x)[0] - E) < 1e-12 * abs(E)
    perm = np.random.default_rng(seed).permutation(n)
    Ep, gp = eg(x[:, perm])
    assert abs(Ep - E) < 1e-12 * abs(E) and np.allclose(gp, g[:, perm], rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("n,emin", [(2, -1.0), (3, -3.0), (4, -6.0)])
@pytest.mark.parametrize("rho", [3.0, 6.0])
def test_unique_small_minima(n, emin, rho):
    off, x = random_starts([n] * 20, 40 + n)
    r = O.minimize(off, x, O.lbfgs_params(pair="morse", rho=rho))
    assert np.all(r["status"] == O.CONVERGED)
    assert np.abs(r["energy"] - emin).max() < 1e-12
