"""Pins of the oracle's energy and gradient (Eq. 1 and its derivative).

Each check is fixed by the mathematics, not by the oracle itself: closed-form
energies of symmetric clusters, the r^-12 / r^-6 scaling law, invariances,
Newton's third law, the virial identity, central finite differences and an
independent extended-precision i<j sum.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_25938_amd.inputs import random_starts

RMIN = 2.0 ** (1.0 / 6.0)


def one(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    return np.array([0, x.shape[1]], np.int32), x


def eg(x):
    off, x = one(x)
    E, g = O.energy_grad(off, x)
    return E[0], g


def spread_cluster(n, seed, dmin=0.85):
    """Random cluster with every pair distance above dmin (rejection sampling)."""
    rng = np.random.default_rng(seed)
    pts = []
    L = 1.3 * n ** (1 / 3) + 1.0
    while len(pts) < n:
        p = rng.uniform(-L / 2, L / 2, 3)
        if all(np.linalg.norm(p - q) > dmin for q in pts):
            pts.append(p)
    return np.ascontiguousarray(np.array(pts).T)


def v_ld(r2):
    inv6 = np.longdouble(1) / (r2 * r2 * r2)
    return inv6 * inv6 - inv6


def energy_longdouble(x):
    """4 sum_{i<j} (r^-12 - r^-6) accumulated in x87 extended precision."""
    xl = x.astype(np.longdouble)
    n = x.shape[1]
    E = np.longdouble(0)
    for i in range(n):
        for j in range(i + 1, n):
            d = xl[:, i] - xl[:, j]
            E += v_ld(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
    return 4 * E


def test_dimer_closed_form():
    for r in [0.9, 1.0, RMIN, 1.3, 2.0, 3.7]:
        x = np.array([[0.0, r], [0.0, 0.0], [0.0, 0.0]])
        E, g = eg(x)
        ref = 4.0 * (r ** -12 - r ** -6)
        assert E == pytest.approx(ref, rel=1e-14, abs=1e-300)
        dEdr = 4.0 * (-12.0 * r ** -13 + 6.0 * r ** -7)
        # gradient on atom 1 (at +r) is +dE/dr along x, atom 0 gets the opposite
        assert g[0, 1] == pytest.approx(dEdr, rel=1e-13)
        assert g[0, 0] == pytest.approx(-dEdr, rel=1e-13)
        assert np.all(g[1:] == 0.0)


def test_dimer_minimum():
    x = np.array([[0.0, RMIN], [0.0, 0.0], [0.0, 0.0]])
    E, g = eg(x)
    assert E == pytest.approx(-1.0, abs=2e-15)
    assert np.max(np.abs(g)) < 1e-13


def test_triangle_and_tetrahedron():
    tri = RMIN * np.array([[0, 1, 0.5], [0, 0, math.sqrt(3) / 2], [0, 0, 0]])
    E, g = eg(tri)
    assert E == pytest.approx(-3.0, abs=1e-14)
    assert np.max(np.abs(g)) < 1e-12
    tet = RMIN / math.sqrt(8.0) * np.array([[1, 1, -1, -1], [1, -1, 1, -1], [1, -1, -1, 1]],
                                          dtype=float)
    E, g = eg(tet)
    assert E == pytest.approx(-6.0, abs=1e-14)
    assert np.max(np.abs(g)) < 1e-12


@pytest.mark.parametrize("n,seed", [(2, 1), (3, 2), (5, 3), (8, 4), (8, 5)])
def test_against_extended_precision_sum(n, seed):
    x = spread_cluster(n, seed, dmin=0.8)
    E, _ = eg(x)
    ref = float(energy_longdouble(x))
    assert abs(E - ref) <= 1e-14 * max(1.0, abs(ref))


@pytest.mark.parametrize("n,seed", [(4, 11), (7, 12), (13, 13)])
def test_scaling_law_and_virial(n, seed):
    """E(lx) = l^-12 A - l^-6 B for all l; the virial sum_i x_i.g_i = -12A + 6B."""
    x = spread_cluster(n, seed)
    E1, g = eg(x)
    E2, _ = eg(1.1 * x)
    # solve for A, B from l = 1 and l = 1.1, check at l = 0.95
    a, b = 1.1 ** -12, 1.1 ** -6
    M = np.array([[1.0, -1.0], [a, -b]])
    A, B = np.linalg.solve(M, np.array([E1, E2]))
    E3, _ = eg(0.95 * x)
    assert E3 == pytest.approx(0.95 ** -12 * A - 0.95 ** -6 * B, rel=1e-9)
    vir = float(np.sum(x * g))
    assert vir == pytest.approx(-12 * A + 6 * B, rel=1e-9, abs=1e-9 * (abs(A) + abs(B)))


@pytest.mark.parametrize("n,seed", [(3, 21), (6, 22), (8, 23)])
def test_central_finite_differences(n, seed):
    x = spread_cluster(n, seed)
    _, g = eg(x)
    h = 1e-6
    fd = np.zeros_like(x)
    for c in range(3):
        for i in range(n):
            xp, xm = x.copy(), x.copy()
            xp[c, i] += h
            xm[c, i] -= h
            fd[c, i] = (eg(xp)[0] - eg(xm)[0]) / (2 * h)
    scale = max(1.0, np.max(np.abs(g)))
    assert np.max(np.abs(fd - g)) <= 1e-7 * scale


@pytest.mark.parametrize("n,seed", [(13, 31), (38, 32), (80, 33)])
def test_invariances_net_force_torque(n, seed):
    off, x = random_starts([n], seed)
    E, g = O.energy_grad(off, x)
    eabs, gabs = O.abs_sums(off, x)
    rng = np.random.default_rng(seed)
    # translation
    Et, gt = O.energy_grad(off, x + rng.normal(size=(3, 1)))
    assert abs(Et[0] - E[0]) <= 1e-12 * eabs[0]
    # rotation
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    Er, gr = O.energy_grad(off, Q @ x)
    assert abs(Er[0] - E[0]) <= 1e-12 * eabs[0]
    assert np.max(np.abs(gr - Q @ g)) <= 1e-11 * np.max(gabs)
    # permutation
    perm = rng.permutation(n)
    Ep, gp = O.energy_grad(off, x[:, perm])
    assert abs(Ep[0] - E[0]) <= 1e-12 * eabs[0]
    assert np.max(np.abs(gp - g[:, perm])) <= 1e-12 * np.max(gabs)
    # zero net force and torque
    assert np.max(np.abs(g.sum(axis=1))) <= 1e-12 * np.sum(gabs)
    torque = np.cross(x.T, g.T).sum(axis=0)
    assert np.max(np.abs(torque)) <= 1e-11 * np.sum(gabs * np.abs(x).max())


def test_batch_is_per_cluster_and_ragged():
    sizes = [0, 1, 2, 13, 0, 38, 5]
    off, x = random_starts(sizes, 7)
    E, g = O.energy_grad(off, x)
    for b, n in enumerate(sizes):
        o = off[b]
        Eb, gb = eg(x[:, o:o + n]) if n > 0 else (0.0, np.zeros((3, 0)))
        assert E[b] == Eb
        assert np.array_equal(g[:, o:o + n], gb)
    assert E[0] == 0.0 and E[1] == 0.0 and np.all(g[:, off[1]:off[2]] == 0.0)


def test_coincident_atoms_are_nonfinite():
    x = np.zeros((3, 2))
    E, _ = eg(x)
    assert not np.isfinite(E)


def test_pairwise_summation_order():
    # Left-to-right gives 2^53 + 2; the pairwise tree ((1+0) + (1+2^53)) gives 2^53.
    big = 2.0 ** 53
    assert O.tree_sum([1.0, 0.0, 1.0, big]) == big
    assert ((1.0 + 0.0) + 1.0) + big == big + 2.0
    # Five values pad to eight leaves: ((1+0)+(1+2^53)) + ((1+0)+(0+0)) = 2^53,
    # while left to right gives 2^53 + 4.
    assert O.tree_sum([1.0, 0.0, 1.0, big, 1.0]) == big
    assert (((1.0 + 0.0) + 1.0) + big) + 1.0 == big + 4.0
    rng = np.random.default_rng(5)
    v = rng.normal(size=1000) * 10.0 ** rng.uniform(-8, 8, size=1000)
    exact = math.fsum(v)
    bound = math.ceil(math.log2(1024)) * 2.0 ** -53 * np.sum(np.abs(v)) * 1.01
    assert abs(O.tree_sum(v) - exact) <= bound
    assert O.tree_sum([]) == 0.0
    assert O.tree_sum([3.5]) == 3.5
