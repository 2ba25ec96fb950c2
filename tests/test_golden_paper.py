"""The paper's printed parameters (tests/golden/paper_parameters.txt) against
the oracle: its defaults, and behaviour that each parameter fixes."""
import math
import os

import numpy as np

from oracle import oracle as O
from paper_2510_25938_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.txt")


def golden():
    vals = {}
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = (t.strip() for t in line.split("="))
                vals[k] = float(v)
    return vals


def test_fixture_is_complete():
    assert set(golden()) == {"perturbation_cube_side_over_stepsize", "metropolis_temperature",
                             "adaptation_interval_steps", "target_acceptance_rate",
                             "bh_steps_per_run", "lj_prefactor", "lj_repulsive_exponent",
                             "lj_attractive_exponent"}


def test_perturbation_fills_a_cube_of_side_two_stepsizes():
    g = golden()
    s = 0.4
    x = np.zeros((3, 50))
    d = np.concatenate([O.perturb(x, s, seed=7, chain=0, step=k, cand=0) for k in range(200)],
                       axis=1)
    half = g["perturbation_cube_side_over_stepsize"] * s / 2
    assert np.all(d >= -half) and np.all(d < half)  # inside the cube
    for c in range(3):  # and filling it along every axis (10000 draws each)
        assert d[c].max() - d[c].min() > 0.999 * 2 * half
    assert np.max(np.sqrt(np.sum(d * d, axis=0))) > 1.05 * half  # corners: a cube, not a ball


def test_adaptation_interval_and_target():
    g = golden()
    n = int(g["adaptation_interval_steps"])
    p = O.bh_params(1, 1, kT=1e-300, seed=0)  # uphill moves always rejected
    assert p.adapt_interval == n and p.target_rate == g["target_acceptance_rate"]
    target = g["target_acceptance_rate"] * n
    for accepts in (int(target) + 1, int(target), int(target) - 1):
        st = O.chain_state(0.0, 0.4)
        for k in range(n):
            O.bh_decide(st, p, 0, [st.e_cur - 1.0 if k < accepts else st.e_cur + 1.0])
            if k < n - 1:
                assert st.step == 0.4  # unchanged inside the window
        grow = accepts > target
        same = accepts == target
        assert st.step == (0.4 if same else 0.4 / 0.9 if grow else 0.4 * 0.9)


def test_metropolis_at_the_paper_temperature():
    """At T = 1.0 an uphill move of T ln 2 passes half of the uniform draws."""
    T = golden()["metropolis_temperature"]
    p = O.bh_params(1, 1, kT=T, seed=11, adapt_interval=10 ** 6)
    dE = T * math.log(2.0)
    acc = sum(O.bh_decide(O.chain_state(0.0, 0.4, step_index=k), p, 0, [dE])[1]
              for k in range(4000))
    assert abs(acc / 4000 - 0.5) < 0.03  # binomial sd 0.008
    assert all(O.bh_decide(O.chain_state(0.0, 0.4, step_index=k), p, 0, [40.0 * T])[1] == 0
               for k in range(200))  # exp(-40) is below every draw here


def test_pair_energy_follows_eq1():
    g = golden()
    a, m, k = g["lj_prefactor"], g["lj_repulsive_exponent"], g["lj_attractive_exponent"]
    for r in (0.95, 2.0 ** (1 / 6), 1.5, 2.5):
        x = np.array([[0.0, r], [0.0, 0.0], [0.0, 0.0]])
        E, _ = O.energy_grad(np.array([0, 2], np.int32), x)
        assert math.isclose(E[0], a * (r ** -m - r ** -k), rel_tol=1e-14)


def test_lj13_chain_workload_has_the_paper_run_length():
    assert inputs.lj13_bh().steps == int(golden()["bh_steps_per_run"])
