"""GPU checks of the host glue: the .molden CLI and the studies module."""
import subprocess
import sys

import numpy as np
import pytest
import torch

from gpu_util import announce
from oracle import oracle as O
from paper_2510_25938_amd import studies
from paper_2510_25938_amd.inputs import planes_to_aos, random_starts
from paper_2510_25938_amd.molden import read_first_geometry, write_geometries

pytestmark = pytest.mark.gpu


def test_cli_writes_accepted_structures(tmp_path):
    _, x = random_starts([13], 99)
    src = tmp_path / "lj13.molden"
    write_geometries(str(src), [planes_to_aos(x)], [0.0], ["Ar"] * 13)
    announce("cli lj13 30 steps")
    trace = tmp_path / "trace.csv"
    out = subprocess.run([sys.executable, "-m", "paper_2510_25938_amd.cli", str(src), "--steps",
                          "30", "--cands", "4", "--quiet", "--trace", str(trace)],
                         capture_output=True, text=True, timeout=180)
    assert out.returncode == 0, out.stderr
    # the per-step series of Figs. 2-3: running lowest trial energy and lowest
    # accepted energy never increase; accepted rows set the current energy
    t = np.genfromtxt(trace, delimiter=",", names=True)
    assert len(t) == 30 and np.all(np.diff(t["e_lowest_trial"]) <= 0)
    assert np.all(np.diff(t["e_best_accepted"]) <= 0)
    acc = t["accepted"] == 1
    assert np.all(t["e_current"][acc] == t["e_trial"][acc])  # FP64: no polish
    assert np.all(t["e_best_accepted"] <= t["e_current"])
    acc = tmp_path / "lj13_accepted.molden"
    text = acc.read_text()
    n_frames = text.count("E = ")
    assert n_frames >= 1 and "accepted structures" in out.stdout
    # every written frame is a minimum whose energy is the one written
    frames = text.split("[GEOMETRIES] XYZ\n")[1].strip().split("\n")
    k = 0
    for _ in range(n_frames):
        n = int(frames[k]); e = float(frames[k + 1].split("=")[1])
        xyz = np.array([[float(v) for v in ln.split()[1:4]] for ln in frames[k + 2:k + 2 + n]])
        E, g = O.energy_grad(np.array([0, n], np.int32), np.ascontiguousarray(xyz.T))
        assert abs(E[0] - e) <= 1e-9 * abs(e)
        k += 2 + n


def test_scaling_study_runs():
    announce("scaling study small")
    rows = studies.scaling(n_atoms=13, steps=20, chains=8, cands=(1, 4))
    assert [r["cands"] for r in rows] == [1, 4]
    assert rows[0]["speedup"] == pytest.approx(1.0) and rows[1]["speedup"] > 1.0
    assert all(r["final_best_mean"] < -40.0 for r in rows)
    assert all(r["chains_hit"] >= 1 for r in rows)  # the LJ13 icosahedron


def oracle_chain_run(off, xmin, emin, cands, seed, steps, chain0=0, step0=0.4):
    params = O.bh_params(off.size - 1, cands, kT=0.8, seed=seed)
    xcur = np.ascontiguousarray(xmin).copy()
    xbest = xcur.copy()
    states = [O.chain_state(float(e), step0) for e in emin]
    tr = O.bh_run(off, xcur, states, params, O.lbfgs_params(), steps, xbest=xbest, chain0=chain0)
    return xcur, xbest, states, tr


def test_scaling_study_fp64_traces_match_oracle():
    """The candidate-count study in FP64: every chain of every candidate count
    takes the oracle's steps bit for bit (trial, decision, running lowest,
    current energy and step size per step)."""
    announce("scaling study fp64 vs oracle (LJ38, 4 chains, 15 steps, n = 1, 8, 16)")
    traces = {}
    rows = studies.scaling(n_atoms=38, steps=15, chains=4, cands=(1, 8, 16), precision="fp64",
                           traces=traces)
    assert [r["cands"] for r in rows] == [1, 8, 16]
    off = traces["offset"]
    for n in (1, 8, 16):
        _, _, _, tro = oracle_chain_run(off, traces["xyz_min"], traces["e_min"], n,
                                        traces[n]["seed"], 15)
        for k in ("e_trial", "e_best", "e_best_acc", "e_cur", "step"):
            assert np.array_equal(traces[n][k], tro[k], equal_nan=True), (n, k)
        assert np.array_equal(traces[n]["accepted"], tro["accepted"]), n


def test_lj38_search_fp64_hit_checked_by_oracle():
    """Global search for LJ38 in FP64 with a fixed seed and step budget: the
    hit is the truncated octahedron by the oracle's energy and gradient and by
    its O_h shells, and the oracle's run of the same chain finds the same
    structure bit for bit."""
    announce("lj38 global search fp64, 1024 chains x 8, at most 400 steps")
    res = studies.lj38(chains=1024, cands=8, seconds=100.0, chunk=25, precision="fp64", seed=38,
                       max_steps=400)
    assert res["found"], res
    xb = np.ascontiguousarray(np.array(res["xyz"]))
    E, g = O.energy_grad(np.array([0, 38], np.int32), xb)
    assert abs(E[0] - studies.LJ38_GLOBAL) <= 1e-6
    assert np.sqrt(np.sum(g * g)) < 1e-6
    assert res["o_h"] and studies.o_h_shells(xb)
    # the oracle runs the hit chain alone from the same start minimum
    k, steps = res["chain"], res["steps"]
    off, x = random_starts([38] * 1024, 38)
    so = np.array([0, 38], np.int32)
    r0 = O.minimize(so, np.ascontiguousarray(x[:, 38 * k:38 * (k + 1)]))
    _, xbest, states, _ = oracle_chain_run(so, r0["xyz"], r0["energy"], 8, 38, steps, chain0=k)
    assert np.array_equal(xbest, xb)
    assert states[0].e_best_acc == E[0]
