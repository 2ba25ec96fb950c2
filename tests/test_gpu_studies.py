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
    out = subprocess.run([sys.executable, "-m", "paper_2510_25938_amd.cli", str(src), "--steps",
                          "30", "--cands", "4", "--quiet"], capture_output=True, text=True,
                         timeout=180)
    assert out.returncode == 0, out.stderr
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
    rows = studies.scaling(n_atoms=13, steps=20, chains=8, cands=(1, 4), target=-44.3268)
    assert [r["cands"] for r in rows] == [1, 4]
    assert rows[0]["speedup"] == pytest.approx(1.0) and rows[1]["speedup"] > 1.0
    assert all(r["final_best_mean"] < -40.0 for r in rows)
