"""CPU checks of the studies module's structure test (no GPU needed)."""
import numpy as np

from oracle import oracle as O
from paper_2510_25938_amd import studies
from paper_2510_25938_amd.inputs import random_starts
from test_oracle_lbfgs import truncated_octahedron38


def test_o_h_shell_check_on_truncated_octahedron():
    from test_oracle_lbfgs import truncated_octahedron38
    x = truncated_octahedron38()
    r = O.minimize(np.array([0, 38], np.int32), x)
    assert studies.o_h_shells(r["xyz"])
    assert not studies.o_h_shells(random_starts([38], 1)[1])
