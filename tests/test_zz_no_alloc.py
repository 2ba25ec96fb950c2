"""GPU check of the allocation-free minimiser entry point.

lj_bh_minimize_batch_noalloc runs the same kernels as lj_bh_minimize_batch
with the library's fixed per-device scratch in place of a caller workspace,
and its size classes in turn on the caller's stream.  Per-cluster results do
not depend on the launch schedule, so every output must equal the workspace
entry point's bit for bit, in both precisions, on two calls in a row, the
second with a smaller batch (the scratch keeps the first call's contents).
"""
import numpy as np
import pytest
import torch

from gpu_util import announce, host_dict, to_dev
from paper_2510_25938_amd import lj
from paper_2510_25938_amd.inputs import random_starts, uniform_sizes

pytestmark = pytest.mark.gpu

KEYS = ("xyz", "energy", "gnorm", "iters", "evals", "status", "xyz_switch")


def compare(sizes, seed, precision, pair="lj"):
    off, x = random_starts(sizes, seed)
    if pair == "lj":
        b, xd = to_dev(off, x)
    else:
        b = lj.ClusterBatch(off, pair=pair, rho=6.0)
        xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    p = lj.lbfgs_params()
    sw = precision == "mixed"
    announce(f"noalloc {precision} {pair} clusters={len(sizes)} max_n={max(sizes)} seed={seed}")
    ref = host_dict(lj.minimize(b, xd, p, precision, switch_point=sw))
    got = host_dict(lj.minimize_noalloc(b, xd, p, precision, switch_point=sw))
    for k in KEYS:
        if ref[k] is None:
            assert got[k] is None
            continue
        assert np.array_equal(got[k], ref[k]), k
    assert np.all(got["status"] == lj.CONVERGED)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_workspace_entry_two_calls(precision):
    # first call: every size class the entry point takes (0-256 atoms)
    big = [0, 1, 2] + list(uniform_sizes(509, 3, 256, 7101))
    compare(big, 7102, precision)
    # second call, smaller: one class only, fewer clusters
    small = list(uniform_sizes(37, 2, 40, 7103))
    compare(small, 7104, precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_workspace_entry_morse(precision):
    """The Morse pair's one-wavefront kernels take their pair matrix in
    dynamic LDS; the allocation-free entry launches them the same way."""
    compare(list(uniform_sizes(300, 2, 40, 7106)), 7107, precision, pair="morse")
    compare(list(uniform_sizes(21, 2, 16, 7108)), 7109, precision, pair="morse")


def test_noalloc_rejects_over_limit_shapes():
    off, x = random_starts([300, 13], 7105)
    b, xd = to_dev(off, x)
    with pytest.raises(lj.LJError) as e:
        lj.minimize_noalloc(b, xd)
    assert e.value.args[1] == lj.E_UNSUPPORTED
    torch.cuda.synchronize()
