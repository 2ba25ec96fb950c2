"""GPU parity of every minimiser shape of the small size classes, including
the packed shapes that minimise two or four clusters per wavefront, and of the
shapes the autotuner installs.

Every shape runs the oracle's summation order, so FP64 results are
bit-identical to the oracle whatever the schedule; mixed results are checked
by the FP64 polish from the recorded switch points, which must equal the
oracle's run from those points bit for bit.
"""
import numpy as np
import pytest
import torch

from gpu_util import announce, host, host_dict, to_dev
from oracle import oracle as O
from paper_2510_25938_amd import lj
from paper_2510_25938_amd.inputs import random_starts, uniform_sizes
from test_gpu_bh import oracle_chains, start_chains
from test_gpu_minimize import oracle_params

pytestmark = pytest.mark.gpu

KEYS = ("xyz", "energy", "gnorm", "iters", "evals", "status")


def forced(c, precision, max_n, shape):
    lj.set_schedule(lj.SCHED_MIN_CLASS[c], precision, max_n, shape)


def reset(c, precision, max_n):
    lj.set_schedule(lj.SCHED_MIN_CLASS[c], precision, max_n, -1)


# class 0: clusters of at most 16 atoms fit every shape; at most 32 atoms the
# one-cluster and two-per-wavefront shapes.  Counts are odd so that the last
# packed workgroup has idle teams.
SMALL = [0, 1, 2, 3] + list(uniform_sizes(301, 4, 16, 8101))
MID = [0, 1, 17] + list(uniform_sizes(257, 2, 32, 8102))


# shapes 4-7 are shapes 0-3 compiled for two wavefronts per SIMD
@pytest.mark.parametrize("sizes,shapes", [(SMALL, tuple(range(8))), (MID, (0, 2, 4, 6))])
@pytest.mark.parametrize("pair", ["lj", "morse"])
def test_class0_shapes_fp64_bitwise(sizes, shapes, pair):
    off, x = random_starts(sizes, 8103 + len(sizes))
    b = lj.ClusterBatch(off, pair=pair, rho=6.0)
    xd = torch.from_numpy(x).cuda()
    p = lj.lbfgs_params()
    op = oracle_params(p)
    op.pair, op.rho = lj.PAIRS[pair], 6.0
    ro = O.minimize(off, x, op)
    try:
        for k in shapes:
            announce(f"class-0 shape {k} fp64 {pair} clusters={b.num} max_n={b.max_n}")
            forced(0, "fp64", b.max_n, k)
            r = host_dict(lj.minimize(b, xd, p, "fp64"))
            for key in KEYS:
                assert np.array_equal(r[key], ro[key]), (k, key)
    finally:
        reset(0, "fp64", b.max_n)
    assert np.all(ro["status"] == lj.CONVERGED)


@pytest.mark.parametrize("sizes,shapes", [(SMALL, tuple(range(8))), (MID, (0, 2, 4, 6))])
def test_class0_shapes_mixed_polish_bitwise(sizes, shapes):
    off, x = random_starts(sizes, 8203 + len(sizes))
    b, xd = to_dev(off, x)
    p = lj.lbfgs_params()
    try:
        for k in shapes:
            announce(f"class-0 shape {k} mixed clusters={b.num} max_n={b.max_n}")
            forced(0, "mixed", b.max_n, k)
            r = host_dict(lj.minimize(b, xd, p, "mixed", switch_point=True))
            ro = O.minimize(off, r["xyz_switch"], oracle_params(p))
            for key in ("xyz", "energy", "gnorm", "status"):
                assert np.array_equal(r[key], ro[key]), (k, key)
            assert np.all(r["status"] == lj.CONVERGED)
    finally:
        reset(0, "mixed", b.max_n)


@pytest.mark.parametrize("c,sizes,shapes", [(1, [65, 13, 80, 100, 128, 70], (0, 1)),
                                            (2, [129, 150, 38, 192, 170], (0, 1))])
def test_class12_shapes_fp64_bitwise(c, sizes, shapes):
    off, x = random_starts(sizes, 8300 + c)
    b, xd = to_dev(off, x)
    p = lj.lbfgs_params()
    ro = O.minimize(off, x, oracle_params(p))
    try:
        for k in shapes:
            announce(f"class-{c} shape {k} fp64 sizes={sizes}")
            forced(c, "fp64", b.max_n, k)
            r = host_dict(lj.minimize(b, xd, p, "fp64"))
            for key in KEYS:
                assert np.array_equal(r[key], ro[key]), (k, key)
    finally:
        reset(c, "fp64", b.max_n)


def test_packed_candidates_in_bh_chains_fp64_bitwise():
    """LJ13 chains whose candidates run four per wavefront: every trace row
    and the final state equal the oracle's basin hopping bit for bit."""
    sizes, steps = [13] * 6, 25
    off, b, r, p = start_chains(sizes, 8401)
    bh = lj.bh_params(cands=8, kT=0.8, seed=8401)
    try:
        forced(0, "fp64", 13, 3)
        announce("bh fp64 6 x LJ13 x 8 candidates, four clusters per wavefront")
        bhx = lj.BasinHopping(b, r["xyz"], r["energy"], bh, p, "fp64", trace_steps=steps,
                              trace_candidates=True)
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            bhx.step(steps)
        side.synchronize()
    finally:
        reset(0, "fp64", 13)
    xcur, xbest, states, tro = oracle_chains(off, r, bh, p, steps)
    torch.cuda.synchronize()
    tr = {k: (None if v is None else v.cpu().numpy()) for k, v in bhx.trace.items()}
    for k in ("e_trial", "e_best", "e_best_acc", "e_cur", "step"):
        assert np.array_equal(tr[k], tro[k], equal_nan=True), k
    assert np.array_equal(tr["e_cand"], tro["ecand"], equal_nan=True)
    assert np.array_equal(host(bhx.xyz_cur), xcur)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotuned_shapes_keep_parity(tmp_path, precision):
    """The autotuner times every valid shape of each class present and installs
    one; the tuned batch still matches the oracle (FP64: bitwise; mixed: the
    polish from the switch points), and the cache installs the same shapes."""
    sizes = list(uniform_sizes(1500, 5, 150, 8501))
    off, x = random_starts(sizes, 8502)
    b, xd = to_dev(off, x)
    announce(f"autotune {precision} {b.num} clusters N 5..150")
    cache = str(tmp_path / "sched.json")
    try:
        res = lj.autotune(b, xd, precision, cache=cache)
        assert res["min_ms"] > 0 and set(res["min_class"]) == {0, 1, 2}
        for c, k in res["min_class"].items():
            assert lj.CLASS_SHAPES[c][k][1] >= min(b.max_n, (64, 128, 256)[c])
        p = lj.lbfgs_params()
        r = host_dict(lj.minimize(b, xd, p, precision, switch_point=precision == "mixed"))
        start = r["xyz_switch"] if precision == "mixed" else x
        ro = O.minimize(off, start, oracle_params(p))
        for key in ("xyz", "energy", "gnorm", "status"):
            assert np.array_equal(r[key], ro[key]), key
        for c in range(3):
            reset(c, precision, b.max_n)
        lj.load_schedules(cache)
        for c, k in res["min_class"].items():
            assert lj.get_schedule(lj.SCHED_MIN_CLASS[c], precision, b.max_n)[0] == k
    finally:
        for c in range(3):
            reset(c, precision, b.max_n)
        lj.set_schedule(lj.SCHED_EVAL, precision, b.max_n, *lj.eval_shape_default(b.max_n))


@pytest.mark.parametrize("shape", [2, 3, 6, 7])
def test_packed_degenerate_clusters(shape):
    """Packed teams with coincident atoms (non-finite energy, which also takes
    the evaluation's IEEE-division repeat), an empty and a one-atom cluster
    and a far-apart pair, beside ordinary ones: every output equals the
    oracle's bit for bit (FP64), and the mixed statuses match."""
    sizes = [5, 0, 1, 2, 13, 16, 3, 9, 11]
    off, x = random_starts(sizes, 8601)
    x = x.copy()
    x[:, 1] = x[:, 0]                 # cluster 0: atoms 0 and 1 coincide
    o = off[3]
    x[:, o + 1] = x[:, o] + [1e7, 0.0, 0.0]  # cluster 3: a pair 1e7 apart
    b, xd = to_dev(off, x)
    p = lj.lbfgs_params()
    ro = O.minimize(off, x, oracle_params(p))
    try:
        for prec in ("fp64", "mixed"):
            announce(f"packed degenerate clusters shape {shape} {prec}")
            forced(0, prec, b.max_n, shape)
            r = host_dict(lj.minimize(b, xd, p, prec))
            assert r["status"][0] == lj.NONFINITE and r["status"][1] == lj.CONVERGED
            assert r["energy"][1] == 0.0 and r["energy"][2] == 0.0 and r["iters"][2] == 0
            if prec == "fp64":
                for key in KEYS:
                    assert np.array_equal(r[key], ro[key], equal_nan=True), key
            else:
                assert np.array_equal(r["status"], ro["status"])
    finally:
        reset(0, "fp64", b.max_n)
        reset(0, "mixed", b.max_n)


def test_packed_candidates_in_mixed_bh_chains():
    """Mixed LJ13 chains whose candidates run the FP32 phase only (no polish)
    four per wavefront: the oracle's selection, Metropolis and adaptation,
    fed the GPU's candidate energies, take the same decisions; every accepted
    candidate's FP64 polish converges and the current structures are minima
    to oracle ||g|| < 1e-6 with the reported energies."""
    from test_gpu_bh import replay_decisions
    sizes, steps = [13] * 24, 20
    off, b, r, p = start_chains(sizes, 8701)
    bh = lj.bh_params(cands=8, kT=0.8, seed=8701)
    try:
        forced(0, "mixed", 13, 3)
        announce("bh mixed 24 x LJ13 x 8 candidates, four clusters per wavefront")
        bhx = lj.BasinHopping(b, r["xyz"], r["energy"], bh, p, "mixed", trace_steps=steps,
                              trace_candidates=True)
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            bhx.step(steps)
        side.synchronize()
    finally:
        reset(0, "mixed", 13)
    torch.cuda.synchronize()
    tr = {k: (None if v is None else v.cpu().numpy()) for k, v in bhx.trace.items()}
    replay_decisions(tr, r["energy"].cpu().numpy(), bh)
    acc = tr["accepted"] == 1
    assert np.all(tr["polish_status"][acc] == lj.CONVERGED)
    Eo, go = O.energy_grad(off, host(bhx.xyz_cur))
    assert np.array_equal(Eo, host(bhx.e_cur))
    gn = np.sqrt(np.add.reduceat((go * go).sum(axis=0), off[:-1]))
    assert np.all(gn < 1e-6)


def test_default_rule_two_waves_per_simd_fp64_bitwise():
    """A one-class batch of more clusters than SIMDs: the built-in rule runs
    class 0 two wavefronts per SIMD; every FP64 output equals the oracle's."""
    sizes = list(uniform_sizes(1100, 30, 40, 8801))
    off, x = random_starts(sizes, 8802)
    b, xd = to_dev(off, x)
    p = lj.lbfgs_params()
    announce(f"default rule fp64 {b.num} clusters N 30..40")
    r = host_dict(lj.minimize(b, xd, p, "fp64"))
    ro = O.minimize(off, x, oracle_params(p))
    for key in KEYS:
        assert np.array_equal(r[key], ro[key]), key
