"""GPU parity of lj_energy_grad_batch (Eq. 1 and its gradient) against the oracle.

FP64: bit-identical energies and gradients on every launch shape (the kernel
follows the oracle's summation order).  Mixed: FP32 pair arithmetic on the
FP32-rounded coordinates; the error against the oracle evaluated at those same
coordinates is bounded by 128 u32 times the sums of absolute pair terms (a
standard a-priori bound: about 50 u32 for the pair arithmetic, including the
1-ulp v_rcp_f32, plus 64 u32 for FP32 accumulation over a 64-partner tile).
"""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_util import U32, announce, host, to_dev
from oracle import oracle as O
from paper_2510_25938_amd import lj
from paper_2510_25938_amd.inputs import random_starts

pytestmark = pytest.mark.gpu

# max_n of each batch selects a different launch shape (W waves x A atoms per lane)
SHAPES = {
    "w1": [0, 1, 2, 3, 13, 38, 63, 64],
    "w2": [65, 5, 100, 128],
    "w4": [129, 150, 200, 256],
    "w8": [257, 300, 512],
    "w16": [513, 1000, 1024],
    "w16a2": [1025, 2048],
    "w16a4": [2049, 4096],
}


@pytest.mark.parametrize("shape", list(SHAPES))
def test_fp64_bitwise(shape):
    sizes = SHAPES[shape]
    off, x = random_starts(sizes, 100 + len(shape))
    announce(f"eval fp64 shape={shape} sizes={sizes}")
    b, xd = to_dev(off, x)
    E, g = lj.energy_grad(b, xd, "fp64")
    Eo, go = O.energy_grad(off, x)
    assert np.array_equal(host(E), Eo)
    assert np.array_equal(host(g), go)


@pytest.mark.parametrize("shape", ["w1", "w2", "w4", "w16"])
def test_mixed_error_bound(shape):
    sizes = SHAPES[shape]
    off, x = random_starts(sizes, 200 + len(shape))
    xf = x.astype(np.float32).astype(np.float64)  # the mixed path's coordinates
    announce(f"eval mixed shape={shape} sizes={sizes}")
    b, xd = to_dev(off, x)
    E, g = lj.energy_grad(b, xd, "mixed")
    Eo, go = O.energy_grad(off, xf)
    eabs, gabs = O.abs_sums(off, xf)
    E, g = host(E), host(g)
    assert np.all(np.abs(E - Eo) <= 128 * U32 * eabs + 1e-300)
    assert np.all(np.abs(g - go) <= 128 * U32 * gabs + 1e-300)


def test_energy_only_and_ragged_empty():
    off, x = random_starts([0, 7, 0, 40, 1], 5)
    announce("eval energy-only ragged")
    b, xd = to_dev(off, x)
    E, g = lj.energy_grad(b, xd, "fp64", grad=False)
    assert g is None
    Eo, _ = O.energy_grad(off, x)
    assert np.array_equal(host(E), Eo)


def test_coincident_atoms_nonfinite():
    x = np.zeros((3, 4))
    x[0, 2], x[0, 3] = 1.0, 2.0  # atoms 0 and 1 coincide
    off = np.array([0, 4], np.int32)
    announce("eval coincident atoms")
    b, xd = to_dev(off, x)
    for prec in ("fp64", "mixed"):
        E, _ = lj.energy_grad(b, xd, prec)
        assert not np.isfinite(host(E)[0])


EXTREME = {"coincident": 0.0, "1e-120": 1e-120, "1e-160": 1e-160, "1e154": 1e154,
           "1e200": 1e200}


def test_fp64_extreme_distances_bitwise():
    """Pair distances outside the range where the FP64 loop's 1/r2 skips the
    general division's scaling and fix-up (r2 < 2^-767: coincident, 1e-120,
    a subnormal r2; r2 >= 2^1022: 1e154, and an r2 that overflows to inf).
    Energies and gradients, NaN and signed infinities included, equal the
    oracle's IEEE results: a non-finite energy triggers the recomputation with
    the full division, and above the range both forms give zero pair terms."""
    xs = []
    for d in EXTREME.values():
        c = np.zeros((3, 4))
        c[0] = [0.0, d, 2.0, 3.5]
        c[1] = [0.0, 0.0, 0.3, -0.2]
        xs.append(c)
    off = np.arange(0, 4 * len(xs) + 1, 4).astype(np.int32)
    x = np.concatenate(xs, axis=1)
    announce(f"eval fp64 extreme distances {list(EXTREME)}")
    b, xd = to_dev(off, x)
    E, g = lj.energy_grad(b, xd, "fp64")
    Eo, go = O.energy_grad(off, x)
    assert np.array_equal(host(E), Eo, equal_nan=True)
    assert np.array_equal(host(g), go, equal_nan=True)
    r = {k: v.cpu().numpy() for k, v in lj.minimize(b, xd, lj.lbfgs_params(), "fp64").items()
         if v is not None}
    ro = O.minimize(off, x)
    for k in ("energy", "gnorm", "iters", "evals", "status"):
        assert np.array_equal(r[k], ro[k], equal_nan=True), k


def test_offsets_above_max_n_are_rejected_per_cluster():
    off, x = random_starts([10, 70, 10], 6)
    announce("eval offsets above max_n")
    b, xd = to_dev(off, x)
    E = torch.empty(3, dtype=torch.float64, device="cuda")
    desc = b.desc(max_n=64)  # lies: cluster 1 has 70 atoms
    st = lj.lib().lj_energy_grad_batch(C.byref(desc), C.c_void_p(xd.data_ptr()),
                                       C.c_void_p(E.data_ptr()), None, lj.FP64,
                                       C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == lj.OK
    E = host(E)
    Eo, _ = O.energy_grad(off, x)
    assert np.isnan(E[1]) and E[0] == Eo[0] and E[2] == Eo[2]


def test_deterministic_repeat():
    off, x = random_starts([1000] * 4 + [13] * 8, 8)
    announce("eval determinism")
    b, xd = to_dev(off, x)
    for prec in ("fp64", "mixed"):
        E1, g1 = lj.energy_grad(b, xd, prec)
        E2, g2 = lj.energy_grad(b, xd, prec)
        assert torch.equal(E1, E2) and torch.equal(g1, g2)


@pytest.mark.parametrize("sizes", [[1000, 700, 13], [200, 150], [1500, 900]])
def test_every_schedule_gives_identical_fp64(sizes):
    """FP64 results do not depend on the workgroup shape (fixed summation order)."""
    off, x = random_starts(sizes, 300 + sizes[0])
    b, xd = to_dev(off, x)
    Eo, go = O.energy_grad(off, x)
    p2 = 1
    while p2 < b.max_n:
        p2 *= 2
    shapes = [(w, a) for w in (1, 2, 4, 8, 16) for a in (1, 2, 4)
              if b.max_n <= 64 * w * a <= 2 * max(64, p2)]
    assert len(shapes) >= 2
    try:
        for w, a in shapes:
            announce(f"eval schedule W={w} A={a} sizes={sizes}")
            lj.set_schedule(lj.SCHED_EVAL, "fp64", b.max_n, w, a)
            E, g = lj.energy_grad(b, xd, "fp64")
            assert np.array_equal(host(E), Eo) and np.array_equal(host(g), go), (w, a)
    finally:
        lj.set_schedule(lj.SCHED_EVAL, "fp64", b.max_n, *lj.eval_shape_default(b.max_n))


def test_autotune_installs_a_valid_schedule(tmp_path):
    off, x = random_starts([1000] * 64, 77)
    b, xd = to_dev(off, x)
    announce("autotune 64 x LJ1000 mixed")
    res = lj.autotune(b, xd, "mixed", cache=str(tmp_path / "sched.json"))
    w, a, ms = res["eval"]
    assert 64 * w * a >= 1000 and ms > 0
    assert res["min_large"] in (0, 1, 2) and res["min_ms"] > 0
    E, g = lj.energy_grad(b, xd, "mixed")
    Eo, go = O.energy_grad(off, x.astype(np.float32).astype(np.float64))
    eabs, gabs = O.abs_sums(off, x.astype(np.float32).astype(np.float64))
    assert np.all(np.abs(host(E) - Eo) <= 128 * U32 * eabs)
    lj.load_schedules(str(tmp_path / "sched.json"))
    assert lj.get_schedule(lj.SCHED_EVAL, "mixed", 1000)[:2] == (w, a)
    # the tuned minimiser shape gives the same FP64 result as the default one
    p = lj.lbfgs_params(max_iter=20)
    sub_off, sub_x = random_starts([300, 500], 78)
    bs, xs = to_dev(sub_off, sub_x)
    ref = None
    for k in range(3):
        lj.set_schedule(lj.SCHED_MIN_LARGE, "fp64", 0, k)
        r = lj.minimize(bs, xs, p, "fp64")
        r = {kk: host(v) for kk, v in r.items() if v is not None}
        if ref is None:
            ref = r
        for kk in ("xyz", "energy", "iters", "evals", "status"):
            assert np.array_equal(r[kk], ref[kk]), (k, kk)
    # restore the built-in schedules for the tests that follow
    lj.set_schedule(lj.SCHED_MIN_LARGE, "fp64", 0, 1)
    lj.set_schedule(lj.SCHED_MIN_LARGE, "mixed", 0, 0)
    lj.set_schedule(lj.SCHED_EVAL, "mixed", 1000, *lj.eval_shape_default(1000))


RING_SIZES = list(range(0, 65))  # ring n = 20 .. 43; ordered below, 64-atom tile above


@pytest.mark.parametrize("sizes", [RING_SIZES[:33], RING_SIZES[33:]])
def test_mixed_ring_across_sizes(sizes):
    """The one-wavefront unique-pair FP32 ring (20 <= N <= 43, replicas in the
    lanes above N, a rotated reaction register) and its neighbours (the ordered
    loop below, the 64-atom tile above) for every N up to 64: within the
    a-priori bound, and Newton's third law to the FP32 accumulation bound."""
    off, x = random_starts(sizes, 940 + len(sizes))
    xf = x.astype(np.float32).astype(np.float64)
    announce(f"eval mixed ring sizes={sizes[0]}..{sizes[-1]}")
    b, xd = to_dev(off, x)
    E, g = lj.energy_grad(b, xd, "mixed")
    E, g = host(E), host(g)
    Eo, go = O.energy_grad(off, xf)
    eabs, gabs = O.abs_sums(off, xf)
    assert np.all(np.abs(E - Eo) <= 128 * U32 * eabs)
    assert np.all(np.abs(g - go) <= 128 * U32 * gabs + 1e-300)
    for k in range(len(sizes)):
        a, z = off[k], off[k + 1]
        net = np.abs(g[:, a:z].sum(axis=1))
        assert np.all(net <= 128 * U32 * gabs[:, a:z].sum(axis=1))


TILE_SIZES = [32, 33, 63, 64, 65, 96, 127, 128, 129, 191, 192, 193, 255, 256, 257, 320, 383,
              448, 511, 512, 513, 640, 767, 896, 1023, 1024, 1025, 1088]


@pytest.mark.parametrize("sizes", [TILE_SIZES[:9], TILE_SIZES[9:18], TILE_SIZES[18:]])
def test_mixed_tiles_across_tile_counts(sizes):
    """The unique-pair FP32 loop (N > 32) for 1 .. 17 tiles of 64 atoms: odd and
    even tile counts (half rounds), partial last tiles, every launch shape the
    batch selects; within the a-priori bound, and Newton's third law holds to
    the FP32 accumulation bound (sum_i g_i = 0)."""
    off, x = random_starts(sizes, 950 + len(sizes))
    xf = x.astype(np.float32).astype(np.float64)
    announce(f"eval mixed tiles sizes={sizes}")
    b, xd = to_dev(off, x)
    E, g = lj.energy_grad(b, xd, "mixed")
    E, g = host(E), host(g)
    Eo, go = O.energy_grad(off, xf)
    eabs, gabs = O.abs_sums(off, xf)
    assert np.all(np.abs(E - Eo) <= 128 * U32 * eabs)
    assert np.all(np.abs(g - go) <= 128 * U32 * gabs + 1e-300)
    for k in range(len(sizes)):
        a, z = off[k], off[k + 1]
        net = np.abs(g[:, a:z].sum(axis=1))
        assert np.all(net <= 128 * U32 * gabs[:, a:z].sum(axis=1))


def test_cluster_above_max_n_that_fits_the_launch_shape_is_evaluated():
    """The evaluation launch is shaped for the descriptor's max_n: a larger
    cluster that still fits that shape is evaluated as usual, one that does
    not gets a NaN energy."""
    sizes = [100, 30, 0, 0, 0, 0, 0]
    off, x = random_starts(sizes, 55)
    b, xd = to_dev(off, x)
    desc = b.desc(max_n=20)  # total 130 <= 7 * 20 passes the host check
    w, a = lj.get_schedule(lj.SCHED_EVAL, "fp64", 20)
    assert 30 <= 64 * w * a < 100  # the shape for 20 atoms holds the 30, not the 100
    E = torch.full((len(sizes),), 7.0, dtype=torch.float64, device=xd.device)
    g = torch.zeros_like(xd)
    announce("eval bad size fp64")
    rc = lj.lib().lj_energy_grad_batch(C.byref(desc), xd.data_ptr(), E.data_ptr(), g.data_ptr(),
                                       lj.FP64, None)
    assert rc == lj.OK
    torch.cuda.synchronize()
    Eh, gh = E.cpu().numpy(), g.cpu().numpy()
    Eo, go = O.energy_grad(off, x)
    assert np.isnan(Eh[0])
    assert Eh[1] == Eo[1] and np.array_equal(gh[:, 100:130], go[:, 100:130])
    assert np.all(Eh[2:] == 0.0)
