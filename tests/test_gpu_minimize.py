"""GPU parity of lj_bh_minimize_batch against the oracle's L-BFGS.

FP64 path: every output (coordinates, energy, gradient norm, iteration and
evaluation counts, status) is bit-identical to the oracle, for every size
class of the persistent launch.  Mixed path: the FP64 polish started at the
GPU's recorded switch point reproduces the oracle run from that point bit for
bit, and every converged result is a minimum to ||g|| < 1e-6 by the oracle's
own gradient.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_util import announce, host_dict, to_dev
from oracle import oracle as O
from paper_2510_25938_amd import lj
from paper_2510_25938_amd.inputs import random_starts

pytestmark = pytest.mark.gpu

KEYS = ("xyz", "energy", "gnorm", "iters", "evals", "status")


def oracle_params(p):
    return O.lbfgs_params(m=p.m, gtol=p.gtol, max_iter=p.max_iter, max_step=p.max_step, c1=p.c1,
                          max_ls=p.max_ls, curv_eps=p.curv_eps)


def assert_same(r, ro, idx=None):
    for k in KEYS:
        a, b = r[k], ro[k]
        if idx is not None and k != "xyz":
            a = a[idx]
        assert np.array_equal(a, b), k


CLASS_SIZES = {
    "c0": [0, 1, 2, 3, 4, 13, 38, 55, 64],
    "c1": [65, 13, 80, 128],
    "c2": [129, 150, 38, 256],
    "c3": [257, 13, 300, 400],
}


@pytest.mark.parametrize("cls", list(CLASS_SIZES))
def test_fp64_bitwise_per_class(cls):
    sizes = CLASS_SIZES[cls]
    off, x = random_starts(sizes, 300 + int(cls[1]))
    p = lj.lbfgs_params()
    announce(f"minimize fp64 class={cls} sizes={sizes}")
    b, xd = to_dev(off, x)
    r = host_dict(lj.minimize(b, xd, p, "fp64"))
    ro = O.minimize(off, x, oracle_params(p))
    assert_same(r, ro)
    assert np.all(r["status"] == lj.CONVERGED)


NARROW = {
    # class 0 with at most 16 atoms: reductions over one 16-lane row
    "c0_16": (list(range(0, 17)) + [13] * 24, 17),
    # class 2 with at most 192 atoms: three wavefronts (three 64-atom tiles)
    "c2_192": ([129, 150, 192, 13, 100, 160, 129, 185], 193),
    # class 1 alone: two wavefronts; with a larger cluster in the batch (the
    # extra one), one wavefront with two atoms per lane
    "c1_beside": ([65, 100, 128, 80, 13, 127, 96, 70], 129),
}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", list(NARROW))
def test_narrow_class_kernels(case, prec):
    """When max_n keeps a size class in the lower part of its range, a leaner
    kernel serves it (16-lane reductions for N <= 16; three wavefronts for
    129 <= N <= 192), and when larger clusters share the batch the 65-128-atom
    class runs one wavefront with two atoms per lane.  The same clusters in a
    batch with one more cluster run the other kernels: every output is
    bit-identical between the two (on the mixed path the 65-128-atom kernels
    sum FP32 pair terms in different orders, so there each polish must equal
    the oracle's from its switch points), and the FP64 path is bit-identical
    to the oracle."""
    sizes, extra = NARROW[case]
    off, x = random_starts(sizes, 4242)
    p = lj.lbfgs_params()
    announce(f"minimize {prec} narrow {case} sizes={sizes[:12]}... extra={extra}")
    b, xd = to_dev(off, x)
    sw = prec == "mixed"
    r = host_dict(lj.minimize(b, xd, p, prec, switch_point=sw))
    off2, x2 = random_starts(sizes + [extra], 4242)
    assert np.array_equal(x2[:, :off[-1]], x)  # the same starts, one more cluster
    b2, xd2 = to_dev(off2, x2)
    r2 = host_dict(lj.minimize(b2, xd2, p, prec, switch_point=sw))
    n = len(sizes)
    if prec == "mixed" and case == "c1_beside":
        # the one-wavefront kernel sums FP32 pair terms in the ordered loop,
        # the two-wavefront one on tiles: each run's polish must reproduce
        # the oracle from its own switch points
        mixed_checks(off, x, r, p)
        mixed_checks(off2, x2, r2, p)
        return
    for k in KEYS:
        a2 = r2[k][:, :off[-1]] if k == "xyz" else r2[k][:n]
        assert np.array_equal(r[k], a2), k
    if prec == "fp64":
        assert_same(r, O.minimize(off, x, oracle_params(p)))
    assert np.all(r["status"] == lj.CONVERGED)


def test_fp64_iteration_cap_large_cluster():
    off, x = random_starts([1000, 600], 31)
    p = lj.lbfgs_params(max_iter=25)
    announce("minimize fp64 N=1000 cap 25")
    b, xd = to_dev(off, x)
    r = host_dict(lj.minimize(b, xd, p, "fp64"))
    ro = O.minimize(off, x, oracle_params(p))
    assert_same(r, ro)
    assert np.all(r["status"] == lj.MAXITER)


def test_fp64_history_sizes_and_params():
    off, x = random_starts([38, 20], 32)
    for kw in (dict(m=0), dict(m=1), dict(m=3), dict(max_step=0.05, c1=0.3), dict(max_ls=2)):
        p = lj.lbfgs_params(**kw)
        announce(f"minimize fp64 params={kw}")
        b, xd = to_dev(off, x)
        r = host_dict(lj.minimize(b, xd, p, "fp64"))
        ro = O.minimize(off, x, oracle_params(p))
        assert_same(r, ro)


def test_fp64_schedule_independence():
    """A cluster's result does not depend on its batch: bitwise equal when run
    alone, inside a large batch, and inside a batch of other size classes."""
    off, x = random_starts([38] * 64 + [150] * 8 + [13] * 40, 33)
    p = lj.lbfgs_params()
    announce("minimize fp64 schedule independence")
    b, xd = to_dev(off, x)
    r = host_dict(lj.minimize(b, xd, p, "fp64"))
    for k in (0, 64, 70, 100):
        o0, o1 = off[k], off[k + 1]
        sub_off = np.array([0, o1 - o0], np.int32)
        bs, xs = to_dev(sub_off, np.ascontiguousarray(x[:, o0:o1]))
        rs = host_dict(lj.minimize(bs, xs, p, "fp64"))
        assert np.array_equal(rs["xyz"], r["xyz"][:, o0:o1])
        for key in KEYS[1:]:
            assert rs[key][0] == r[key][k]


def test_degenerate_inputs():
    x = np.zeros((3, 5))
    x[0] = [0.0, 0.0, 1.0, 2.0, 3.0]  # atoms 0 and 1 coincide
    off = np.array([0, 5, 5, 6], np.int32)  # plus an empty and a 1-atom cluster
    x = np.concatenate([x, np.zeros((3, 1))], axis=1)
    announce("minimize degenerate inputs")
    b, xd = to_dev(off, x)
    for prec in ("fp64", "mixed"):
        r = host_dict(lj.minimize(b, xd, lj.lbfgs_params(), prec))
        assert list(r["status"]) == [lj.NONFINITE, lj.CONVERGED, lj.CONVERGED]
        assert r["energy"][1] == 0.0 and r["energy"][2] == 0.0 and r["iters"][1] == 0


def mixed_checks(off, x, r, p):
    """P2: the oracle's FP64 run from the switch point equals the GPU polish."""
    ro = O.minimize(off, r["xyz_switch"], oracle_params(p))
    assert np.array_equal(r["xyz"], ro["xyz"])
    assert np.array_equal(r["energy"], ro["energy"])
    assert np.array_equal(r["gnorm"], ro["gnorm"])
    assert np.array_equal(r["status"], ro["status"])
    Ef, gf = O.energy_grad(off, r["xyz"])
    assert np.array_equal(Ef, r["energy"])
    conv = r["status"] == lj.CONVERGED
    for bidx in np.nonzero(conv)[0]:
        gb = gf[:, off[bidx]:off[bidx + 1]]
        assert np.sqrt(np.sum(gb * gb)) < 1e-6
    return ro


@pytest.mark.parametrize("sizes", [[13] * 16 + [38] * 16, [65, 100, 128, 129, 150, 200], [300, 257]])
def test_mixed_polish_reproduces_oracle_from_switch_point(sizes):
    off, x = random_starts(sizes, 400 + len(sizes))
    p = lj.lbfgs_params()
    announce(f"minimize mixed+polish sizes={sizes}")
    b, xd = to_dev(off, x)
    r = host_dict(lj.minimize(b, xd, p, "mixed", switch_point=True))
    mixed_checks(off, x, r, p)
    assert np.mean(r["status"] == lj.CONVERGED) >= 0.9


def test_mixed_without_polish_reports_fp64_energy():
    off, x = random_starts([300, 40], 41)
    p = lj.lbfgs_params(polish=0, max_iter=60)
    announce("minimize mixed no-polish")
    b, xd = to_dev(off, x)
    r = host_dict(lj.minimize(b, xd, p, "mixed"))
    Eo, go = O.energy_grad(off, r["xyz"])
    assert np.array_equal(r["energy"], Eo)
    for k in range(2):
        gb = go[:, off[k]:off[k + 1]]
        assert r["gnorm"][k] == np.sqrt(O.tree_sum(np.sum(gb * gb, axis=0))) or \
            abs(r["gnorm"][k] - np.sqrt(np.sum(gb * gb))) <= 1e-12 * r["gnorm"][k]
    assert set(r["status"]) <= {lj.MAXITER, lj.SWITCHED, lj.CONVERGED}


def test_mixed_deterministic():
    off, x = random_starts([38] * 32 + [100] * 4, 42)
    announce("minimize mixed determinism")
    b, xd = to_dev(off, x)
    r1 = host_dict(lj.minimize(b, xd, lj.lbfgs_params(), "mixed"))
    r2 = host_dict(lj.minimize(b, xd, lj.lbfgs_params(), "mixed"))
    for k in KEYS:
        assert np.array_equal(r1[k], r2[k])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_short_workspace_is_rejected_before_any_work(prec):
    """A missing or one-byte-short workspace returns LJ_E_WORKSPACE and
    enqueues nothing: coordinates and outputs keep their values."""
    off, x = random_starts([13, 38, 80], 41)
    b, xd = to_dev(off, x)
    p = lj.lbfgs_params()
    nb = lj.minimize_workspace_bytes(b, p, prec)
    assert nb > 0
    announce(f"short workspace minimize prec={prec} need={nb}")
    x0 = xd.clone()
    for size in (nb - 1, 1):
        ws = torch.empty(size, dtype=torch.uint8, device=xd.device)
        with pytest.raises(lj.LJError) as err:
            lj.minimize(b, xd, p, prec, workspace=ws, inplace=True)
        assert err.value.args[1] == lj.E_WORKSPACE
    e = torch.full((b.num,), 7.0, dtype=torch.float64, device=xd.device)
    i = torch.full((b.num,), -5, dtype=torch.int32, device=xd.device)
    st = lj.lib().lj_bh_minimize_batch(C.byref(b.desc()), xd.data_ptr(), e.data_ptr(),
                                       e.data_ptr(), i.data_ptr(), i.data_ptr(), i.data_ptr(),
                                       None, C.byref(p), lj.precision_code(prec), None, nb, None)
    assert st == lj.E_WORKSPACE
    torch.cuda.synchronize()
    assert torch.equal(xd, x0)
    assert torch.all(e == 7.0) and torch.all(i == -5)
    # the exact size is accepted and gives the default path's result
    ws = torch.empty(nb, dtype=torch.uint8, device=xd.device)
    r = host_dict(lj.minimize(b, xd, p, prec, workspace=ws))
    ref = host_dict(lj.minimize(b, xd, p, prec))
    for k in KEYS:
        assert np.array_equal(r[k], ref[k]), k


def test_autotune_short_workspace_is_rejected():
    off, x = random_starts([300, 400], 43)
    b, xd = to_dev(off, x)
    L = lj.lib()
    nb = int(L.lj_autotune_workspace_bytes(C.byref(b.desc()), lj.MIXED))
    assert nb > 0
    announce(f"short workspace autotune need={nb}")
    ws = torch.empty(nb - 1, dtype=torch.uint8, device=xd.device)
    t0, t1 = C.c_float(-2.0), C.c_float(-2.0)
    st = L.lj_autotune(C.byref(b.desc()), xd.data_ptr(), lj.MIXED, ws.data_ptr(), nb - 1, None,
                       C.byref(t0), C.byref(t1))
    assert st == lj.E_WORKSPACE and t0.value == -2.0 and t1.value == -2.0


def test_largest_supported_cluster():
    """A cluster of LJ_MAX_ATOMS_MIN atoms beside small ones: FP64 bit-identical
    to the oracle over a capped run; without polish the mixed path reports the
    oracle's FP64 energy at the coordinates it returns."""
    off, x = random_starts([lj.MAX_ATOMS_MIN, 1, 13], 51)
    b, xd = to_dev(off, x)
    p = lj.lbfgs_params(max_iter=8)
    announce(f"minimize fp64 N={lj.MAX_ATOMS_MIN} cap 8")
    r = host_dict(lj.minimize(b, xd, p, "fp64"))
    assert_same(r, O.minimize(off, x, oracle_params(p)))
    announce(f"minimize mixed N={lj.MAX_ATOMS_MIN} cap 8 no polish")
    rm = host_dict(lj.minimize(b, xd, lj.lbfgs_params(max_iter=8, polish=0), "mixed"))
    Eo, _ = O.energy_grad(off, rm["xyz"])
    assert np.array_equal(rm["energy"], Eo)


def test_cluster_above_max_n_is_flagged_and_left_alone():
    """A cluster larger than the descriptor's max_n gets LJ_BADSIZE and keeps
    its coordinates; the other clusters are minimised as usual."""
    sizes = [13, 30, 2]
    off, x = random_starts(sizes, 53)
    b, xd = to_dev(off, x)
    p = lj.lbfgs_params()
    desc = b.desc(max_n=20)  # 30 > 20; total 45 <= 3 * 20 passes the host check
    dev = xd.device
    sub_off = np.array([0, 13, 15], np.int32)
    sub_x = np.ascontiguousarray(np.concatenate([x[:, 0:13], x[:, 43:45]], axis=1))
    ro = O.minimize(sub_off, sub_x, oracle_params(p))
    for prec in (lj.FP64, lj.MIXED):
        announce(f"minimize bad size prec={prec}")
        xw = xd.clone()
        e = torch.full((3,), 7.0, dtype=torch.float64, device=dev)
        gn = e.clone()
        it = torch.full((3,), -5, dtype=torch.int32, device=dev)
        ev, st = it.clone(), it.clone()
        nb = int(lj.lib().lj_minimize_workspace_bytes(C.byref(desc), C.byref(p), prec))
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        rc = lj.lib().lj_bh_minimize_batch(C.byref(desc), xw.data_ptr(), e.data_ptr(),
                                           gn.data_ptr(), it.data_ptr(), ev.data_ptr(),
                                           st.data_ptr(), None, C.byref(p), prec, ws.data_ptr(),
                                           nb, None)
        assert rc == lj.OK
        torch.cuda.synchronize()
        status = st.cpu().numpy()
        assert list(status) == [lj.CONVERGED, lj.BADSIZE, lj.CONVERGED]
        assert torch.equal(xw[:, 13:43], xd[:, 13:43])
        if prec == lj.FP64:
            xo = xw.cpu().numpy()
            assert np.array_equal(xo[:, 0:13], ro["xyz"][:, 0:13])
            assert np.array_equal(xo[:, 43:45], ro["xyz"][:, 13:15])
            assert np.array_equal(e.cpu().numpy()[[0, 2]], ro["energy"])


def test_many_caller_streams():
    """Calls on many caller streams: the first ones get side streams for their
    size classes, later ones run the classes in turn on the caller's stream.
    FP64 results are the same on every stream."""
    off, x = random_starts([13, 80, 150, 38], 57)
    b, xd = to_dev(off, x)
    p = lj.lbfgs_params(max_iter=40)
    ref = host_dict(lj.minimize(b, xd, p, "fp64"))
    streams = [torch.cuda.Stream() for _ in range(20)]
    announce("minimize fp64 on 20 caller streams")
    outs = []
    for s in streams:
        with torch.cuda.stream(s):
            outs.append(lj.minimize(b, xd, p, "fp64", stream=s))
    torch.cuda.synchronize()
    for o in outs:
        assert_same(host_dict(o), ref)


def test_fp64_class1_kernel_follows_batch_size():
    """FP64 batches of 65-128-atom clusters with at least one cluster per SIMD
    run the one-wavefront two-slot kernel, smaller ones two wavefronts: the
    clusters they share give bit-identical outputs."""
    simds = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    sizes = [65 + (k * 37) % 64 for k in range(simds)]
    off, x = random_starts(sizes, 59)
    p = lj.lbfgs_params(max_iter=60)
    announce(f"minimize fp64 class 1: {simds} clusters vs {simds - 1}")
    b, xd = to_dev(off, x)
    big = host_dict(lj.minimize(b, xd, p, "fp64"))
    off2 = off[:simds]  # one cluster fewer
    b2, xd2 = to_dev(off2, np.ascontiguousarray(x[:, :off2[-1]]))
    small = host_dict(lj.minimize(b2, xd2, p, "fp64"))
    for k in KEYS:
        a = big[k][:, :off2[-1]] if k == "xyz" else big[k][:simds - 1]
        assert np.array_equal(a, small[k]), k
