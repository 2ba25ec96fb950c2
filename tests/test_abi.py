"""CPU checks of the C ABI: the library loads, exports every symbol declared in
include/lj_bh.h, and rejects bad arguments on the host before touching a device."""
import ctypes as C
import os
import re

import pytest

from paper_2510_25938_amd import lj

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lj_bh.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lj_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_surface():
    assert declared_functions() == sorted(lj.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = lj.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_status_strings_and_version():
    L = lj.lib()
    assert L.lj_abi_version() == 4
    assert L.lj_status_string(lj.OK) == b"LJ_OK"
    for s in (lj.E_ARG, lj.E_HIP, lj.E_WORKSPACE, lj.E_UNSUPPORTED):
        assert L.lj_status_string(s).startswith(b"LJ_E_")


def test_pair_selection_is_validated_on_the_host():
    L = lj.lib()
    # int32, ptr, int32, int64, int32, double, double, double (natural alignment)
    assert C.sizeof(lj.Batch) == 64
    for pair, rho in ((2, 6.0), (-1, 6.0), (lj.PAIRS["morse"], 0.0), (lj.PAIRS["morse"], -3.0),
                      (lj.PAIRS["morse"], float("nan")), (lj.PAIRS["morse"], float("inf"))):
        b = lj.Batch(2, 16, 13, 26, pair, rho)
        assert L.lj_energy_grad_batch(C.byref(b), 16, 16, None, lj.FP64, None) == lj.E_ARG
        assert b"pair" in L.lj_last_error()
        p = lj.lbfgs_params()
        assert (L.lj_bh_minimize_batch(C.byref(b), None, None, None, None, None, None, None,
                                       C.byref(p), lj.FP64, None, 0, None) == lj.E_ARG)
    with pytest.raises(ValueError):
        lj.ClusterBatch([0, 3], device="cpu", pair="buckingham")


def test_units_are_validated_on_the_host():
    L = lj.lib()
    p = lj.lbfgs_params()
    for sg, ep in ((-1.0, 1.0), (1.0, -2.0), (float("nan"), 1.0), (1.0, float("inf"))):
        b = lj.Batch(2, 16, 13, 26, 0, 0.0, sg, ep)
        assert L.lj_energy_grad_batch(C.byref(b), 16, 16, None, lj.FP64, None) == lj.E_ARG
        assert b"sigma" in L.lj_last_error()
    # basin hopping runs in reduced units only
    b = lj.Batch(2, 16, 13, 26, 0, 0.0, 2.0, 1.0)
    bh = lj.bh_params()
    assert L.lj_bh_workspace_bytes(C.byref(b), C.byref(bh), C.byref(p), lj.FP64) == 0
    st = lj.BhState(*([16] * 8))
    assert (L.lj_bh_step(C.byref(b), C.byref(st), C.byref(bh), C.byref(p), lj.FP64, 1, None,
                         16, 1 << 20, None) == lj.E_UNSUPPORTED)
    assert b"reduced units" in L.lj_last_error()


def test_defaults():
    p = lj.lbfgs_params()
    assert (p.m, p.gtol, p.max_iter, p.max_step, p.c1, p.max_ls) == (10, 1e-6, 10000, 0.2, 1e-4, 30)
    assert p.polish == 1 and p.curv_eps == 1e-10


def test_argument_errors_are_host_side():
    L = lj.lib()
    bad = lj.Batch(-1, None, 0, 0)
    assert L.lj_energy_grad_batch(C.byref(bad), None, None, None, lj.FP64, None) == lj.E_ARG
    assert b"num" in L.lj_last_error()
    big = lj.Batch(1, 16, lj.MAX_ATOMS_EVAL + 1, 10)
    assert L.lj_energy_grad_batch(C.byref(big), None, None, None, lj.FP64, None) == lj.E_UNSUPPORTED
    big = lj.Batch(1, 16, lj.MAX_ATOMS_MIN + 1, 10)
    p = lj.lbfgs_params()
    assert (L.lj_bh_minimize_batch(C.byref(big), None, None, None, None, None, None, None,
                                   C.byref(p), lj.FP64, None, 0, None) == lj.E_UNSUPPORTED)
    ok = lj.Batch(2, 16, 13, 26)
    assert L.lj_energy_grad_batch(C.byref(ok), 16, 16, None, 7, None) == lj.E_ARG
    p.m = 11
    assert (L.lj_bh_minimize_batch(C.byref(ok), None, None, None, None, None, None, None,
                                   C.byref(p), lj.FP64, None, 0, None) == lj.E_ARG)
    p = lj.lbfgs_params(gtol=0.0)
    assert (L.lj_bh_minimize_batch(C.byref(ok), None, None, None, None, None, None, None,
                                   C.byref(p), lj.FP64, None, 0, None) == lj.E_ARG)
    inconsistent = lj.Batch(2, 16, 13, 27)  # total_atoms > num * max_n
    assert L.lj_energy_grad_batch(C.byref(inconsistent), 16, 16, None, 0, None) == lj.E_ARG
    bh = lj.bh_params(cands=lj.MAX_CANDS + 1)
    p = lj.lbfgs_params()
    assert L.lj_bh_workspace_bytes(C.byref(ok), C.byref(bh), C.byref(p), lj.FP64) == 0
    st = lj.BhState()
    bh = lj.bh_params()
    assert (L.lj_bh_step(C.byref(ok), C.byref(st), C.byref(bh), C.byref(p), lj.FP64, 1, None,
                         None, 0, None) == lj.E_ARG)  # NULL state arrays


def test_noalloc_limits_are_host_side():
    L = lj.lib()
    p = lj.lbfgs_params()
    big = lj.Batch(2, 16, lj.NOALLOC_MAX_ATOMS + 1, 2 * lj.NOALLOC_MAX_ATOMS + 2)
    assert (L.lj_bh_minimize_batch_noalloc(C.byref(big), 16, 16, 16, 16, 16, 16, None,
                                           C.byref(p), lj.FP64, None) == lj.E_UNSUPPORTED)
    assert b"use lj_bh_minimize_batch" in L.lj_last_error()
    many = lj.Batch(lj.NOALLOC_MAX_CLUSTERS + 1, 16, 13, 13 * (lj.NOALLOC_MAX_CLUSTERS + 1))
    assert (L.lj_bh_minimize_batch_noalloc(C.byref(many), 16, 16, 16, 16, 16, 16, None,
                                           C.byref(p), lj.MIXED, None) == lj.E_WORKSPACE)
    assert b"static scratch" in L.lj_last_error()
    ok = lj.Batch(2, 16, 13, 26)
    assert (L.lj_bh_minimize_batch_noalloc(C.byref(ok), 16, None, 16, 16, 16, 16, None,
                                           C.byref(p), lj.FP64, None) == lj.E_ARG)
    assert (L.lj_bh_minimize_batch_noalloc(C.byref(ok), 16, 16, 16, 16, 16, 16, None,
                                           C.byref(p), 5, None) == lj.E_ARG)
    empty = lj.Batch(0, None, 0, 0)
    assert (L.lj_bh_minimize_batch_noalloc(C.byref(empty), None, None, None, None, None, None,
                                           None, C.byref(p), lj.FP64, None) == lj.OK)
    # the published limits: the work list of the largest batch plus the
    # size-class table and counters (256-byte aligned) fill the scratch exactly
    assert 4 * lj.NOALLOC_MAX_CLUSTERS + 2 * 256 == lj.NOALLOC_SCRATCH_BYTES


def test_empty_batches_are_no_ops():
    L = lj.lib()
    empty = lj.Batch(0, None, 0, 0)
    p = lj.lbfgs_params()
    assert L.lj_energy_grad_batch(C.byref(empty), None, None, None, lj.FP64, None) == lj.OK
    assert (L.lj_bh_minimize_batch(C.byref(empty), None, None, None, None, None, None, None,
                                   C.byref(p), lj.MIXED, None, 0, None) == lj.OK)


def test_cluster_batch_validation():
    with pytest.raises(ValueError):
        lj.ClusterBatch([1, 2], device="cpu")
    with pytest.raises(ValueError):
        lj.ClusterBatch([0, 5, 3], device="cpu")
    b = lj.ClusterBatch([0, 13, 13, 51], device="cpu")
    assert b.num == 3 and b.max_n == 38 and b.total == 51 and list(b.sizes) == [13, 0, 38]


def test_schedule_table_validation():
    L = lj.lib()
    assert L.lj_set_schedule(lj.SCHED_EVAL, lj.FP64, 1000, 3, 1) == lj.E_ARG  # W = 3
    assert L.lj_set_schedule(lj.SCHED_EVAL, lj.FP64, 1000, 4, 2) == lj.E_ARG  # 512 slots
    assert L.lj_set_schedule(lj.SCHED_MIN_LARGE, lj.MIXED, 0, 3, 0) == lj.E_ARG
    assert L.lj_set_schedule(7, lj.FP64, 10, 1, 1) == lj.E_ARG
    assert lj.get_schedule(lj.SCHED_EVAL, "fp64", 1000) == (16, 1)  # built-in rule
    lj.set_schedule(lj.SCHED_EVAL, "fp64", 1000, 4, 4)
    assert lj.get_schedule(lj.SCHED_EVAL, "fp64", 1000) == (4, 4)
    assert lj.get_schedule(lj.SCHED_EVAL, "fp64", 600) == (4, 4)  # same power-of-two key
    assert lj.get_schedule(lj.SCHED_EVAL, "mixed", 1000) == (16, 1)
    lj.set_schedule(lj.SCHED_EVAL, "fp64", 1000, 16, 1)
    assert lj.get_schedule(lj.SCHED_MIN_LARGE, "mixed")[0] == 0  # default 16 x 1
    assert lj.get_schedule(lj.SCHED_MIN_LARGE, "fp64")[0] == 1  # default 8 x 2
    lj.set_schedule(lj.SCHED_MIN_LARGE, "mixed", 0, 2)
    assert lj.get_schedule(lj.SCHED_MIN_LARGE, "mixed")[0] == 2
    lj.set_schedule(lj.SCHED_MIN_LARGE, "mixed", 0, 0)


def test_class_schedule_validation():
    L = lj.lib()
    c0, c1, c2 = lj.SCHED_MIN_CLASS
    assert lj.get_schedule(c0, "fp64", 13) == (-1, 0)  # no entry: the built-in rule
    assert L.lj_set_schedule(c0, lj.FP64, 40, 3, 0) == lj.E_ARG  # four per wave holds <= 16
    assert b"holds at most 16" in L.lj_last_error()
    assert L.lj_set_schedule(c0, lj.FP64, 40, 7, 0) == lj.E_ARG  # four per wave, 2 per SIMD
    assert L.lj_set_schedule(c0, lj.FP64, 40, 8, 0) == lj.E_ARG  # no shape 8
    assert L.lj_set_schedule(c2, lj.FP64, 100, 0, 0) == lj.E_ARG  # no class-2 clusters
    assert L.lj_set_schedule(c2, lj.FP64, 250, 1, 0) == lj.E_ARG  # three waves hold <= 192
    lj.set_schedule(c0, "fp64", 13, 3)
    assert lj.get_schedule(c0, "fp64", 13) == (3, 4)
    assert lj.get_schedule(c0, "fp64", 9) == (3, 4)  # same power-of-two key
    assert lj.get_schedule(c0, "mixed", 13) == (-1, 0)
    lj.set_schedule(c0, "fp64", 13, 7)
    assert lj.get_schedule(c0, "fp64", 13) == (7, 4)
    lj.set_schedule(c0, "fp64", 13, -1)
    assert lj.get_schedule(c0, "fp64", 13) == (-1, 0)
    lj.set_schedule(c1, "mixed", 150, 1)
    assert lj.get_schedule(c1, "mixed", 150) == (1, 1)
    assert lj.get_schedule(c1, "mixed", 120) == (-1, 0)  # another largest class
    lj.set_schedule(c1, "mixed", 150, -1)
