"""GPU parity of the Morse pair (the pair-potential extension) against the oracle.

FP64: energies, gradients, minimisations and basin-hopping chains are
bit-identical to the oracle (the kernels follow the oracle's summation order,
IEEE sqrt and division, and the same Cody-Waite exp).  Mixed: FP32 pair
arithmetic on the FP32-rounded coordinates, with the error bound derived for
this pair: the relative error of t = exp(rho (1 - r)) from the FP32 square
root, the rounded exponent and the hardware exp2 is at most about
(6 rho r + 2) u32, which the energy t (t - 2) and the force c t (t - 1) / r
at most double; with 64 u32 for the FP32 tile sums the bound is
(12 rho r_max + 128) u32 times the sums of absolute pair terms.  Mixed
minimisations: the FP64 polish from the recorded switch point reproduces the
oracle bit for bit.  Units: sigma / epsilon conversion of the inputs and
outputs.
"""
import numpy as np
import pytest
import torch

from gpu_util import U32, announce, host, host_dict
from oracle import oracle as O
from paper_2510_25938_amd import lj
from paper_2510_25938_amd.inputs import random_starts, uniform_sizes

pytestmark = pytest.mark.gpu

SHAPES = {
    "w1": ([0, 1, 2, 3, 13, 38, 39, 40, 41, 63, 64], 6.0),
    "w2": ([65, 5, 100, 128], 3.0),
    "w4": ([129, 150, 200, 256], 14.0),
    "w8": ([257, 300, 512], 6.0),
    "w16": ([513, 1000], 10.0),
    "w16a2": ([1025, 1500], 6.0),
}


def morse_dev(off, x, rho):
    b = lj.ClusterBatch(off, device="cuda", pair="morse", rho=rho)
    return b, torch.from_numpy(np.ascontiguousarray(x)).cuda()


def oracle_params(p, rho):
    return O.lbfgs_params(m=p.m, gtol=p.gtol, max_iter=p.max_iter, max_step=p.max_step, c1=p.c1,
                          max_ls=p.max_ls, curv_eps=p.curv_eps, pair="morse", rho=rho)


@pytest.mark.parametrize("shape", list(SHAPES))
def test_fp64_bitwise(shape):
    sizes, rho = SHAPES[shape]
    off, x = random_starts(sizes, 600 + len(shape))
    announce(f"morse eval fp64 shape={shape} sizes={sizes} rho={rho}")
    b, xd = morse_dev(off, x, rho)
    E, g = lj.energy_grad(b, xd, "fp64")
    Eo, go = O.energy_grad(off, x, "morse", rho)
    assert np.array_equal(host(E), Eo)
    assert np.array_equal(host(g), go)


@pytest.mark.parametrize("shape", ["w1", "w2", "w4", "w16"])
def test_mixed_error_bound(shape):
    sizes, rho = SHAPES[shape]
    off, x = random_starts(sizes, 700 + len(shape))
    xf = x.astype(np.float32).astype(np.float64)
    announce(f"morse eval mixed shape={shape} sizes={sizes} rho={rho}")
    b, xd = morse_dev(off, x, rho)
    E, g = lj.energy_grad(b, xd, "mixed")
    E, g = host(E), host(g)
    Eo, go = O.energy_grad(off, xf, "morse", rho)
    eabs, gabs = O.abs_sums(off, xf, "morse", rho)
    for k in range(len(sizes)):
        a, z = off[k], off[k + 1]
        if z - a < 2:
            assert E[k] == 0.0 and np.all(g[:, a:z] == 0.0)
            continue
        span = np.ptp(xf[:, a:z], axis=1)
        c = (12.0 * rho * float(np.linalg.norm(span)) + 128.0) * U32
        assert abs(E[k] - Eo[k]) <= c * eabs[k]
        assert np.all(np.abs(g[:, a:z] - go[:, a:z]) <= c * gabs[:, a:z] + 1e-300)


@pytest.mark.parametrize("lo,hi,rho", [(0, 33, 6.0), (33, 65, 3.0)])
def test_mixed_ring_across_sizes(lo, hi, rho):
    """Every N up to 64 for the Morse pair: the one-wavefront FP32 ring
    (20 <= N <= 43) and the ordered loop around it, within the derived bound;
    Newton's third law to the FP32 accumulation bound."""
    sizes = list(range(lo, hi))
    off, x = random_starts(sizes, 720 + lo)
    xf = x.astype(np.float32).astype(np.float64)
    announce(f"morse eval mixed ring sizes={lo}..{hi - 1} rho={rho}")
    b, xd = morse_dev(off, x, rho)
    E, g = lj.energy_grad(b, xd, "mixed")
    E, g = host(E), host(g)
    Eo, go = O.energy_grad(off, xf, "morse", rho)
    eabs, gabs = O.abs_sums(off, xf, "morse", rho)
    for k in range(len(sizes)):
        a, z = off[k], off[k + 1]
        span = np.ptp(xf[:, a:z], axis=1) if z > a else np.zeros(3)
        c = (12.0 * rho * float(np.linalg.norm(span)) + 128.0) * U32
        assert abs(E[k] - Eo[k]) <= c * eabs[k]
        assert np.all(np.abs(g[:, a:z] - go[:, a:z]) <= c * gabs[:, a:z] + 1e-300)
        assert np.all(np.abs(g[:, a:z].sum(axis=1)) <= c * gabs[:, a:z].sum(axis=1) + 1e-300)


@pytest.mark.parametrize("sizes,rho", [([2, 3, 4, 13, 38, 64], 6.0), ([80, 13, 128], 3.0),
                                       ([150, 200], 10.0), ([300, 13], 6.0),
                                       ([80, 150, 13, 127], 6.0)])
def test_fp64_minimize_bitwise(sizes, rho):
    off, x = random_starts(sizes, 800 + len(sizes))
    p = lj.lbfgs_params()
    announce(f"morse minimize fp64 sizes={sizes} rho={rho}")
    b, xd = morse_dev(off, x, rho)
    r = host_dict(lj.minimize(b, xd, p, "fp64"))
    ro = O.minimize(off, x, oracle_params(p, rho))
    for k in ("xyz", "energy", "gnorm", "iters", "evals", "status"):
        assert np.array_equal(r[k], ro[k]), k
    assert np.all(r["status"] == lj.CONVERGED)
    small = {2: -1.0, 3: -3.0, 4: -6.0}
    for k, n in enumerate(sizes):
        if n in small:
            assert abs(r["energy"][k] - small[n]) < 1e-12


@pytest.mark.parametrize("rho", [6.0, 3.0])
def test_fp64_minimize_every_small_size_bitwise(rho):
    """Every size 0 .. 44 in one batch: the one-wavefront kernel evaluates the
    Morse pair over unique pairs up to 40 atoms (pair matrix in LDS, ordered
    sums) and in the ordered loop above; both match the oracle bit for bit."""
    sizes = list(range(0, 45))
    off, x = random_starts(sizes, 870 + int(rho))
    p = lj.lbfgs_params()
    announce(f"morse minimize fp64 sizes=0..44 rho={rho}")
    b, xd = morse_dev(off, x, rho)
    r = host_dict(lj.minimize(b, xd, p, "fp64"))
    ro = O.minimize(off, x, oracle_params(p, rho))
    for k in ("xyz", "energy", "gnorm", "iters", "evals", "status"):
        assert np.array_equal(r[k], ro[k]), k


@pytest.mark.parametrize("shape", [0, 1])
def test_fp64_degenerate_clusters_unique_pairs(shape):
    """Coincident atoms (a non-finite gradient), empty, one- and two-atom
    clusters and a pair 1e7 apart beside ordinary ones, through the
    one-wavefront kernels that evaluate the Morse pair over unique pairs
    (64-lane and 16-lane reductions): every output equals the oracle's bit for
    bit, NaNs included."""
    sizes = [5, 0, 1, 2, 13, 16, 3, 9, 11]
    off, x = random_starts(sizes, 880 + shape)
    x = x.copy()
    x[:, 1] = x[:, 0]                        # cluster 0: atoms 0 and 1 coincide
    o = off[3]
    x[:, o + 1] = x[:, o] + [1e7, 0.0, 0.0]  # cluster 3: a pair 1e7 apart
    p = lj.lbfgs_params()
    announce(f"morse degenerate clusters class-0 shape {shape}")
    b, xd = morse_dev(off, x, 6.0)
    ro = O.minimize(off, x, oracle_params(p, 6.0))
    lj.set_schedule(lj.SCHED_MIN_CLASS[0], "fp64", b.max_n, shape)
    try:
        r = host_dict(lj.minimize(b, xd, p, "fp64"))
    finally:
        lj.set_schedule(lj.SCHED_MIN_CLASS[0], "fp64", b.max_n, -1)
    for k in ("xyz", "energy", "gnorm", "iters", "evals", "status"):
        assert np.array_equal(r[k], ro[k], equal_nan=True), k
    assert r["status"][0] == lj.NONFINITE


def test_fp64_autotuned_shapes_keep_parity(tmp_path):
    """The autotuner on a Morse batch times the one-wavefront kernels with
    their pair matrix in dynamic LDS beside the other shapes; whatever it
    installs, the FP64 results stay bit-identical to the oracle."""
    sizes = list(uniform_sizes(300, 2, 150, 8901))
    off, x = random_starts(sizes, 8902)
    b, xd = morse_dev(off, x, 6.0)
    p = lj.lbfgs_params()
    announce(f"morse autotune fp64 {b.num} clusters N 2..150")
    try:
        res = lj.autotune(b, xd, "fp64", cache=str(tmp_path / "sched.json"))
        assert set(res["min_class"]) == {0, 1, 2}
        r = host_dict(lj.minimize(b, xd, p, "fp64"))
    finally:
        for c in range(3):
            lj.set_schedule(lj.SCHED_MIN_CLASS[c], "fp64", b.max_n, -1)
        lj.set_schedule(lj.SCHED_EVAL, "fp64", b.max_n, *lj.eval_shape_default(b.max_n))
    ro = O.minimize(off, x, oracle_params(p, 6.0))
    for k in ("xyz", "energy", "gnorm", "iters", "evals", "status"):
        assert np.array_equal(r[k], ro[k]), k


@pytest.mark.parametrize("sizes,rho", [([13] * 8 + [38] * 8, 6.0), ([100, 150], 6.0)])
def test_mixed_polish_reproduces_oracle_from_switch_point(sizes, rho):
    off, x = random_starts(sizes, 850 + len(sizes))
    p = lj.lbfgs_params()
    announce(f"morse minimize mixed sizes={sizes} rho={rho}")
    b, xd = morse_dev(off, x, rho)
    r = host_dict(lj.minimize(b, xd, p, "mixed", switch_point=True))
    ro = O.minimize(off, r["xyz_switch"], oracle_params(p, rho))
    for k in ("xyz", "energy", "gnorm", "status"):
        assert np.array_equal(r[k], ro[k]), k
    assert np.mean(r["status"] == lj.CONVERGED) >= 0.9


def test_fp64_chain_bitwise():
    sizes, rho, steps, seed = [13, 20], 6.0, 30, 25102593811
    off, x = random_starts(sizes, seed)
    p = lj.lbfgs_params()
    b, xd = morse_dev(off, x, rho)
    announce(f"morse bh fp64 sizes={sizes} steps={steps}")
    r = lj.minimize(b, xd, p, "fp64")
    bh = lj.bh_params(cands=4, kT=0.8, seed=seed)
    chain = lj.BasinHopping(b, r["xyz"], r["energy"], bh, p, "fp64", trace_steps=steps)
    chain.step(steps)
    torch.cuda.synchronize()
    xcur = r["xyz"].cpu().numpy().copy()
    states = [O.chain_state(float(e), 0.4) for e in r["energy"].cpu().numpy()]
    params = O.bh_params(len(sizes), bh.cands, kT=bh.kT, adapt_interval=bh.adapt_interval,
                         target_rate=bh.target_rate, factor=bh.factor, seed=bh.seed)
    xbest = xcur.copy()
    tro = O.bh_run(off, xcur, states, params, oracle_params(p, rho), steps, xbest=xbest)
    tr = {k: (None if v is None else v.cpu().numpy()) for k, v in chain.trace.items()}
    for k in ("e_trial", "e_best", "e_best_acc", "e_cur", "step"):
        assert np.array_equal(tr[k], tro[k], equal_nan=True), k
    assert np.array_equal(tr["accepted"], tro["accepted"])
    assert np.array_equal(host(chain.xyz_cur), xcur)
    assert np.array_equal(host(chain.xyz_best), xbest)


@pytest.mark.parametrize("pair", ["lj", "morse"])
@pytest.mark.parametrize("sigma,eps", [(2.0, 0.25), (1.3, 0.7)])
def test_units_rescale_inputs_and_outputs(pair, sigma, eps):
    """Powers of two convert exactly (bitwise results); other factors round the
    reduced coordinates once, which moves E and g by a few ulps (1e-12)."""
    exact = sigma == 2.0
    rtol = 0.0 if exact else 1e-12
    rho = 6.0
    off, x = random_starts([13, 38], 901)
    xs = x * sigma  # the same clusters in units of sigma
    announce(f"units pair={pair} sigma={sigma} eps={eps}")
    b = lj.ClusterBatch(off, device="cuda", pair=pair, rho=rho)
    E, g = lj.energy_grad(b, torch.from_numpy(xs).cuda(), "fp64", sigma=sigma, epsilon=eps)
    Eo, go = O.energy_grad(off, xs / sigma, pair, rho)
    E, g = host(E), host(g)
    if exact:
        assert np.array_equal(E, eps * Eo) and np.array_equal(g, (eps / sigma) * go)
    np.testing.assert_allclose(E, eps * Eo, rtol=rtol, atol=0)
    np.testing.assert_allclose(g, (eps / sigma) * go, rtol=rtol,
                               atol=rtol * np.abs(go).max() * eps / sigma)
    r = host_dict(lj.minimize(b, torch.from_numpy(xs).cuda(), lj.lbfgs_params(), "fp64",
                              sigma=sigma, epsilon=eps))
    ro = O.minimize(off, xs / sigma, O.lbfgs_params(pair=pair, rho=rho))
    if exact:
        assert np.array_equal(r["energy"], eps * ro["energy"])
        assert np.array_equal(r["xyz"], sigma * ro["xyz"])
    else:  # a one-ulp change of a start may change the minimum reached
        assert np.all(r["status"] == lj.CONVERGED)
        assert np.all(r["gnorm"] < 1e-6 * eps / sigma)  # the reduced tolerance, converted
