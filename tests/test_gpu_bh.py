"""GPU parity of lj_bh_step (perturb, minimise, select, Metropolis, adapt).

FP64 chains are bit-identical to the oracle's basin-hopping run (every trace
row and the final state).  Mixed chains are checked by replay: the oracle's
selection / Metropolis / adaptation, fed the GPU's candidate energies, takes
the same decisions bit for bit.  Graph replays equal eager execution.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_util import announce, host, to_dev
from oracle import oracle as O
from paper_2510_25938_amd import lj
from paper_2510_25938_amd.inputs import random_starts

pytestmark = pytest.mark.gpu


def start_chains(sizes, seed, precision="fp64"):
    off, x = random_starts(sizes, seed)
    b, xd = to_dev(off, x)
    p = lj.lbfgs_params()
    r = lj.minimize(b, xd, p, "fp64")
    torch.cuda.synchronize()
    return off, b, r, p


def oracle_chains(off, r, bh, p, steps, step0=0.4):
    xcur = r["xyz"].cpu().numpy().copy()
    e0 = r["energy"].cpu().numpy()
    states = [O.chain_state(float(e), step0) for e in e0]
    params = O.bh_params(len(e0), bh.cands, kT=bh.kT, adapt_interval=bh.adapt_interval,
                         target_rate=bh.target_rate, factor=bh.factor, seed=bh.seed)
    lp = O.lbfgs_params(m=p.m, gtol=p.gtol, max_iter=p.max_iter, max_step=p.max_step, c1=p.c1,
                        max_ls=p.max_ls, curv_eps=p.curv_eps)
    xbest = xcur.copy()
    tr = O.bh_run(off, xcur, states, params, lp, steps, xbest=xbest)
    return xcur, xbest, states, tr


def gpu_trace(bhx):
    torch.cuda.synchronize()
    return {k: (None if v is None else v.cpu().numpy()) for k, v in bhx.trace.items()}


@pytest.mark.parametrize("sizes,steps,cands", [([13], 200, 8), ([13, 20, 38], 25, 4),
                                               ([2, 13], 30, 1)])
def test_fp64_chain_bitwise(sizes, steps, cands):
    seed = 25102593801 + len(sizes)
    off, b, r, p = start_chains(sizes, seed)
    bh = lj.bh_params(cands=cands, kT=0.8, seed=seed)
    announce(f"bh fp64 sizes={sizes} steps={steps} cands={cands}")
    bhx = lj.BasinHopping(b, r["xyz"], r["energy"], bh, p, "fp64", trace_steps=steps,
                          trace_candidates=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        bhx.step(steps)
    stream.synchronize()
    xcur, xbest, states, tro = oracle_chains(off, r, bh, p, steps)
    tr = gpu_trace(bhx)
    for k in ("e_trial", "e_best", "e_best_acc", "e_cur", "step"):
        assert np.array_equal(tr[k], tro[k], equal_nan=True), k
    assert np.array_equal(tr["accepted"], tro["accepted"])
    assert np.array_equal(tr["e_cand"], tro["ecand"], equal_nan=True)
    assert np.all(tr["polish_status"] == -1)  # nothing is polished on the FP64 path
    assert np.array_equal(host(bhx.xyz_cur), xcur)
    assert np.array_equal(host(bhx.xyz_best), xbest)
    assert np.array_equal(host(bhx.e_cur), [s.e_cur for s in states])
    assert np.array_equal(host(bhx.step_size), [s.step for s in states])
    assert np.array_equal(host(bhx.step_index), [s.step_index for s in states])
    assert np.array_equal(host(bhx.win_accepts), [s.win_accepts for s in states])
    if sizes == [13]:
        assert states[0].e_best_acc == pytest.approx(-44.326801, abs=1e-6)


def test_graph_replays_match_eager():
    """Per-step graph replays (with host reads in between) equal eager steps."""
    sizes = [13, 38]
    off, b, r, p = start_chains(sizes, 77)
    bh = lj.bh_params(cands=8, seed=77)
    announce("bh graph vs eager")
    g = lj.BasinHopping(b, r["xyz"], r["energy"], bh, p, "fp64", trace_steps=12)
    e = lj.BasinHopping(b, r["xyz"], r["energy"], bh, p, "fp64", trace_steps=12)
    side = torch.cuda.Stream()
    captured = lj.graph_captures()
    for k in range(12):
        with torch.cuda.stream(side):
            g.step(1)  # captured once, replayed
        side.synchronize()
        e.step(1, stream=torch.cuda.default_stream())  # null stream: eager launches
        torch.cuda.synchronize()
        assert torch.equal(g.xyz_cur, e.xyz_cur), k
        assert torch.equal(g.e_cur, e.e_cur) and torch.equal(g.step_size, e.step_size), k
    # the first step captured the graph, the other eleven replayed it
    assert lj.graph_captures() == captured + 1
    tg, te = gpu_trace(g), gpu_trace(e)
    for k in tg:
        if tg[k] is not None:
            assert np.array_equal(tg[k], te[k], equal_nan=True), k


def replay_decisions(tr, e0, bh, step0=0.4):
    """Feed the GPU's candidate energies through the oracle's decision logic."""
    C_, S = tr["e_trial"].shape
    params = O.bh_params(C_, bh.cands, kT=bh.kT, adapt_interval=bh.adapt_interval,
                         target_rate=bh.target_rate, factor=bh.factor, seed=bh.seed)
    for c in range(C_):
        st = O.chain_state(float(e0[c]), step0)
        for k in range(S):
            sel, acc, _, esel = O.bh_decide(st, params, c, tr["e_cand"][c, k])
            assert acc == tr["accepted"][c, k], (c, k)
            assert (np.isnan(esel) and np.isnan(tr["e_trial"][c, k])) or esel == tr["e_trial"][c, k]
            assert st.step == tr["step"][c, k], (c, k)
            assert st.e_best_seen == tr["e_best"][c, k], (c, k)
            # the GPU's current energy after an accepted move is the polished one
            st.e_cur = tr["e_cur"][c, k]


@pytest.mark.parametrize("chains,steps", [(6, 40), (64, 12)])
def test_mixed_chains_replay(chains, steps):
    sizes = list(np.random.default_rng(chains).integers(38, 76, size=chains))
    off, b, r, p = start_chains(sizes, 900 + chains)
    bh = lj.bh_params(cands=8, seed=900 + chains)
    announce(f"bh mixed replay chains={chains} steps={steps}")
    bhx = lj.BasinHopping(b, r["xyz"], r["energy"], bh, p, "mixed", trace_steps=steps,
                          trace_candidates=True)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        bhx.step(steps)
    side.synchronize()
    tr = gpu_trace(bhx)
    replay_decisions(tr, r["energy"].cpu().numpy(), bh)
    # every accepted candidate's FP64 polish converged, and nothing else was
    # polished
    acc = tr["accepted"] == 1
    assert np.all(tr["polish_status"][acc] == lj.CONVERGED)
    assert np.all(tr["polish_status"][~acc] == -1)
    # current structures are FP64 minima to ||g|| < 1e-6 by the oracle's own
    # gradient, with the reported energy
    xc = host(bhx.xyz_cur)
    Eo, go = O.energy_grad(off, xc)
    assert np.array_equal(Eo, host(bhx.e_cur))
    for c in range(chains):
        gb = go[:, off[c]:off[c + 1]]
        assert np.sqrt(np.sum(gb * gb)) < 1e-6
    assert np.all(tr["accepted"].sum(axis=1) > 0)


def test_steps_alternating_streams_match_one_stream():
    """Steps of one chain set issued on two streams in turn, with no host
    synchronisation, equal the same steps on one stream: each step waits for
    the previous one wherever it ran."""
    sizes = [13, 38, 55, 20]
    off, b, r, p = start_chains(sizes, 4242)
    bh = lj.bh_params(cands=8, seed=4242)
    announce("bh alternating streams vs one stream")
    alt = lj.BasinHopping(b, r["xyz"], r["energy"], bh, p, "mixed", trace_steps=10)
    one = lj.BasinHopping(b, r["xyz"], r["energy"], bh, p, "mixed", trace_steps=10)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for k in range(10):
        alt.step(1, stream=s1 if k % 2 == 0 else s2)
        if k == 4:
            alt.step(0)  # a no-op call on the current stream keeps the order
    for k in range(10):
        one.step(1, stream=s1)
    torch.cuda.synchronize()
    ta, to = gpu_trace(alt), gpu_trace(one)
    for k in ta:
        if ta[k] is not None:
            assert np.array_equal(ta[k], to[k], equal_nan=True), k
    assert torch.equal(alt.xyz_cur, one.xyz_cur) and torch.equal(alt.e_cur, one.e_cur)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_bh_short_workspace_is_rejected(prec):
    """lj_bh_step with a missing or short workspace returns LJ_E_WORKSPACE and
    leaves the chain state as it was."""
    off, b, r, p = start_chains([13, 38], 45)
    bh = lj.bh_params(cands=4, seed=3)
    chains = lj.BasinHopping(b, r["xyz"], r["energy"], bh, p, prec)
    announce(f"short workspace bh_step prec={prec} need={chains.workspace.numel()}")
    before = [t.clone() for t in (chains.xyz_cur, chains.e_cur, chains.step_size,
                                  chains.win_accepts, chains.step_index)]
    L = lj.lib()
    for ws, nb in ((None, chains.workspace.numel()),
                   (chains.workspace.data_ptr(), chains.workspace.numel() - 1)):
        st = L.lj_bh_step(C.byref(b.desc()), C.byref(chains.state), C.byref(bh), C.byref(p),
                          lj.precision_code(prec), 2, None, ws, nb, None)
        assert st == lj.E_WORKSPACE
    torch.cuda.synchronize()
    after = (chains.xyz_cur, chains.e_cur, chains.step_size, chains.win_accepts,
             chains.step_index)
    for a, z in zip(before, after):
        assert torch.equal(a, z)


def test_threads_on_separate_streams_match_serial_runs():
    """Two host threads, each on its own stream: one steps basin-hopping chains
    of two size classes (the first step captures its graph), the other runs
    eager minimisations of three size classes.  Each thread's results equal
    the same work done alone, bit for bit."""
    import threading

    off, b, r, p = start_chains([38, 70, 38, 70], 47)
    bh = lj.bh_params(cands=4, seed=11)
    moff, mx = random_starts([13, 80, 150, 38], 49)
    mb, mxd = to_dev(moff, mx)
    announce("threads: bh_step mixed (38, 70) x 4 steps || minimize fp64 (13, 80, 150, 38) x 6")

    def bh_run(stream):
        ch = lj.BasinHopping(b, r["xyz"], r["energy"], bh, p, "mixed")
        torch.cuda.synchronize()
        for _ in range(4):
            ch.step(1, stream=stream)
        return ch

    ref_bh = bh_run(None)
    ref_min = lj.minimize(mb, mxd, p, "fp64")
    torch.cuda.synchronize()

    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    chains = lj.BasinHopping(b, r["xyz"], r["energy"], bh, p, "mixed")
    torch.cuda.synchronize()
    outs, errors = [], []

    def thread_a():
        try:
            with torch.cuda.stream(sa):
                for _ in range(4):
                    chains.step(1, stream=sa)
            sa.synchronize()
        except Exception as e:  # reported below
            errors.append(e)

    def thread_b():
        try:
            with torch.cuda.stream(sb):
                for _ in range(6):
                    outs.append(lj.minimize(mb, mxd, p, "fp64", stream=sb))
            sb.synchronize()
        except Exception as e:
            errors.append(e)

    ta, tb = threading.Thread(target=thread_a), threading.Thread(target=thread_b)
    ta.start()
    tb.start()
    ta.join()
    tb.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for name in ("xyz_cur", "e_cur", "step_size", "win_accepts", "step_index", "e_best_seen",
                 "e_best_acc", "xyz_best"):
        assert torch.equal(getattr(chains, name), getattr(ref_bh, name)), name
    assert len(outs) == 6
    for o in outs:
        for k in ("xyz", "energy", "gnorm", "iters", "evals", "status"):
            assert torch.equal(o[k], ref_min[k]), k


def test_graph_cache_eviction_and_recapture():
    """More distinct step graphs than the cache holds: evicted graphs are
    recaptured on their next use, and every chain equals an eager run."""
    off, b, r, p = start_chains([13], 61)
    bh = lj.bh_params(cands=4, seed=5)
    announce("bh graph cache eviction: 18 chain sets")
    side = torch.cuda.Stream()
    graphed = [lj.BasinHopping(b, r["xyz"], r["energy"], bh, p, "fp64") for _ in range(18)]
    eager = [lj.BasinHopping(b, r["xyz"], r["energy"], bh, p, "fp64") for _ in range(18)]
    torch.cuda.synchronize()
    for rnd in range(2):
        for g in graphed:  # 18 keys through a 16-entry cache, twice
            with torch.cuda.stream(side):
                g.step(2, stream=side)
    side.synchronize()
    for e in eager:
        e.step(4, stream=torch.cuda.default_stream())  # null stream: eager launches
    torch.cuda.synchronize()
    for g, e in zip(graphed, eager):
        for name in ("xyz_cur", "e_cur", "step_size", "win_accepts", "step_index", "xyz_best"):
            assert torch.equal(getattr(g, name), getattr(e, name)), name
