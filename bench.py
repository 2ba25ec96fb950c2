"""Benchmark of the batched local-minimisation hot path on one MI355X.

Workload (one step): 1024 independent LJ38 clusters from seeded random starts
in a cube of side 1.2 * 38^(1/3), each minimised with L-BFGS (m = 10) to
||g||_2 < 1e-6 in one call of lj_bh_minimize_batch.  The headline value is the
mixed path (FP32 pair arithmetic, FP64 reductions / curvature pairs / Armijo,
FP64 polish); the FP64 path is timed the same way for the speedup.  Inputs
are resident in HBM before the timed region; each step restores the starts
with one device copy (0.9 MB) and minimises them.

Also measured: the standalone pair kernel (lj_energy_grad_batch) on 256
clusters of N = 1000, and the CPU oracle on the host (one thread).

Prints one JSON line.  --gpus N with N > 1 is not supported (one GPU).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12  # MI355X vector FP32, published
PEAK_FP64 = 78.6e12   # MI355X vector FP64, published
FLOP_PER_PAIR = 27    # algorithmic FLOP per unique pair evaluation (E and gradient)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("lj_device.hpp", "lj_kernels.hpp", "lj_minimize.hip"):
        with open(os.path.join(ROOT, "paper_2510_25938_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(key):
    """HBM bytes per launch from committed rocprofv3 counter runs, if current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_sha") != kernel_source_hash() or key not in t:
        return None
    return t[key]["hbm_bytes_per_launch"]


def load_pair_counters(key, launch_ms):
    """Counted FLOP/s and VALU issue rate of the pair kernel from committed SQ
    counter runs (profiles/pair_counters.json), if current, at this run's
    launch duration."""
    path = os.path.join(ROOT, "profiles", "pair_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_sha") != kernel_source_hash() or key not in t:
        return None
    k = t[key]
    s = launch_ms * 1e-3
    flop = k["counted_flop_fp32"] + k["counted_flop_fp64"]
    return {"counted_flop_per_launch": flop, "counted_tflops": flop / s / 1e12,
            "valu_insts_per_launch": k["valu_insts"],
            "valu_issue_frac": k["valu_insts"] / s / t["valu_issue_peak_per_s"]}


def load_issue(key, launch_ms):
    """VALU issue rate of the minimiser from committed SQ counter runs, if current.

    The kernel runs one wavefront per SIMD, so its bound is instruction issue:
    the peak is one wave64 VALU instruction per SIMD every 4 cycles
    (256 CUs x 4 SIMDs x 2.4 GHz / 4)."""
    path = os.path.join(ROOT, "profiles", "issue.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_sha") != kernel_source_hash() or key not in t:
        return None
    k, peak = t[key], t["valu_issue_peak_per_s"]
    rate = k["valu_insts_per_launch"] / (launch_ms * 1e-3)
    return {"valu_insts_per_launch": k["valu_insts_per_launch"],
            "valu_per_iteration": round(k["valu_per_iteration"], 1),
            "cycles_per_instruction": round(k["cycles_per_instruction"], 2),
            "achieved_ginst_per_s": rate / 1e9, "peak_ginst_per_s": peak / 1e9,
            "frac": rate / peak,
            "counted_tflop_per_s": (k["counted_flop_fp32"] + k["counted_flop_fp64"])
            / (launch_ms * 1e-3) / 1e12}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_pool(O, off, x, ref):
    """The oracle under the paper's parallel scheme: a pool of workers over the
    candidates (threads here: the oracle's C entry point runs without the GIL),
    one contiguous slice of clusters per worker, on up to 16 host cores."""
    import concurrent.futures as cf
    B = off.size - 1
    P = max(1, min(16, os.cpu_count() or 1))
    cuts = np.linspace(0, B, P + 1).astype(int)

    def work(k):
        a, b = cuts[k], cuts[k + 1]
        return O.minimize(off[a:b + 1] - off[a], x[:, off[a]:off[b]])

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(P) as ex:
        parts = list(ex.map(work, range(P)))
    s = time.perf_counter() - t0
    same = all(np.array_equal(r["energy"], ref["energy"][cuts[k]:cuts[k + 1]])
               for k, r in enumerate(parts))
    return {"value": B / s, "unit": "minimisations/s", "cores": P, "kind": "oracle",
            "sample": f"all {B} LJ38 starts, {P} worker threads over contiguous slices "
                      f"({s:.2f} s)", "matches_one_thread": same}


def pair_kernel(lj, large_clusters, dev, stream, torch):
    """lj_energy_grad_batch on 256 clusters of N = 1000, FP32-pair and FP64."""
    wl4 = large_clusters()
    off4, x4 = wl4.starts()
    b4 = lj.ClusterBatch(off4, device=dev)
    x4d = torch.from_numpy(x4).to(dev)
    out = {}
    for prec, peak in (("mixed", PEAK_FP32), ("fp64", PEAK_FP64)):
        with torch.cuda.stream(stream):
            for _ in range(3):
                lj.energy_grad(b4, x4d, prec, stream=stream)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            reps = 20
            e0.record(stream)
            for _ in range(reps):
                lj.energy_grad(b4, x4d, prec, stream=stream)
            e1.record(stream)
            stream.synchronize()
        ms = e0.elapsed_time(e1) / reps
        pairs = b4.num * 1000 * 999 / 2
        flops = FLOP_PER_PAIR * pairs
        w, a = lj.get_schedule(lj.SCHED_EVAL, prec, 1000)
        out[prec] = {"workload": "256 x LJ1000 energy+gradient", "schedule": f"{w} waves x {a} atoms",
                     "ms": ms, "pair_evals_per_s": pairs / (ms * 1e-3),
                     "achieved_tflops": flops / (ms * 1e-3) / 1e12,
                     "peak_tflops": peak / 1e12, "frac_of_peak": flops / (ms * 1e-3) / peak}
        cnt = load_pair_counters(f"pair_{prec}_lj1000_256", ms)
        if cnt is not None:
            cnt["counted_frac_of_peak"] = cnt["counted_tflops"] * 1e12 / peak
            out[prec]["counters"] = cnt
    return out


def timed(torch, stream, fn, reps=5, setup=None):
    """Median GPU time (ms) of fn(arg) on `stream` over `reps` calls, after one
    warm-up call; arg = setup() is prepared before each call, outside the
    timed region (None without setup).  Returns (median ms, last result)."""
    times, out = [], None
    with torch.cuda.stream(stream):
        for k in range(reps + 1):
            arg = setup() if setup else None
            stream.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            out = fn(arg)
            e1.record(stream)
            stream.synchronize()
            if k > 0:
                times.append(e0.elapsed_time(e1))
    return float(np.median(times)), out


def pool_size():
    return max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                      else (os.cpu_count() or 1)))


def oracle_minimize_pool(O, off, x, params=None, P=None):
    """The oracle over a batch on P worker threads (contiguous slices of
    clusters; its C entry point runs without the GIL).  Returns (merged
    results, wall seconds, P)."""
    import concurrent.futures as cf
    off = np.asarray(off, np.int64)
    B = off.size - 1
    P = P or pool_size()
    P = max(1, min(P, B))
    cuts = np.linspace(0, B, P + 1).astype(int)

    def work(k):
        a, b = cuts[k], cuts[k + 1]
        return O.minimize((off[a:b + 1] - off[a]).astype(np.int32),
                          np.ascontiguousarray(x[:, off[a]:off[b]]), params)

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(P) as ex:
        parts = list(ex.map(work, range(P)))
    sec = time.perf_counter() - t0
    merged = {k: np.concatenate([q[k] for q in parts], axis=-1) for k in parts[0]}
    return merged, sec, P


def oracle_chains_pool(O, off, xmin, e0, w, steps, P=None):
    """The oracle's FP64 basin hopping of a set of chains, one contiguous
    slice of chains per worker thread (each slice keeps its chains' random
    streams).  Returns (trace, final states, xcur, wall seconds, P)."""
    import concurrent.futures as cf
    off = np.asarray(off, np.int64)
    nch = off.size - 1
    P = max(1, min(P or pool_size(), nch))
    cuts = np.linspace(0, nch, P + 1).astype(int)
    params = O.bh_params(nch, w.cands, kT=w.kT, seed=w.seed)

    def part(i):
        a, e = cuts[i], cuts[i + 1]
        so = (off[a:e + 1] - off[a]).astype(np.int32)
        xs = np.ascontiguousarray(xmin[:, off[a]:off[e]])
        st = [O.chain_state(float(q), w.step0) for q in e0[a:e]]
        tr = O.bh_run(so, xs, st, params, O.lbfgs_params(), steps, chain0=a)
        return xs, st, tr

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(P) as ex:
        parts = list(ex.map(part, range(P)))
    sec = time.perf_counter() - t0
    tr = {k: np.concatenate([q[2][k] for q in parts]) for k in parts[0][2]}
    states = [s for q in parts for s in q[1]]
    xcur = np.concatenate([q[0] for q in parts], axis=1)
    return tr, states, xcur, sec, P


def per_cluster_equal(a, b, off):
    """Share of clusters whose coordinates, energy and status are identical."""
    B = off.size - 1
    return float(np.mean([np.array_equal(a["xyz"][:, off[k]:off[k + 1]],
                                          b["xyz"][:, off[k]:off[k + 1]])
                          and a["energy"][k] == b["energy"][k]
                          and a["status"][k] == b["status"][k] for k in range(B)]))


def errors_at_results(O, off, h, pair="lj", rho=6.0):
    """The oracle's energy and gradient norm at every GPU result: the largest
    |E_reported - E_oracle| and the largest oracle ||g||."""
    Eo, go = O.energy_grad(off, h["xyz"], pair=pair, rho=rho)
    gn = np.sqrt(np.add.reduceat((go * go).sum(axis=0), off[:-1])) if off[-1] > 0 else go
    return {"energy_abs_err_max_vs_oracle_at_result": float(np.max(np.abs(h["energy"] - Eo))),
            "gnorm_oracle_at_result_max": float(np.max(gn)),
            "gnorm_oracle_at_result_median": float(np.median(gn))}


WORKLOADS = ("lj13bh", "uneven", "large", "morse", "chains", "small")


def workloads(lj, inputs, torch, stream, oracle=None, only=None):
    """Every benchmark workload at full size (beside the headline LJ38 batch);
    `only`, one of WORKLOADS, runs a single one (for profiler runs)."""
    res = {}
    if only in (None, "lj13bh"):
        res.update(lj13_chain(lj, inputs, torch, stream, oracle))
    if only in (None, "uneven"):
        res.update(uneven_batch(lj, inputs, torch, stream, oracle))
    if only in (None, "large"):
        res.update(large_batch(lj, inputs, torch, stream, oracle))
    if only in (None, "morse"):
        res.update(morse_batch(lj, inputs, torch, stream, oracle))
    if only in (None, "chains"):
        res.update(many_chains(lj, inputs, torch, stream, oracle))
    if only in (None, "small"):
        res.update(small_batch(lj, inputs, torch, stream, oracle))
    return res


def reset_class_schedules(lj, max_n):
    for prec in ("fp64", "mixed"):
        for c in range(3):
            if c <= lj._class_of(max_n):
                lj.set_schedule(lj.SCHED_MIN_CLASS[c], prec, max_n, -1)


def small_batch(lj, inputs, torch, stream, O):
    """16384 LJ13 clusters, FP64 and mixed, in one call: the built-in
    schedule (four clusters per wavefront at this batch size) against one
    cluster per wavefront reduced over a 16-lane row, the fastest one-cluster
    shape.  The oracle on the first 512 clusters checks the FP64 results."""
    dev = "cuda"
    w = inputs.lj13_batch()
    off, x = w.starts()
    b = lj.ClusterBatch(off, device=dev)
    xd = torch.from_numpy(x).to(dev)
    pairs = (b.sizes * (b.sizes - 1) // 2).astype(np.int64)
    entry, host = minimize_legs(lj, b, xd, lj.lbfgs_params(), torch, stream, pairs)
    entry["shape"] = "four clusters per wavefront"
    one = {}
    for prec in ("fp64", "mixed"):
        lj.set_schedule(lj.SCHED_MIN_CLASS[0], prec, b.max_n, 1)
        ms, _ = timed(torch, stream, lambda _: lj.minimize(b, xd, lj.lbfgs_params(), prec,
                                                           stream=stream))
        one[prec] = {"ms": ms, "minimisations_per_s": b.num / (ms * 1e-3)}
    reset_class_schedules(lj, b.max_n)
    entry["one_cluster_per_wavefront"] = one
    entry["speedup_packed_vs_one_per_wavefront"] = {
        p: one[p]["ms"] / entry[p]["ms"] for p in ("fp64", "mixed")}
    if O is not None:
        sub = 512
        t0 = time.perf_counter()
        ro = O.minimize(off[:sub + 1], x[:, :off[sub]])
        sec = time.perf_counter() - t0
        h = {k: (v[:, :off[sub]] if k == "xyz" else v[:sub]) for k, v in host["fp64"].items()}
        entry["cpu_oracle"] = {"minimisations_per_s": sub / sec, "cores": 1,
                               "sample": f"the first {sub} clusters, FP64, one thread "
                                         f"({sec:.2f} s)"}
        entry["parity"] = {"fp64_bitwise_frac_subset": per_cluster_equal(h, ro, off[:sub + 1]),
                           "fp64_subset": sub,
                           **{"mixed_" + k: v for k, v in
                              errors_at_results(O, off, host["mixed"]).items()}}
    return {w.name: entry}


def lj13_chain(lj, inputs, torch, stream, oracle):
    """LJ13 basin hopping: 1 chain x 8 candidates x 200 steps, FP64, one graph
    per step.  The chain object is built outside the timed region."""
    dev = "cuda"
    w = inputs.lj13_bh()
    off, x = w.starts()
    b = lj.ClusterBatch(off, device=dev)
    r0 = lj.minimize(b, torch.from_numpy(x).to(dev), lj.lbfgs_params(), "fp64", stream=stream)
    stream.synchronize()

    def setup():
        return lj.BasinHopping(b, r0["xyz"], r0["energy"],
                               lj.bh_params(cands=w.cands, kT=w.kT, seed=w.seed),
                               lj.lbfgs_params(), "fp64", step0=w.step0, trace_steps=w.steps)

    def chain(c):
        c.step(w.steps, stream=stream)
        return c
    ms, c = timed(torch, stream, chain, setup=setup)
    e_best = float(c.e_best_acc[0].item())
    entry = {"chain_steps_per_s": w.steps / (ms * 1e-3), "ms": ms, "reps": 5, "stat": "median",
             "best_energy": e_best, "reached_lj13_minimum": abs(e_best + 44.326801) < 1e-6}
    # the autotuner on the step's candidate batch (8 perturbed copies of the
    # start minimum), then the chain again with the tuned shapes
    cand_off = np.arange(w.cands + 1, dtype=np.int32) * 13
    cb = lj.ClusterBatch(cand_off, device=dev)
    xc8 = r0["xyz"].repeat(1, w.cands).contiguous()
    xc8 = xc8 + 0.4 * (2 * torch.rand(xc8.shape, generator=torch.Generator(device=dev)
                                      .manual_seed(w.seed), device=dev, dtype=torch.float64) - 1)
    tune = lj.autotune(cb, xc8, "fp64", stream=stream)
    ms_t, c_t = timed(torch, stream, chain, setup=setup)
    entry["tuned"] = {"chain_steps_per_s": w.steps / (ms_t * 1e-3), "ms": ms_t,
                      "class0_shape": tune["min_class"].get(0),
                      "same_chain": bool(torch.equal(c_t.xyz_cur, c.xyz_cur))}
    reset_class_schedules(lj, 13)
    if oracle is not None:
        xc = r0["xyz"].cpu().numpy().copy()
        st = [oracle.chain_state(float(r0["energy"][0].item()), w.step0)]
        t0 = time.perf_counter()
        tro = oracle.bh_run(off, xc, st, oracle.bh_params(1, w.cands, kT=w.kT, seed=w.seed),
                            oracle.lbfgs_params(), w.steps)
        entry["cpu_oracle_chain_steps_per_s"] = w.steps / (time.perf_counter() - t0)
        entry["cpu_oracle_cores"] = 1
        tr = {k: v.cpu().numpy() for k, v in c.trace.items() if v is not None}
        entry["fp64_trace_bitwise"] = bool(
            all(np.array_equal(tr[k], tro[k], equal_nan=True)
                for k in ("e_trial", "e_best", "e_best_acc", "e_cur", "step"))
            and np.array_equal(tr["accepted"], tro["accepted"])
            and np.array_equal(c.xyz_cur.cpu().numpy(), xc))
    return {w.name: entry}


def minimize_legs(lj, b, xd, params, torch, stream, pairs):
    entry, host = {}, {}
    for prec in ("mixed", "fp64"):
        ms, r = timed(torch, stream, lambda _: lj.minimize(b, xd, params, prec, stream=stream))
        h = {k: v.cpu().numpy() for k, v in r.items() if v is not None}
        ev = h["evals"].astype(np.int64)
        entry[prec] = {"ms": ms, "minimisations_per_s": b.num / (ms * 1e-3),
                       "pair_evals_per_s": float((ev * pairs).sum()) / (ms * 1e-3),
                       "converged_frac": float(np.mean(h["status"] == lj.CONVERGED)),
                       "median_iters": float(np.median(h["iters"])),
                       "max_iters": int(h["iters"].max())}
        host[prec] = h
    entry["reps"], entry["stat"] = 5, "median"
    entry["speedup_mixed_vs_fp64"] = entry["fp64"]["ms"] / entry["mixed"]["ms"]
    return entry, host


def uneven_batch(lj, inputs, torch, stream, O):
    """4096 clusters, N uniform on 13..150: one call, mixed + polish and FP64;
    the oracle on the full batch (a pool of threads) and one thread on the
    first 256 clusters; per-result errors of both paths."""
    dev = "cuda"
    w = inputs.uneven_batch()
    off, x = w.starts()
    b = lj.ClusterBatch(off, device=dev)
    xd = torch.from_numpy(x).to(dev)
    params = lj.lbfgs_params()
    pairs = (b.sizes * (b.sizes - 1) // 2).astype(np.int64)
    entry, host = minimize_legs(lj, b, xd, params, torch, stream, pairs)
    tuned = {}
    for prec in ("mixed", "fp64"):
        t0 = time.perf_counter()
        res = lj.autotune(b, xd, prec, stream=stream)
        tune_s = time.perf_counter() - t0
        ms, r = timed(torch, stream, lambda _: lj.minimize(b, xd, params, prec, stream=stream))
        tuned[prec] = {"ms": ms, "default_ms": entry[prec]["ms"], "shapes": res["min_class"],
                       "autotune_s": tune_s,
                       "same_results": bool(torch.equal(r["energy"].cpu(),
                                                        torch.from_numpy(host[prec]["energy"])))}
    reset_class_schedules(lj, b.max_n)
    lj.set_schedule(lj.SCHED_EVAL, "mixed", b.max_n, *lj.eval_shape_default(b.max_n))
    lj.set_schedule(lj.SCHED_EVAL, "fp64", b.max_n, *lj.eval_shape_default(b.max_n))
    entry["tuned"] = tuned
    if O is None:
        return {w.name: entry}
    ro, sec, P = oracle_minimize_pool(O, off, x)
    sub = 256
    t0 = time.perf_counter()
    O.minimize(off[:sub + 1], x[:, :off[sub]])
    sec1 = time.perf_counter() - t0
    entry["cpu_oracle"] = {
        "pool": {"minimisations_per_s": b.num / sec, "cores": P,
                 "sample": f"all {b.num} clusters, {P} worker threads ({sec:.2f} s)"},
        "one_thread": {"minimisations_per_s": sub / sec1, "cores": 1,
                       "sample": f"the first {sub} clusters ({sec1:.2f} s)"}}
    with torch.cuda.stream(stream):
        rs = lj.minimize(b, xd, params, "mixed", switch_point=True, stream=stream)
    stream.synchronize()
    hs = {k: v.cpu().numpy() for k, v in rs.items() if v is not None}
    rp, _, _ = oracle_minimize_pool(O, off, hs["xyz_switch"])
    rel = np.abs(host["mixed"]["energy"] - ro["energy"]) / np.abs(ro["energy"])
    entry["parity"] = {
        "fp64_bitwise_frac": per_cluster_equal(host["fp64"], ro, off),
        "mixed_rerun_equals_timed": bool(np.array_equal(hs["xyz"], host["mixed"]["xyz"])),
        "mixed_polish_bitwise_frac": per_cluster_equal(hs, rp, off),
        "mixed_same_minimum_frac_1e-6": float(np.mean(rel <= 1e-6)),
        "mixed_energy_rel_err_median": float(np.median(rel)),
        **{"mixed_" + k: v for k, v in errors_at_results(O, off, host["mixed"]).items()}}
    return {w.name: entry}


def large_batch(lj, inputs, torch, stream, O):
    """256 clusters of N = 1000, 500-iteration cap, mixed without polish and
    FP64; the oracle on a 32-cluster subset (a pool of threads)."""
    dev = "cuda"
    w = inputs.large_clusters()
    off, x = w.starts()
    b = lj.ClusterBatch(off, device=dev)
    xd = torch.from_numpy(x).to(dev)
    params = lj.lbfgs_params(max_iter=500, polish=0)
    pairs = (b.sizes * (b.sizes - 1) // 2).astype(np.int64)
    entry, host = minimize_legs(lj, b, xd, params, torch, stream, pairs)
    if O is None:
        return {w.name: entry}
    sub = 32
    so = off[:sub + 1]
    ro, sec, P = oracle_minimize_pool(O, so, x[:, :off[sub]], O.lbfgs_params(max_iter=500))
    entry["cpu_oracle"] = {"minimisations_per_s": sub / sec, "cores": P,
                           "sample": f"the first {sub} clusters, FP64, {P} worker threads "
                                     f"({sec:.2f} s)"}
    h64 = {k: (v[:, :off[sub]] if k == "xyz" else v[:sub]) for k, v in host["fp64"].items()}
    entry["parity"] = {
        "fp64_bitwise_frac_subset": per_cluster_equal(h64, ro, so),
        "fp64_subset": sub,
        **{"mixed_" + k: v for k, v in errors_at_results(O, off, host["mixed"]).items()}}
    return {w.name: entry}


def morse_batch(lj, inputs, torch, stream, O):
    """The Morse pair (range 6) on the LJ38 batch shape: FP64 and mixed."""
    dev = "cuda"
    w = inputs.morse38_batch()
    off, x = w.starts()
    rho = w.extra["rho"]
    b = lj.ClusterBatch(off, device=dev, pair=w.extra["pair"], rho=rho)
    xd = torch.from_numpy(x).to(dev)
    pairs = (b.sizes * (b.sizes - 1) // 2).astype(np.int64)
    entry, host = minimize_legs(lj, b, xd, lj.lbfgs_params(), torch, stream, pairs)
    entry.update(pair="morse", rho=rho)
    if O is None:
        return {w.name: entry}
    op = O.lbfgs_params(pair="morse", rho=rho)
    sub = 64
    t0 = time.perf_counter()
    O.minimize(off[:sub + 1], x[:, :off[sub]], op)
    sec1 = time.perf_counter() - t0
    ro, sec, P = oracle_minimize_pool(O, off, x, op)
    entry["cpu_oracle"] = {
        "pool": {"minimisations_per_s": b.num / sec, "cores": P,
                 "sample": f"all {b.num} clusters, {P} worker threads ({sec:.2f} s)"},
        "one_thread": {"minimisations_per_s": sub / sec1, "cores": 1,
                       "sample": f"the first {sub} clusters ({sec1:.2f} s)"}}
    entry["parity"] = {
        "fp64_bitwise_frac": per_cluster_equal(host["fp64"], ro, off),
        **{"mixed_" + k: v for k, v in errors_at_results(O, off, host["mixed"], "morse",
                                                         rho).items()}}
    return {w.name: entry}


def many_chains(lj, inputs, torch, stream, O):
    """512 chains x 8 candidates, mixed (polish of accepted) and FP64: 20 steps
    per timed run (fresh chains each run, built outside the timed region);
    the oracle on the first 16 chains for the same 20 steps (a pool of
    threads; chains are independent, so its rate scales x32 to all 512)."""
    dev = "cuda"
    w = inputs.many_chains()
    off, x = w.starts()
    b = lj.ClusterBatch(off, device=dev)
    r0 = lj.minimize(b, torch.from_numpy(x).to(dev), lj.lbfgs_params(), "fp64", stream=stream)
    stream.synchronize()
    steps = 20
    entry = {"steps_timed": steps, "steps_in_workload": w.steps, "reps": 5, "stat": "median"}
    chains = {}
    for prec in ("mixed", "fp64"):
        def setup():
            c = lj.BasinHopping(b, r0["xyz"], r0["energy"],
                                lj.bh_params(cands=w.cands, kT=w.kT, seed=w.seed),
                                lj.lbfgs_params(), prec, step0=w.step0, trace_steps=steps,
                                trace_candidates=True)
            chains[prec] = c
            return c
        ms, _ = timed(torch, stream, lambda c: c.step(steps, stream=stream), setup=setup)
        entry[prec] = {"ms_per_step": ms / steps, "chain_steps_per_s": b.num * steps / (ms * 1e-3),
                       "minimisations_per_s": b.num * w.cands * steps / (ms * 1e-3)}
    entry["speedup_mixed_vs_fp64"] = entry["fp64"]["ms_per_step"] / entry["mixed"]["ms_per_step"]
    if O is None:
        return {w.name: entry}
    sub = 16
    xmin, e0 = r0["xyz"].cpu().numpy(), r0["energy"].cpu().numpy()
    tro, states, xcur, sec, P = oracle_chains_pool(O, off[:sub + 1], xmin[:, :off[sub]],
                                                   e0[:sub], w, steps)
    entry["cpu_oracle"] = {"chain_steps_per_s": sub * steps / sec, "cores": P,
                           "sample": f"the first {sub} chains x {steps} steps, FP64, {P} worker "
                                     f"threads ({sec:.2f} s); the same rate holds for 512 chains "
                                     f"(x32 the time)"}
    t64 = {k: v.cpu().numpy()[:sub] for k, v in chains["fp64"].trace.items() if v is not None}
    tm = {k: v.cpu().numpy() for k, v in chains["mixed"].trace.items() if v is not None}
    same = [all(np.array_equal(t64[k][c], tro[k][c], equal_nan=True)
                for k in ("e_trial", "e_best", "e_best_acc", "e_cur", "step", "accepted"))
            and np.array_equal(t64["e_cand"][c], tro["ecand"][c], equal_nan=True)
            for c in range(sub)]
    acc = tm["accepted"] == 1
    xm = chains["mixed"].xyz_cur.cpu().numpy()
    hm = {"xyz": xm, "energy": chains["mixed"].e_cur.cpu().numpy()}
    entry["parity"] = {
        "fp64_chain_bitwise_frac_subset": float(np.mean(same)), "fp64_subset_chains": sub,
        "mixed_accepted_polish_converged_frac": float(np.mean(tm["polish_status"][acc] ==
                                                              lj.CONVERGED)),
        **{"mixed_current_" + k: v for k, v in errors_at_results(O, off, hm).items()}}
    return {w.name: entry}


def candidate_sweep(O, cands=(1, 2, 4, 8, 16), steps=30, seed=2510):
    """The paper's parallel scheme on the host (Parallel Evaluation of
    Candidates; Figs. 4-5 in kind): one LJ38 chain with n candidates per step,
    run twice for each n with the same random streams, once with the n
    minimisations of a step in turn on one thread and once on a pool of
    min(n, 16) worker threads with a barrier per step.  speedup = serial time
    / pool time; efficiency = speedup / workers."""
    import concurrent.futures as cf

    from paper_2510_25938_amd.inputs import random_starts
    off, x = random_starts([38], seed)
    r0 = O.minimize(off, x)
    one = np.array([0, 38], np.int32)

    def run(n, workers):
        params = O.bh_params(1, n, kT=0.8, seed=seed + n)
        st = O.chain_state(float(r0["energy"][0]), 0.4)
        xcur = r0["xyz"].copy()
        with cf.ThreadPoolExecutor(workers) as ex:
            t0 = time.perf_counter()
            for _ in range(steps):
                cand = [O.perturb(xcur, st.step, params.seed, 0, st.step_index, j)
                        for j in range(n)]
                res = list(ex.map(lambda c: O.minimize(one, c), cand))
                sel, acc, _, _ = O.bh_decide(st, params, 0,
                                             np.array([r["energy"][0] for r in res]))
                if acc:
                    xcur = res[sel]["xyz"]
            return time.perf_counter() - t0, st.e_cur

    rows = []
    for n in cands:
        P = max(1, min(n, pool_size()))
        t1, e1 = run(n, 1)
        tp, ep = run(n, P)
        rows.append({"cands": n, "workers": P, "ms_per_step_serial": 1e3 * t1 / steps,
                     "ms_per_step_pool": 1e3 * tp / steps, "speedup": t1 / tp,
                     "efficiency": t1 / tp / P, "same_chain": bool(e1 == ep)})
    return {"workload": f"one LJ38 chain, {steps} steps per candidate count, FP64 oracle",
            "rows": rows}


def iteration_cost(lj, inputs, torch, stream):
    """Where an L-BFGS iteration's time goes when each cluster runs alone on
    its SIMD: 8 clusters (one wavefront each, the rest of the chip idle) and
    the full 1024-cluster LJ38 batch, FP64 and the FP32 phase of the mixed
    path, with m = 10, 3 and 0 pairs of history and a tolerance no run reaches
    (300-iteration cap).  From the slowest cluster's iterations and
    evaluations: the two-loop cost per stored pair, (t(10) - t(3)) / 7, and a
    fit of t = fixed + evaluations x cost per evaluation over m = 3 and m = 0
    (steepest descent evaluates ~5 times per iteration)."""
    out = {}
    for n, count in ((13, 8), (38, 8), (38, 1024)):
        sizes = np.full(count, n)
        off, x = inputs.random_starts(sizes, inputs.SEED_BASE + 8)
        b = lj.ClusterBatch(off)
        xd = torch.from_numpy(x).cuda()
        for prec in ("fp64", "mixed"):
            rows = {}
            for m in (10, 3, 0):
                p = lj.lbfgs_params(m=m, gtol=1e-30, gtol_mixed_per_atom=1e-30, max_iter=300,
                                    polish=0)
                ms, r = timed(torch, stream, lambda _: lj.minimize(b, xd, p, prec, stream=stream))
                it = int(r["iters"].max().item())
                ev = int(r["evals"].max().item())
                rows[m] = dict(ms=ms, iters_max=it, evals_max=ev,
                               us_per_iteration=1e3 * ms / max(it, 1))
            t10, t3, t0 = (rows[m]["us_per_iteration"] for m in (10, 3, 0))
            e3 = rows[3]["evals_max"] / max(rows[3]["iters_max"], 1)
            e0 = rows[0]["evals_max"] / max(rows[0]["iters_max"], 1)
            pair = (t10 - t3) / 7.0
            per_eval = (t0 - t3 + 3.0 * pair) / (e0 - e3) if e0 > e3 else None
            fixed = t0 - e0 * per_eval if per_eval is not None else None
            out[f"lj{n}x{count}_{prec}"] = dict(
                by_history=rows, us_two_loop_per_pair=pair, us_per_evaluation=per_eval,
                us_fixed_per_iteration=fixed)
    return out


def mixed_result_errors(lj, O, batch, starts, params, off, hm, stream, torch):
    """Error of every mixed-path result against the oracle (untimed).

    The oracle re-evaluates E and ||g|| at each GPU minimum, and polishes in
    FP64 from each GPU switch point (recorded by one more untimed run, which
    must reproduce the timed run's results): the GPU polish is expected to
    equal that run bit for bit."""
    with torch.cuda.stream(stream):
        r = lj.minimize(batch, starts, params, "mixed", switch_point=True, stream=stream)
    stream.synchronize()
    h = {k: v.cpu().numpy() for k, v in r.items() if v is not None}
    B = len(off) - 1
    Eo, go = O.energy_grad(off, hm["xyz"])
    gn = np.array([np.sqrt(np.sum(go[:, off[b]:off[b + 1]] ** 2)) for b in range(B)])
    ro = O.minimize(off, h["xyz_switch"])
    same = [np.array_equal(h["xyz"][:, off[b]:off[b + 1]], ro["xyz"][:, off[b]:off[b + 1]])
            and h["energy"][b] == ro["energy"][b] and h["gnorm"][b] == ro["gnorm"][b]
            and h["status"][b] == ro["status"][b] for b in range(B)]
    return {"mixed_rerun_equals_timed": bool(np.array_equal(h["xyz"], hm["xyz"])
                                             and np.array_equal(h["energy"], hm["energy"])),
            "mixed_polish_bitwise_frac": float(np.mean(same)),
            "mixed_energy_abs_err_max_vs_oracle_at_result": float(np.max(np.abs(hm["energy"] - Eo))),
            "mixed_gnorm_oracle_at_result_max": float(np.max(gn)),
            "mixed_gnorm_rel_err_max_vs_oracle_at_result": float(np.max(np.abs(hm["gnorm"] - gn) / gn))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--count", type=int, default=1024, help="LJ38 clusters per step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-pair", action="store_true", help="skip the standalone pair kernel")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the other benchmark workloads")
    ap.add_argument("--only", choices=["mixed", "fp64", "pair", "itercost", *WORKLOADS],
                    help="run one leg only and print its timing (for profiler runs)")
    ap.add_argument("--copy-ref", action="store_true",
                    help="run a plain 256 MiB device-to-device copy 5 times (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(chains shard across GPUs without communication; see the design notes).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2510_25938_amd import lj
    from paper_2510_25938_amd.inputs import large_clusters, lj38_batch

    dev = "cuda"
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    if args.copy_ref:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        with torch.cuda.stream(stream):
            for _ in range(5):
                dst.copy_(src)
        stream.synchronize()
        print(json.dumps({"copy_ref_bytes_read": nbytes, "copy_ref_bytes_written": nbytes,
                          "launches": 5}), flush=True)
        return
    if args.only == "itercost":
        from paper_2510_25938_amd import inputs as inputs_mod
        print(json.dumps({"only": "itercost",
                          "iteration_cost": iteration_cost(lj, inputs_mod, torch, stream)}),
              flush=True)
        return
    if args.only in WORKLOADS:
        from paper_2510_25938_amd import inputs as inputs_mod
        res = workloads(lj, inputs_mod, torch, stream, None, only=args.only)
        print(json.dumps({"only": args.only, "workload": res}), flush=True)
        return
    wl = lj38_batch(args.count)
    off, x = wl.starts()
    n = 38
    batch = lj.ClusterBatch(off, device=dev)
    starts = torch.from_numpy(x).to(dev)
    work = torch.empty_like(starts)
    params = lj.lbfgs_params()
    pairs_per_eval = n * (n - 1) // 2

    def run(precision, steps, warmup):
        ws = torch.empty(max(lj.minimize_workspace_bytes(batch, params, precision), 1),
                         dtype=torch.uint8, device=dev)
        ev_t = []
        out = None
        with torch.cuda.stream(stream):
            for k in range(warmup + steps):
                if k == warmup:
                    stream.synchronize()
                    t0 = time.perf_counter()
                work.copy_(starts)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                out = lj.minimize(batch, work, params, precision, workspace=ws, stream=stream,
                                  inplace=True)
                e1.record(stream)
                if k >= warmup:
                    ev_t.append((e0, e1))
            stream.synchronize()
            wall = time.perf_counter() - t0
        kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ev_t]))
        host = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
        evals = host["evals"].astype(np.int64)
        pair_evals = int(evals.sum()) * pairs_per_eval
        return dict(wall=wall, kern_ms=kern_ms, host=host, pair_evals=pair_evals)

    B = batch.num
    if args.only in ("mixed", "fp64"):
        r = run(args.only, args.steps, args.warmup)
        it, ev = r["host"]["iters"].astype(np.int64), r["host"]["evals"].astype(np.int64)
        print(json.dumps({"only": args.only, "kernel_ms": r["kern_ms"],
                          "minimisations_per_s": B * args.steps / r["wall"],
                          "pair_evals_per_launch": r["pair_evals"],
                          "iters_sum": int(it.sum()), "iters_max": int(it.max()),
                          "evals_sum": int(ev.sum()), "evals_max": int(ev.max())}), flush=True)
        return
    if args.only == "pair":
        args.no_cpu = True
    else:
        mixed = run("mixed", args.steps, args.warmup)
        fp64 = run("fp64", args.steps, args.warmup)

    def summary(r):
        st = r["host"]["status"]
        return dict(minimisations_per_s=B * args.steps / r["wall"],
                    ms_per_step=1e3 * r["wall"] / args.steps,
                    kernel_ms=r["kern_ms"],
                    pair_evals_per_s=r["pair_evals"] / (r["kern_ms"] * 1e-3),
                    converged_frac=float(np.mean(st == lj.CONVERGED)),
                    lsfail_frac=float(np.mean(st == lj.LSFAIL)),
                    median_iters=float(np.median(r["host"]["iters"])),
                    median_evals=float(np.median(r["host"]["evals"])),
                    mean_energy=float(np.mean(r["host"]["energy"])))

    if args.only == "pair":
        pair = pair_kernel(lj, large_clusters, dev, stream, torch)
        print(json.dumps({"only": "pair", "pair_kernel": pair}), flush=True)
        return
    sm, s64 = summary(mixed), summary(fp64)

    # Sampled parity against the oracle (FP64: bitwise; mixed: same-minimum rate).
    parity = {}
    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O

        # one thread pinned to one host core for the oracle leg, then restored
        aff = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
        core = min(aff) if aff else None
        if core is not None:
            os.sched_setaffinity(0, {core})
        try:
            t0 = time.perf_counter()
            ro = O.minimize(off, x)
            cpu_s = time.perf_counter() - t0
        finally:
            if aff:
                os.sched_setaffinity(0, aff)
        cpu = {"value": B / cpu_s, "unit": "minimisations/s", "cores": 1, "kind": "oracle",
               "sample": f"all {B} LJ38 starts of the workload, FP64 L-BFGS, one host thread "
                         f"pinned to core {core} ({cpu_s:.2f} s)", "cpu_model": cpu_model(),
               "host_cores": len(aff) if aff else os.cpu_count()}
        cpu["pool"] = oracle_pool(O, off, x, ro)
        cpu["candidate_sweep"] = candidate_sweep(O)
        h64, hm = fp64["host"], mixed["host"]
        parity["fp64_bitwise_frac"] = float(np.mean(
            [np.array_equal(h64["xyz"][:, off[b]:off[b + 1]], ro["xyz"][:, off[b]:off[b + 1]])
             and h64["energy"][b] == ro["energy"][b] for b in range(B)]))
        rel = np.abs(hm["energy"] - ro["energy"]) / np.abs(ro["energy"])
        parity["mixed_same_minimum_frac_1e-6"] = float(np.mean(rel <= 1e-6))
        parity["mixed_energy_rel_err_median"] = float(np.median(rel))
        parity.update(mixed_result_errors(lj, O, batch, starts, params, off, hm, stream, torch))

    # Standalone pair kernel: 256 clusters of N = 1000.
    pair = None if args.no_pair else pair_kernel(lj, large_clusters, dev, stream, torch)

    from paper_2510_25938_amd import inputs as inputs_mod
    others = None
    if not args.no_workloads:
        orc = None
        if not args.no_cpu:
            from oracle import oracle as orc
        others = workloads(lj, inputs_mod, torch, stream, orc)

    # Roofline of the dominant kernel (the persistent minimiser, mixed path):
    # algorithmic FLOP = 27 per unique pair evaluation over every evaluation of
    # the launch, divided by its average duration from HIP events.
    flops = FLOP_PER_PAIR * mixed["pair_evals"]
    achieved = flops / (mixed["kern_ms"] * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
            "frac": achieved / (PEAK_FP32 / 1e12),
            "traffic": load_traffic("minimize_mixed_lj38_1024"),
            "kernel": "minimize_kernel<mixed, 1 wave, 1 atom/lane, history in registers>",
            "note": "27 FLOP per unique pair evaluation (both phases) over the launch; "
                    "peak = FP32 vector 157.3 TFLOP/s (packed FP32 is disabled in this build)",
            "flop_per_launch": flops, "launch_ms": mixed["kern_ms"],
            "valu_issue": load_issue("minimize_mixed_lj38_1024", mixed["kern_ms"])}

    line = {
        "metric": "local minimisations/sec and LJ pair-evals/sec, FP64 vs mixed, 1 MI355X",
        "value": sm["minimisations_per_s"],
        "unit": "minimisations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sm["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair arithmetic + f64 (mixed)",
        "data": "synthetic",
        "config": {"workload": f"lj38-batch-{B}: {B} LJ38 random cube starts (side 4.0344), "
                               "L-BFGS m=10 to ||g||_2 < 1e-6, mixed + FP64 polish",
                   "candidates": B, "atoms": n, "gtol": 1e-6, "m": 10},
        "pair_evals_per_s": sm["pair_evals_per_s"],
        "mixed": sm,
        "fp64": s64,
        "speedup_mixed_vs_fp64": sm["minimisations_per_s"] / s64["minimisations_per_s"],
        "parity": parity,
        "roofline": roof,
        "cpu_baseline": cpu,
        "pair_kernel": pair,
        "workloads": others,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
