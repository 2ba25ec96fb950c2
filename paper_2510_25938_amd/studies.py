"""Studies built on lj_bh_step (host glue, no new kernels).

scaling: the paper's candidate-count experiment (Results, Figs. 4-5): one
    basin-hopping chain with n concurrent candidates per step, n in
    {1, 2, 4, ..., 64}; reports wall time per step, time to reach a target
    energy, and speedup / efficiency relative to n = 1.  Many independent
    chains are run side by side (a batch of identical chains with different
    seeds) so the time to target is averaged over chains.
    The default target is the chain's global minimum as computed from its
    symmetric structure (LJ13 icosahedron -44.326801, LJ38 truncated
    octahedron -173.928427).
lj38: global search for LJ38 (Results, Fig. 6): many chains from random
    starts until one reaches the truncated-octahedral global minimum; the hit
    is confirmed by its energy (-173.928427, Wales & Doye 1997) and by the
    O_h shell structure (6 + 8 + 24 atoms at three radii).

    python -m paper_2510_25938_amd.studies scaling [--atoms 38] [--steps 200]
    python -m paper_2510_25938_amd.studies lj38 [--chains 512] [--seconds 60]
"""
import argparse
import json
import sys
import time

import numpy as np

LJ38_GLOBAL = -173.928427
LJ13_GLOBAL = -44.326801
GLOBAL_MINIMA = {13: LJ13_GLOBAL, 38: LJ38_GLOBAL}


def _setup(n_atoms, chains, seed, torch, lj, inputs):
    off, x = inputs.random_starts([n_atoms] * chains, seed)
    b = lj.ClusterBatch(off)
    r = lj.minimize(b, torch.from_numpy(x).cuda(), lj.lbfgs_params(), "fp64")
    torch.cuda.synchronize()
    return b, r


def scaling(n_atoms=38, steps=200, chains=64, cands=(1, 2, 4, 8, 16, 32, 64), kT=0.8,
            precision="mixed", target="global", seed=2510, traces=None):
    """Steps/s and time to target for one chain per candidate count (averaged over
    `chains` independent chains run side by side).  target="global" uses the
    computed global minimum of LJ13 or LJ38 (None: no target).  With `traces`
    (a dict), the start minima and every candidate count's per-step trace are
    stored in it."""
    import torch

    from . import inputs, lj
    if target == "global":
        target = GLOBAL_MINIMA.get(n_atoms)
    b, r = _setup(n_atoms, chains, seed, torch, lj, inputs)
    if traces is not None:
        traces["offset"] = b.offset_host
        traces["xyz_min"] = r["xyz"].cpu().numpy()
        traces["e_min"] = r["energy"].cpu().numpy()
    out = []
    stream = torch.cuda.Stream()
    for n in cands:
        ch = lj.BasinHopping(b, r["xyz"], r["energy"], lj.bh_params(cands=n, kT=kT, seed=seed + n),
                             lj.lbfgs_params(), precision, trace_steps=steps)
        with torch.cuda.stream(stream):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ch.step(steps, stream=stream)
            e1.record(stream)
            stream.synchronize()
        ms = e0.elapsed_time(e1)
        best = ch.trace["e_best"].cpu().numpy()  # running lowest per chain and step
        if traces is not None:
            traces[n] = {k: v.cpu().numpy() for k, v in ch.trace.items() if v is not None}
            traces[n]["seed"] = seed + n
        row = {"cands": n, "ms_per_step": ms / steps, "final_best_mean": float(best[:, -1].mean())}
        if target is not None:
            hit = best <= target + 1e-6
            first = np.where(hit.any(axis=1), hit.argmax(axis=1) + 1, -1)
            row["chains_hit"] = int((first > 0).sum())
            row["median_steps_to_target"] = float(np.median(first[first > 0])) if (first > 0).any() else None
            row["median_ms_to_target"] = (row["median_steps_to_target"] * ms / steps
                                          if row["median_steps_to_target"] else None)
        out.append(row)
    base = out[0]["ms_per_step"]
    for row in out:
        # work per step grows with n: speedup = n * t(1) / t(n) (candidates per unit time)
        row["speedup"] = row["cands"] * base / row["ms_per_step"]
        row["efficiency"] = row["speedup"] / row["cands"]
    return out


def o_h_shells(xyz):
    """True if the structure has the LJ38 truncated-octahedron shells 6 + 8 + 24."""
    X = np.asarray(xyz).T
    rad = np.sort(np.linalg.norm(X - X.mean(axis=0), axis=1))
    if len(rad) != 38:
        return False
    shells = (rad[:6], rad[6:14], rad[14:])
    tight = all(np.ptp(s) < 1e-4 for s in shells)
    gaps = rad[6] - rad[5] > 0.1 and rad[14] - rad[13] > 0.1
    return bool(tight and gaps)


def lj38(chains=512, cands=8, seconds=60.0, chunk=50, kT=0.8, precision="mixed", seed=38,
         max_steps=None):
    """Run many LJ38 chains until one finds the global minimum, time runs out or
    max_steps steps are done.  On a hit, the result holds the chain, its best
    structure (planes) and the O_h shell check."""
    import torch

    from . import inputs, lj
    b, r = _setup(38, chains, seed, torch, lj, inputs)
    ch = lj.BasinHopping(b, r["xyz"], r["energy"], lj.bh_params(cands=cands, kT=kT, seed=seed),
                         lj.lbfgs_params(), precision)
    t0 = time.perf_counter()
    steps = 0
    result = {"chains": chains, "cands": cands, "precision": precision, "found": False}
    while time.perf_counter() - t0 < seconds and (max_steps is None or steps < max_steps):
        ch.step(chunk)
        torch.cuda.synchronize()
        steps += chunk
        best = ch.e_best_acc.cpu().numpy()
        k = int(np.argmin(best))
        result.update(steps=steps, seconds=time.perf_counter() - t0, lowest=float(best[k]))
        if best[k] <= LJ38_GLOBAL + 1e-6:
            off = b.offset_host
            xb = ch.xyz_best.cpu().numpy()[:, off[k]:off[k + 1]]
            result.update(found=True, chain=k, o_h=o_h_shells(xb), xyz=xb.tolist())
            break
    return result


def main(argv=None):
    ap = argparse.ArgumentParser(description="basin-hopping studies on the GPU")
    sub = ap.add_subparsers(dest="study", required=True)
    s = sub.add_parser("scaling")
    s.add_argument("--atoms", type=int, default=38)
    s.add_argument("--steps", type=int, default=200)
    s.add_argument("--chains", type=int, default=64)
    s.add_argument("--precision", default="mixed")
    s.add_argument("--target", default="global",
                   help='"global" (computed LJ13 / LJ38 minimum), "none" or an energy')
    g = sub.add_parser("lj38")
    g.add_argument("--chains", type=int, default=512)
    g.add_argument("--cands", type=int, default=8)
    g.add_argument("--seconds", type=float, default=60.0)
    g.add_argument("--precision", default="mixed")
    args = ap.parse_args(argv)
    if args.study == "scaling":
        target = {"global": "global", "none": None}.get(args.target)
        if target is None and args.target != "none":
            target = float(args.target)
        for row in scaling(args.atoms, args.steps, args.chains, precision=args.precision,
                           target=target):
            print(json.dumps(row), flush=True)
    else:
        res = lj38(args.chains, args.cands, args.seconds, precision=args.precision)
        res.pop("xyz", None)
        print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
