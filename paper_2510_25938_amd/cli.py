"""Command line: adaptive, parallel basin hopping of one LJ cluster on the GPU.

    python -m paper_2510_25938_amd.cli input.molden [--steps 200] [--cands 8]
        [--kT 1.0] [--step0 0.4] [--precision fp64|mixed] [--seed S]
        [--pair lj|morse] [--rho 6.0] [--sigma 1.0] [--trace steps.csv]

Reads the first geometry of input.molden (Methodology, "Initial Structures
and Input"), minimises it, runs the basin-hopping loop of the Algorithm
Overview (perturb, n candidates minimised together, select, Metropolis,
adapt every 10 steps toward 50 % acceptance) through lj_bh_step, and writes
every accepted structure to input_accepted.molden (Running the Code).  Prints
one line per step: the trial energy, the decision and the running lowest
trial energy (the three series of Fig. 2), the lowest accepted energy so far
(Fig. 3) and the step size.  --trace FILE also writes these series per step
as CSV.
"""
import argparse
import os
import sys

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("molden", help="input .molden file; its first geometry is the start")
    ap.add_argument("--steps", type=int, default=200, help="basin-hopping steps (default 200)")
    ap.add_argument("--cands", type=int, default=8,
                    help="candidates perturbed and minimised per step (default 8)")
    ap.add_argument("--kT", type=float, default=1.0,
                    help="Metropolis temperature in units of epsilon (default 1.0)")
    ap.add_argument("--step0", type=float, default=0.4,
                    help="initial step size: half the side of the perturbation cube (default 0.4)")
    ap.add_argument("--interval", type=int, default=10,
                    help="steps between step-size adaptations (default 10)")
    ap.add_argument("--target", type=float, default=0.5,
                    help="target acceptance rate of the adaptation (default 0.5)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="fp64, or FP32 pair arithmetic with FP64 L-BFGS and polish (default fp64)")
    ap.add_argument("--seed", type=int, default=2510, help="random-stream seed (default 2510)")
    ap.add_argument("--sigma", type=float, default=1.0,
                    help="length unit of the file in LJ sigma (coordinates are divided by it)")
    ap.add_argument("--pair", default="lj", choices=["lj", "morse"],
                    help="pair potential: Eq. (1) or the Morse pair (well depth 1 at r = 1)")
    ap.add_argument("--rho", type=float, default=6.0, help="Morse range")
    ap.add_argument("--quiet", action="store_true", help="no per-step lines")
    ap.add_argument("--trace", default=None,
                    help="write the per-step series (Figs. 2-3) to this CSV file")
    args = ap.parse_args(argv)

    import torch

    from . import lj
    from .inputs import aos_to_planes, planes_to_aos
    from .molden import read_first_geometry, write_geometries

    flat, syms = read_first_geometry(args.molden)
    n = len(syms)
    x = aos_to_planes(flat / args.sigma)
    batch = lj.ClusterBatch(np.array([0, n], np.int32), pair=args.pair, rho=args.rho)
    xd = torch.from_numpy(x).to("cuda")
    params = lj.lbfgs_params()
    r = lj.minimize(batch, xd, params, "fp64")
    bh = lj.bh_params(cands=args.cands, kT=args.kT, adapt_interval=args.interval,
                      target_rate=args.target, seed=args.seed)
    chain = lj.BasinHopping(batch, r["xyz"], r["energy"], bh, params, args.precision,
                            step0=args.step0, trace_steps=args.steps)
    frames, energies, rows = [], [], []
    for k in range(args.steps):
        chain.step(1)
        torch.cuda.synchronize()
        t = {key: chain.trace[key][0, k].item()
             for key in ("e_trial", "accepted", "e_best", "e_best_acc", "e_cur", "step",
                         "polish_status")}
        acc = int(t["accepted"])
        if acc:
            frames.append(planes_to_aos(chain.xyz_cur.cpu().numpy()) * args.sigma)
            energies.append(float(chain.e_cur[0].item()))
        rows.append((k + 1, t["e_trial"], acc, t["e_best"], t["e_best_acc"], t["e_cur"], t["step"],
                     int(t["polish_status"])))
        if not args.quiet:
            print(f"step {k + 1:5d}  E_trial {t['e_trial']:14.8f}  "
                  f"{'accept' if acc else 'reject'}  E_low {t['e_best']:14.8f}  "
                  f"E_best_acc {t['e_best_acc']:14.8f}  s {t['step']:.5f}", flush=True)
    if args.trace:
        with open(args.trace, "w") as fh:
            fh.write("step,e_trial,accepted,e_lowest_trial,e_best_accepted,e_current,step_size,"
                     "polish_status\n")
            for row in rows:
                fh.write(f"{row[0]},{row[1]:.12f},{row[2]},{row[3]:.12f},{row[4]:.12f},"
                         f"{row[5]:.12f},{row[6]:.10f},{row[7]}\n")
    out = os.path.splitext(args.molden)[0] + "_accepted.molden"
    write_geometries(out, frames, energies, syms)
    print(f"{len(frames)} accepted structures -> {out}; lowest accepted "
          f"{chain.e_best_acc[0].item():.8f}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
