"""Driver for hardware-counter collection on the finite-difference kernel.

Hardware counters (rocprofv3 --pmc) serialise every dispatch, so a full
fitness evaluation (thousands of launches) is too slow to profile that way.
This driver sets up a workload's whole batch as bench.py does (the full
workload: 128 particles x 32 shots on the 601 x 1841 grid at 5 m; the
realistic one: 32 particles x 16 shots on the 301 x 921 grid; or the
three-size batch: 64 particles x 16 shots, particle p on grid p mod 3 of
201 x 601, 301 x 921 and 401 x 1201, one dt and nt) and runs one
untimed and `reps` timed launches of the finite-difference kernel through
empso_time_tuning, after one device-to-device copy of a known size whose
counter readings calibrate the byte counters. Usage:

  rocprofv3 --pmc FETCH_SIZE -- python3 paper_1905_12795_amd/counters.py --workload full --bz 240 --tsteps 4
"""
import argparse
import json
import math
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1905_12795_amd import fd  # noqa: E402
from workloads.configs import config  # noqa: E402
from workloads.models import uniform_particles  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="full", choices=("full", "realistic", "batched"))
    ap.add_argument("--particles", type=int, default=0, help="particles of the batch (0: the workload's)")
    ap.add_argument("--bz", type=int, default=160)
    ap.add_argument("--tsteps", type=int, default=3)
    ap.add_argument("--reps", type=int, default=4)
    ap.add_argument("--copy-mib", type=int, default=1024)
    args = ap.parse_args()

    n = args.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    geoms = config(args.workload)
    geoms = geoms if isinstance(geoms, list) else [geoms]
    g = geoms[0]
    npart = args.particles or g["particles"]
    probs = [fd.Problem(q) for q in geoms]
    if len({p.nt for p in probs}) != 1:          # one batch shares dt and nt
        dt = min(p.dt for p in probs)
        nt = int(math.floor(g["tmax"] / dt + 1e-9)) + 1
        probs = [fd.Problem(q, dt=dt, nt=nt) for q in geoms]
    obs = [torch.zeros((p.nshots, p.nt, p.nrec), dtype=torch.float32, device="cuda") for p in probs]
    pop = [k % len(probs) for k in range(npart)]
    X = uniform_particles(npart, g["node_lo"], g["node_hi"], g["particle_seed"])
    fb = fd.FitnessBatch(probs, obs, pop)
    tu = fd.default_tuning()
    tu.bz, tu.tsteps = args.bz, args.tsteps
    us = fb.time_tuning(X, tu, reps=args.reps)
    points = sum(probs[q].info.Nz * probs[q].info.Nx * probs[q].nshots for q in pop)
    print(json.dumps({"workload": args.workload, "particles": npart,
                      "copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
                      "kernel_launches": 1 + args.reps, "tuning": tu.as_dict(),
                      "points_per_launch": points, "updates_per_launch": points * args.tsteps,
                      "us_per_time_step": us}), flush=True)


if __name__ == "__main__":
    main()
