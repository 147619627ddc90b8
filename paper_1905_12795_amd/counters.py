"""Driver for hardware-counter collection on the finite-difference kernel.

Hardware counters (rocprofv3 --pmc) serialise every dispatch, so a full
fitness evaluation (thousands of launches) is too slow to profile that way.
This driver sets up a workload's whole batch as bench.py does (the full
workload: 128 particles x 32 shots on the 601 x 1841 grid at 5 m; or the
realistic one: 32 particles x 16 shots on the 301 x 921 grid) and runs one
untimed and `reps` timed launches of the finite-difference kernel through
empso_time_tuning, after one device-to-device copy of a known size whose
counter readings calibrate the byte counters. Usage:

  rocprofv3 --pmc FETCH_SIZE -- python3 paper_1905_12795_amd/counters.py --workload full --bz 240 --tsteps 4
"""
import argparse
import json
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
    ap.add_argument("--workload", default="full", choices=("full", "realistic"))
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

    g = config(args.workload)
    npart = args.particles or g["particles"]
    prob = fd.Problem(g)
    obs = torch.zeros((prob.nshots, prob.nt, prob.nrec), dtype=torch.float32, device="cuda")
    X = uniform_particles(npart, g["node_lo"], g["node_hi"], g["particle_seed"])
    fb = fd.FitnessBatch([prob], [obs], [0] * npart)
    tu = fd.default_tuning()
    tu.bz, tu.tsteps = args.bz, args.tsteps
    us = fb.time_tuning(X, tu, reps=args.reps)
    points = prob.info.Nz * prob.info.Nx * prob.nshots * npart
    print(json.dumps({"workload": args.workload, "particles": npart,
                      "copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
                      "kernel_launches": 1 + args.reps, "tuning": tu.as_dict(),
                      "points_per_launch": points, "updates_per_launch": points * args.tsteps,
                      "us_per_time_step": us}), flush=True)


if __name__ == "__main__":
    main()
