"""Benchmark of the fitness-evaluation hot path on one MI355X.

One step = one elitist-PSO iteration of the realistic workload: the host FP64
swarm hands 32 particles (5 x 12 control nodes each) to the HIP library, which
interpolates each onto the 301 x 921 grid (10 m, 40-point absorbing layer),
models all 16 shots of every particle (512 runs, 8114 time steps each) and
reduces the l2 misfits to 32 fitness values; the swarm then moves (Eq. 1-2
plus elitist mutation). Observed data and inputs are resident in HBM before
the timed region.

Printed JSON line: fitness evals/s (particles fully evaluated per second),
Gpt-updates/s, the HBM roofline of the dominant stencil kernel, and the
oracle's throughput on the host cores over a bounded sample.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per grid-point update of the scheme: read u^n and
# u^{n-1}, write u^{n+1} and u^n (FP32). The coefficient field is
# shared by the 16 shots of a particle and excluded. A launch that advances T
# time steps performs T updates per point.
BYTES_PER_UPDATE = 16
METRIC = "fitness evals/s and Gpt-updates/s on 1 MI355X; % HBM peak; surrogate vs plain"


def kernel_source_hash():
    """Hash of the stencil kernel's source text: the RunDesc descriptor it
    reads plus everything from its memory-access helpers to the end of the
    k_tb template. Edits to the file's other kernels and entry points leave
    the committed counter measurements valid."""
    src = open(os.path.join(ROOT, "paper_1905_12795_amd", "csrc", "fd.hip"), "rb").read()
    a = src.index(b"struct RunDesc {")
    a2 = src.index(b"};", a) + 2
    b = src.index(b"// Scalar and vector accesses through explicit address spaces")
    c = src.index(b"// Sample u^n (held in buffer `par`)")
    return hashlib.sha256(src[a:a2] + src[b:c]).hexdigest()[:16]


def strip_rows(Nz, bz, T):
    """Height of the z-strips the library launches for tile height bz and depth
    T on a grid of Nz padded rows (its tiling rule: about bz rows, balanced,
    rounded so that 8(T-1) fill steps plus the rows make whole 10-step
    blocks). Counter summaries apply to the launched tiles, so two tunings
    with the same depth and strips share them."""
    n = -(-Nz // bz)
    fill = 8 * (T - 1)
    return -(-(-(-Nz // n) + fill) // 10) * 10 - fill


def _counters_apply(d, per_launch_updates, tu, Nz):
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return False
    if d.get("updates_per_launch") != per_launch_updates:
        return False
    t = d.get("tuning", {})
    if t.get("tsteps") != tu.tsteps or "bz" not in t:
        return False
    return strip_rows(Nz, t["bz"], tu.tsteps) == strip_rows(Nz, tu.bz, tu.tsteps)


def measured_traffic(per_launch_updates, tu, Nz):
    """HBM bytes per stencil launch from the committed counter summary, if it
    was taken on the current kernel source with this tuning; else None."""
    path = os.path.join(ROOT, "profiles", "k_tb_realistic_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    return d.get("hbm_bytes_per_launch") if _counters_apply(d, per_launch_updates, tu, Nz) else None


# VALU issue capacity of the GPU: 256 compute units x 4 SIMDs, each issuing
# one wave64 FP32 vector instruction per 4 cycles (16 lanes), at 2.4 GHz.
SIMDS = 256 * 4
CLOCK_HZ = 2.4e9
CYCLES_PER_VALU = 4


def measured_valu(per_launch_updates, tu, Nz):
    """Wave-level VALU instructions per stencil launch (SQ_INSTS_VALU) from the
    committed counter summary, if it was taken on the current kernel source
    with this tuning; else None."""
    path = os.path.join(ROOT, "profiles", "k_tb_realistic_valu.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    return d.get("valu_instructions_per_launch") if _counters_apply(d, per_launch_updates, tu, Nz) else None


def cpu_baseline(geom, dt, nt, threads, steps):
    """Oracle throughput on the host: the forward runs of 1 particle x all shots
    over the first `steps` time steps (all of them by default: one complete
    evaluation; the misfit's own cost is negligible next to the modelling)."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import fd as ofd
    from workloads.configs import true_model

    op = ofd.Problem(geom, dt=dt, nt=nt)
    vel = ofd.pad_edge(true_model(geom), op.nbl)
    wav = op.wavelet[:steps]

    def run(s):
        spts = ofd.point_weights(op.src[s], op.dz, op.dx, op.nz, op.nx, op.nbl)
        return ofd.forward_run(vel, op.damp, op.dz, op.dx, op.dt, steps, wav, spts, op.rec_pts, op.nrec)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(run, range(op.nshots)))
    el = time.perf_counter() - t0
    Nz, Nx = op.nz + 2 * op.nbl, op.nx + 2 * op.nbl
    upd = op.nshots * Nz * Nx * (steps - 1)
    rate = upd / el
    per_eval = op.nshots * Nz * Nx * (nt - 1)
    return {"value": rate / per_eval, "unit": "fitness evals/s", "cores": threads, "kind": "oracle",
            "sample": "1 particle x %d shots x %d of %d time steps (FP64 C oracle, one thread per "
                      "shot); %.3g s for %.3g point-updates = %.3g Gpt-updates/s, as fitness evaluations "
                      "of the whole record" % (op.nshots, steps, nt, el, upd, rate / 1e9),
            "gpt_updates_per_s": rate / 1e9, "seconds": el}


def gradient_report(prob, dobs, reps=3):
    """Misfit gradient of a smooth starting model over the same 16 shots
    (outside the timed region): seconds per gradient with HIP events, and the
    point-update rate of its three passes (forward with checkpoints, segment
    recomputation, adjoint)."""
    import torch

    from paper_1905_12795_amd import fd

    nz, nx = prob.info.nz, prob.info.nx
    z = np.arange(nz, dtype=np.float64)[:, None] / (nz - 1)
    v0 = torch.tensor(np.repeat(1500.0 + 4000.0 * z, nx, axis=1), dtype=torch.float32, device="cuda")
    ws = fd.workspace(fd.lib.empso_gradient_workspace_bytes(prob.handle, 0))
    fd.gradient(prob, v0, dobs, 0, ws)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        mis, _g = fd.gradient(prob, v0, dobs, 0, ws)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1000.0 / reps
    upd = 3 * prob.updates_per_run * prob.nshots
    return {"workload": "realistic geometry, 16 shots, nt %d, a linear 1500-5500 m/s starting model" % prob.nt,
            "seconds_per_gradient": sec, "gpt_updates_per_s_three_passes": upd / sec / 1e9,
            "misfit": float(mis), "workspace_gib": ws.numel() / 2 ** 30}


def _strict(v):
    """The result with non-finite floats replaced by None (strict JSON)."""
    if isinstance(v, dict):
        return {k: _strict(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [_strict(x) for x in v]
    if isinstance(v, float) and not math.isfinite(v):
        return None
    return v


def surrogate_report(seeds=(1, 2, 3, 4), iters=30):
    """Surrogate vs plain (outside the timed region): the seed average of the
    mini search's best-misfit curves, plus the network's inference on 1024
    candidates and one training step (batch 256) timed with HIP events."""
    import torch

    from paper_1905_12795_amd import fd, search
    from paper_1905_12795_amd.surrogate import Surrogate
    from workloads.configs import config, true_model
    from workloads.models import uniform_particles

    g = config("mini")
    prob = fd.Problem(g)
    dobs = search.observed_data(prob, true_model(g))
    hp = search.mean_history([search.run(g, dobs, prob, iters, "plain", seed=s) for s in seeds])
    hs = search.mean_history([search.run(g, dobs, prob, iters, "screened", seed=s, K=16) for s in seeds])
    e, t = search.evals_to_reach(hs, 1.01 * hp[-1]["best"])
    finite = lambda v: v if np.isfinite(v) else None          # noqa: E731  (strict JSON)
    rep = {"workload": "mini: 101x301 at 10 m, 4 shots, 3x6 nodes, 32 particles, %d iterations, K = 16; "
                       "curves averaged over seeds %s" % (iters, ",".join(map(str, seeds))),
           "plain_final_misfit": hp[-1]["best"], "plain_fd_evals": hp[-1]["evaluations"],
           "plain_wall_s": hp[-1]["wall_s"], "screened_final_misfit": hs[-1]["best"],
           "screened_fd_evals_to_plain_final": finite(e), "screened_wall_s_to_plain_final": finite(t)}
    # network timings at the surrogate workload's shape (D = 60, H = 256)
    gs = config("surrogate")
    sur = Surrogate(gs["node_lo"], gs["node_hi"], seed=0)
    X = uniform_particles(2048, gs["node_lo"], gs["node_hi"], 0)
    sur.add(X, np.exp(np.random.default_rng(0).normal(5, 1, 2048)))
    Xc = torch.tensor(uniform_particles(1024, gs["node_lo"], gs["node_hi"], 1), dtype=torch.float32, device="cuda")
    idx = torch.arange(256, dtype=torch.int32, device="cuda")
    for _ in range(3):
        sur.net.predict(Xc)
        sur.net.train_step(sur.X, sur.f, idx, sur.mu, sur.sigma, 1e-4)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    reps = 20
    e0.record()
    for _ in range(reps):
        sur.net.predict(Xc)
    e1.record()
    for _ in range(reps):
        sur.net.train_step(sur.X, sur.f, idx, sur.mu, sur.sigma, 1e-4)
    e2.record()
    torch.cuda.synchronize()
    D, H = sur.D, sur.net.H
    mac = D * H + 2 * H * H + H
    pred_ms = e0.elapsed_time(e1) / reps
    train_ms = e1.elapsed_time(e2) / reps
    rep.update({"predict_1024_ms": pred_ms, "predict_tflops": 2 * 1024 * mac / (pred_ms * 1e-3) / 1e12,
                "train_step_256_ms": train_ms, "train_tflops": 3 * 2 * 256 * mac / (train_ms * 1e-3) / 1e12,
                "bf16_mfma_peak_tflops": 2500.0})
    return rep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate-vs-plain report")
    ap.add_argument("--no-gradient", action="store_true", help="skip the misfit-gradient report")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="time steps of the oracle sample (0: the whole record, one complete evaluation)")
    ap.add_argument("--bz", type=int, default=None, help="fix the tile height (default: autotune)")
    ap.add_argument("--tsteps", type=int, default=None, help="fix the temporal-blocking depth")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the runs shard trivially by particle or shot; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1905_12795_amd import fd
    from paper_1905_12795_amd.pso import EMPSO
    from workloads.configs import config, true_model

    dev = "cuda"
    g = config("realistic")
    prob = fd.Problem(g)
    vp = torch.tensor(true_model(g), dtype=torch.float32, device=dev)
    dobs = fd.forward_shots(prob, vp)
    swarm = EMPSO(g["node_lo"], g["node_hi"], g["particles"], gen=10, seed=g["particle_seed"])
    fb = fd.FitnessBatch([prob], [dobs], [0] * g["particles"])
    if args.bz or args.tsteps:
        tu = fd.default_tuning()
        tu.bz = args.bz or tu.bz
        tu.tsteps = args.tsteps or tu.tsteps
        fb.tuning = tu
        tuned = None
    else:
        tuned = fb.autotune(swarm.ask())      # setup, untimed
        tu = fb.tuning
    T = tu.tsteps
    nsteps = prob.nt - 1
    n_main, n_tail = nsteps // T, nsteps % T
    points = fb.updates // nsteps             # grid points of all runs (one update each per time step)
    upd_per_step = fb.updates                 # one step = one fitness call = all time steps of all runs
    upd_per_launch = points * T

    def step():
        f = fb(swarm.ask())
        swarm.tell(f.cpu().numpy())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        x = swarm.ask()
        ev0[k].record()
        f = fb(x)
        ev1[k].record()
        swarm.tell(f.cpu().numpy())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = [a.elapsed_time(b) for a, b in zip(ev0, ev1)]
    ms_step = 1000.0 * wall / args.steps
    evals_per_s = g["particles"] * args.steps / wall
    gpt = upd_per_step * args.steps / wall / 1e9
    # Dominant kernel: the T-step launch. The fitness call is one graph on the
    # current stream: the events around it bound its launches' average
    # duration from above (the call also holds a few tiny kernels and
    # (nt-1) mod T single-step launches, counted as 1/T of a launch each).
    launch_s = (np.mean(gpu_ms) / 1000.0) / (n_main + n_tail / T)
    # isolated timing of the same kernel (HIP events on the launch stream)
    iso_us_step = fb.time_tuning(swarm.ask(), tu, reps=8)
    alg = upd_per_launch * BYTES_PER_UPDATE
    achieved = alg / launch_s / 1e9
    traffic = measured_traffic(upd_per_launch, tu, prob.info.Nz)
    valu = measured_valu(upd_per_launch, tu, prob.info.Nz)
    out = {
        "metric": METRIC, "value": evals_per_s, "unit": "fitness evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "realistic: 301x921 grid at 10 m + 40-point layer, 32 particles x 16 "
                               "shots (512 runs), 461 receivers, 5 Hz Ricker, 3 s (nt %d), 5x12 nodes, "
                               "one EMPSO iteration per step" % prob.nt,
                   "runs_per_step": g["particles"] * prob.nshots, "nt": prob.nt,
                   "tuning": tu.as_dict(), "autotuned": tuned is not None},
        "gpt_updates_per_s": gpt,
        "fitness_call_ms": float(np.mean(gpu_ms)),
        "best_fitness": float(swarm.fg),
        "roofline": {"bound": "hbm", "kernel": "k_tb<%d> (tiles of about %d rows)" % (T, tu.bz), "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": alg, "updates_per_launch": upd_per_launch,
                     "bytes_per_update": BYTES_PER_UPDATE, "time_steps_per_launch": T,
                     "avg_launch_us": launch_s * 1e6, "isolated_launch_us": iso_us_step * T,
                     "measured_frac": None if traffic is None else traffic / launch_s / 1e9 / HBM_PEAK_GBS,
                     # the kernel's binding limit: share of the VALU issue capacity its
                     # counted instructions take over the measured launch time
                     "valu_instructions_per_launch": valu,
                     "valu_issue_frac": None if valu is None else
                     valu * CYCLES_PER_VALU / (SIMDS * CLOCK_HZ * launch_s)},
    }
    if not args.no_gradient:
        out["gradient"] = gradient_report(prob, dobs)
    if not args.no_surrogate:
        out["surrogate"] = surrogate_report()
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(g, prob.dt, prob.nt, threads, args.cpu_steps or prob.nt)
    print(json.dumps(_strict(out), allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
