"""Benchmark of the fitness-evaluation hot path on one MI355X.

Headline workload: the full search at scale, one EMPSO iteration of 128
particles x 32 shots on the 601 x 1841 grid at 5 m (681 x 1921 with the
40-point absorbing layer), 921 receivers, 6 Hz Ricker, 4 s record (nt 21,636),
8 x 20 control nodes: 4,096 forward runs, about 93 GB of wavefields resident
in HBM. One iteration is 1.2e14 point-updates (over two minutes on the GPU),
so one bench step is one block of time steps of that evaluation: all 4,096
runs advance by `block` (about 400) time steps through the library's
block-wise fitness entry point, with source injection, receiver residuals and
their accumulation fused in the stencil kernel. The block that reaches the
last time step takes the final sample, reduces the 128 fitness values,
returns them to the host swarm (Eq. 1-2 and elitist mutation in FP64) and the
next block starts the next iteration (interpolation of the new particles onto
the grid, coefficient fields). Observed data and all inputs are resident in
HBM before the timed region.

value = fitness evaluations per second (a particle with all its 32 shots over
the whole record), derived from the measured point-update rate: the steps
perform a known fraction of the iteration's updates.

Also reported: the realistic workload (32 particles x 16 shots, 301 x 921) and
the three-size batch (64 particles x 16 shots over 201 x 601, 301 x 921,
401 x 1201) as whole iterations per call (HIP graph replay); the roofline of
the dominant stencil kernel; the misfit gradient; the surrogate network; and
the FP64 oracle's throughput on the host cores over a bounded sample.
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
# Algorithmic HBM bytes per grid-point update of a single-pass scheme: read u^n
# and u^{n-1}, write u^{n+1} and u^n (FP32); the coefficient field is shared by
# all shots of a particle and excluded. Temporal blocking of depth T performs T
# updates per point per launch, so this "effective" rate may exceed the peak.
BYTES_PER_UPDATE = 16
METRIC = "fitness evals/s and Gpt-updates/s on 1 MI355X; % HBM peak; surrogate vs plain"

# VALU issue capacity: 256 compute units x 4 SIMDs, each issuing one wave64
# FP32 vector instruction per 4 cycles (16 lanes per cycle), at 2.4 GHz: 39.3 T
# lane-operations/s. (The published 157.3 TFLOP/s FP32 vector figure is the
# same issue rate with packed two-wide FMAs counted as 4 FLOPs per lane-op.)
SIMDS = 256 * 4
LANES_PER_CYCLE = 16
CLOCK_HZ = 2.4e9
CYCLES_PER_VALU = 4
VALU_PEAK_GOPS = SIMDS * LANES_PER_CYCLE * CLOCK_HZ / 1e9
# Algorithmic VALU operations of one point-update as the scheme is evaluated
# (one operation per add, multiply, fused multiply-add or reciprocal): the
# Laplacian as a sum of small terms (19: three adds per neighbour distance
# for its z and x pairs, one FMA per distance with its weight, and one FMA per
# distance but the farthest subtracting the centre), the increment's
# difference, its FMA with the coefficient, and the update (22); a damped
# point adds the damping sum, 1 + a, its reciprocal, 1 - a, and two
# multiplies (28).
OPS_UNDAMPED = 22
OPS_DAMPED = 28


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


def committed_counter(name, key, per_launch_updates, tu, Nz):
    """A per-launch figure from a committed counter summary (profiles/<name>:
    one measurement, or several under "entries", one per tiling), if one was
    taken on the current kernel source with this tuning's tiles; else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    for e in d.get("entries", [d]):
        if _counters_apply(e, per_launch_updates, tu, Nz):
            return e.get(key)
    return None


def damped_share(info):
    """Share of a run's padded points inside the absorbing layer (a != 0)."""
    phys = info.nz * info.nx
    return 1.0 - phys / float(info.Nz * info.Nx)


def alg_ops_per_update(info):
    s = damped_share(info)
    return OPS_UNDAMPED * (1.0 - s) + OPS_DAMPED * s


def cpu_baseline(geom, dt, nt, steps, threads):
    """The FP64 oracle on the host over a bounded sample of the workload: the
    first `steps` time steps of `threads` shots of one particle (the true
    model), one shot per thread, and of one shot on one thread; the
    per-update rate is extrapolated to whole fitness evaluations (all shots,
    all nt - 1 steps)."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import fd as ofd
    from workloads.configs import true_model

    op = ofd.Problem(geom, dt=dt, nt=nt)
    vel = ofd.pad_edge(true_model(geom), op.nbl)
    wav = op.wavelet[:steps]

    def run(s):
        spts = ofd.point_weights(op.src[s], op.dz, op.dx, op.nz, op.nx, op.nbl)
        return ofd.forward_run(vel, op.damp, op.dz, op.dx, op.dt, steps, wav, spts, op.rec_pts, op.nrec)

    Nz, Nx = op.nz + 2 * op.nbl, op.nx + 2 * op.nbl
    nsh = min(threads, op.nshots)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(run, range(nsh)))
    el = time.perf_counter() - t0
    t0 = time.perf_counter()
    run(0)
    el1 = time.perf_counter() - t0
    upd = nsh * Nz * Nx * (steps - 1)
    rate = upd / el
    rate1 = Nz * Nx * (steps - 1) / el1
    per_eval = op.nshots * Nz * Nx * (nt - 1)
    return {"value": rate / per_eval, "unit": "fitness evals/s", "cores": threads, "kind": "oracle",
            "nproc": os.cpu_count(),
            "sample": "FP64 C oracle (triple loop), true model, the first %d of %d time steps of %d of %d "
                      "shots, one shot per thread on %d threads (%.1f s, %.3g point-updates), and one shot "
                      "on one thread (%.1f s); fitness evals/s extrapolated from the per-update rate to %d "
                      "shots x %d steps" % (steps, nt, nsh, op.nshots, threads, el, upd, el1, op.nshots, nt - 1),
            "extrapolated": True,
            "gpt_updates_per_s": rate / 1e9, "single_core_gpt_updates_per_s": rate1 / 1e9,
            "single_core_fitness_evals_per_s": rate1 / per_eval, "seconds": el + el1}


def gradient_report(prob, dobs, reps=3):
    """Misfit gradient of a smooth starting model over the realistic
    geometry's 16 shots (outside the timed region): seconds per gradient with
    HIP events and the point-update rate of its passes, at the default
    checkpoint interval (forward pass with checkpoints, segment recomputation,
    adjoint: three passes) and, when the GPU has the memory, with every time
    level kept (one forward pass and the adjoint)."""
    import torch

    from paper_1905_12795_amd import fd

    nz, nx = prob.info.nz, prob.info.nx
    z = np.arange(nz, dtype=np.float64)[:, None] / (nz - 1)
    v0 = torch.tensor(np.repeat(1500.0 + 4000.0 * z, nx, axis=1), dtype=torch.float32, device="cuda")
    out = {"workload": "realistic geometry, 16 shots, nt %d, a linear 1500-5500 m/s starting model" % prob.nt}
    for name, K, passes in (("checkpointed", 0, 3), ("every_level_kept", prob.nt - 1, 2)):
        need = fd.lib.empso_gradient_workspace_bytes(prob.handle, K)
        if K and torch.cuda.mem_get_info()[0] < need + (8 << 30):
            out[name] = {"skipped": "needs %.1f GB" % (need / 1e9)}
            continue
        ws = fd.workspace(need)
        fd.gradient(prob, v0, dobs, K, ws)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            mis, _g = fd.gradient(prob, v0, dobs, K, ws)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1000.0 / reps
        upd = passes * prob.updates_per_run * prob.nshots
        out[name] = {"checkpoint_every": K, "seconds_per_gradient": sec,
                     "gpt_updates_per_s_over_passes": upd / sec / 1e9, "passes": passes,
                     "misfit": float(mis), "workspace_gib": ws.numel() / 2 ** 30}
        del ws
        torch.cuda.empty_cache()
    return out


def _strict(v):
    """The result with non-finite floats replaced by None (strict JSON)."""
    if isinstance(v, dict):
        return {k: _strict(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [_strict(x) for x in v]
    if isinstance(v, float) and not math.isfinite(v):
        return None
    return v


def surrogate_report(seeds=(1, 2, 3, 4), iters=30, rank_seeds=tuple(range(1, 9))):
    """Surrogate vs plain (outside the timed region): the seed average of the
    mini search's best-misfit curves; the network's choice among 16 candidate
    moves against a random choice among the same candidates (all evaluated by
    the FD fitness, after 6, 12 and 18 iterations of online training, with
    95 % intervals over the seeds); and the network's inference on 1024
    candidates and one training step (batch 256) timed with HIP events."""
    import torch

    from paper_1905_12795_amd import experiments, fd, search
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
    _rows, rk = experiments.surrogate_ranking("mini", rank_seeds, (6, 12, 18), 16, emit=False)
    rep["candidate_ranking"] = dict(rk, note="per seed: Spearman of prediction and FD misfit over all 512 "
                                             "candidates; log-misfit gain of the network's pick over a random "
                                             "pick among the same candidates, and of the best candidate")
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


def whole_iterations(name, calls):
    """Whole EMPSO iterations of a smaller workload through the one-call
    fitness path (HIP graph replay), autotuned: seconds per iteration from
    HIP events around each fitness call, Gpt-updates/s and fitness evals/s."""
    import torch

    from paper_1905_12795_amd import fd
    from paper_1905_12795_amd.pso import EMPSO
    from workloads.configs import config, true_model

    geoms = config(name)
    geoms = geoms if isinstance(geoms, list) else [geoms]
    probs = [fd.Problem(g) for g in geoms]
    if len({p.nt for p in probs}) != 1:          # one batch shares dt and nt
        dt = min(p.dt for p in probs)
        nt = int(math.floor(geoms[0]["tmax"] / dt + 1e-9)) + 1
        probs = [fd.Problem(g, dt=dt, nt=nt) for g in geoms]
    obs = [fd.forward_shots(p, torch.tensor(true_model(g), dtype=torch.float32, device="cuda"))
           for p, g in zip(probs, geoms)]
    g0 = geoms[0]
    npart = g0["particles"]
    pop = [p % len(probs) for p in range(npart)]
    swarm = EMPSO(g0["node_lo"], g0["node_hi"], npart, gen=10, seed=g0["particle_seed"])
    fb = fd.FitnessBatch(probs, obs, pop)
    fb.autotune(swarm.ask())
    swarm.tell(fb(swarm.ask()).cpu().numpy())
    torch.cuda.synchronize()
    e0 = [torch.cuda.Event(enable_timing=True) for _ in range(calls)]
    e1 = [torch.cuda.Event(enable_timing=True) for _ in range(calls)]
    t0 = time.perf_counter()
    for k in range(calls):
        x = swarm.ask()
        e0[k].record()
        f = fb(x)
        e1[k].record()
        swarm.tell(f.cpu().numpy())
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / calls
    sec = float(np.mean([a.elapsed_time(b) for a, b in zip(e0, e1)])) / 1000.0
    upd = fb.updates
    phys = sum(probs[q].info.nz * probs[q].info.nx * probs[q].nshots * (probs[q].nt - 1) for q in pop)
    out = {"grids": [[p.info.nz, p.info.nx] for p in probs], "particles": npart,
           "runs": int(sum(probs[q].nshots for q in pop)), "nt": probs[0].nt, "calls": calls,
           "seconds_per_iteration": wall, "fitness_call_s": sec,
           "fitness_evals_per_s": npart / wall, "gpt_updates_per_s": upd / wall / 1e9,
           "gpt_updates_per_s_physical": phys / wall / 1e9, "tuning": fb.tuning.as_dict()}
    del fb
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--block", type=int, default=400, help="time steps per bench step (rounded to the depth)")
    ap.add_argument("--particles", type=int, default=0, help="particles of the headline batch (0: all 128)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate-vs-plain report")
    ap.add_argument("--no-gradient", action="store_true", help="skip the misfit-gradient report")
    ap.add_argument("--no-others", action="store_true", help="skip the realistic and three-size workloads")
    ap.add_argument("--cpu-steps", type=int, default=1000, help="time steps of the oracle sample")
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

    def say(*a):
        print(*a, file=sys.stderr, flush=True)

    g = config("full")
    npart = args.particles or g["particles"]
    prob = fd.Problem(g)
    info = prob.info
    vp = torch.tensor(true_model(g), dtype=torch.float32, device="cuda")
    dobs = fd.forward_shots(prob, vp)
    del vp
    swarm = EMPSO(g["node_lo"], g["node_hi"], npart, gen=50, seed=g["particle_seed"])
    fb = fd.FitnessBatch([prob], [dobs], [0] * npart)
    say("headline batch: %d runs, workspace %.1f GB" % (npart * prob.nshots, fb.ws.numel() / 1e9))
    if args.bz or args.tsteps:
        tu = fd.default_tuning()
        tu.bz = args.bz or tu.bz
        tu.tsteps = args.tsteps or tu.tsteps
        fb.tuning = tu
        tuned = False
    else:
        fb.autotune(swarm.ask())              # setup, untimed
        tu = fb.tuning
        tuned = True
    T = tu.tsteps
    say("tuning", tu.as_dict())
    last = prob.nt - 1
    block = max(T, int(round(args.block / T)) * T)
    points = npart * prob.nshots * info.Nz * info.Nx          # padded points of all runs
    phys_points = npart * prob.nshots * info.nz * info.nx
    upd_per_eval = prob.nshots * info.Nz * info.Nx * last       # one particle, all shots, whole record
    state = {"n": 0, "x": None, "iterations": 0}

    def step():
        """One block of time steps of the current iteration's evaluation;
        returns the number of time steps it advanced."""
        n0 = state["n"]
        if n0 == 0:
            state["x"] = swarm.ask()
        n1 = min(n0 + block, last)
        f = fb.steps(state["x"] if n0 == 0 else None, n0, n1)
        if n1 == last:
            swarm.tell(f.cpu().numpy())
            state["iterations"] += 1
            n1 = 0
        state["n"] = n1
        return (n1 if n1 else last) - n0

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    adv = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev0[k].record()
        adv.append(step())
        ev1[k].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = [a.elapsed_time(b) for a, b in zip(ev0, ev1)]
    tsteps_done = int(sum(adv))
    upd = points * tsteps_done
    gpt = upd / wall / 1e9
    evals_per_s = upd / wall / upd_per_eval
    # Dominant kernel: k_tb<T> over all runs. Each step enqueues its block's
    # launches on the current stream between two events, so the events bound
    # the launches' average duration from above (a block that starts or ends
    # an iteration also holds the state clearing, the coefficients, or the
    # last sample and the reduction).
    launches = sum(a // T + (a % T) / T for a in adv)
    launch_s = (float(np.sum(gpu_ms)) / 1000.0) / launches
    iso_us_step = fb.time_tuning(state["x"] if state["x"] is not None else swarm.ask(), tu, reps=6)
    upd_per_launch = points * T
    ops = alg_ops_per_update(info)
    achieved = upd_per_launch * ops / launch_s / 1e9
    traffic = committed_counter("k_tb_full_traffic.json", "hbm_bytes_per_launch", upd_per_launch, tu, info.Nz)
    valu = committed_counter("k_tb_full_valu.json", "valu_instructions_per_launch", upd_per_launch, tu, info.Nz)
    eff = upd_per_launch * BYTES_PER_UPDATE / launch_s / 1e9
    out = {
        "metric": METRIC, "value": evals_per_s, "unit": "fitness evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1000.0 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "full: 601x1841 grid at 5 m + 40-point layer (681x1921), %d particles x 32 "
                               "shots (%d runs, resident), 921 receivers, 6 Hz Ricker, 4 s (nt %d), 8x20 "
                               "nodes; one step = %d time steps of all runs of one EMPSO iteration's "
                               "evaluation (%d steps per iteration)"
                               % (npart, npart * prob.nshots, prob.nt, block, -(-last // block)),
                   "runs": npart * prob.nshots, "nt": prob.nt, "time_steps_per_step": block,
                   "time_steps_timed": tsteps_done, "iterations_completed": state["iterations"],
                   "tuning": tu.as_dict(), "autotuned": tuned},
        "value_derivation": "fitness evals/s = point-updates/s / (32 shots x 681 x 1921 x %d updates per "
                            "evaluation), from the timed steps' updates" % last,
        "gpt_updates_per_s": gpt,
        "gpt_updates_per_s_physical": phys_points * tsteps_done / wall / 1e9,
        "roofline": {"bound": "alu", "kernel": "k_tb<%d> over %d runs (strips of about %d rows)"
                     % (T, npart * prob.nshots, tu.bz),
                     "achieved": achieved, "peak": VALU_PEAK_GOPS, "unit": "Gop/s (VALU lane-operations)",
                     "frac": achieved / VALU_PEAK_GOPS, "traffic": traffic,
                     "algorithmic_ops_per_update": ops, "updates_per_launch": upd_per_launch,
                     "time_steps_per_launch": T, "avg_launch_us": launch_s * 1e6,
                     "isolated_launch_us": iso_us_step * T,
                     "valu_instructions_per_launch": valu,
                     "valu_issue_frac": None if valu is None else
                     valu * CYCLES_PER_VALU / (SIMDS * CLOCK_HZ * launch_s),
                     "hbm_effective_gbs": eff, "hbm_effective_frac": eff / HBM_PEAK_GBS,
                     "hbm_measured_gbs": None if traffic is None else traffic / launch_s / 1e9,
                     "hbm_measured_frac": None if traffic is None else traffic / launch_s / 1e9 / HBM_PEAK_GBS,
                     "hbm_peak_gbs": HBM_PEAK_GBS},
    }
    say(json.dumps(_strict(out)))
    cpu_geom, cpu_dt, cpu_nt = g, prob.dt, prob.nt
    del fb, dobs
    torch.cuda.empty_cache()
    if not args.no_others:
        out["realistic"] = whole_iterations("realistic", 3)
        say("realistic", json.dumps(out["realistic"]))
        out["batched"] = whole_iterations("batched", 2)
        say("batched", json.dumps(out["batched"]))
    if not args.no_gradient:
        gr = config("realistic")
        pr = fd.Problem(gr)
        d = fd.forward_shots(pr, torch.tensor(true_model(gr), dtype=torch.float32, device="cuda"))
        out["gradient"] = gradient_report(pr, d)
        say("gradient", json.dumps(out["gradient"]))
    if not args.no_surrogate:
        out["surrogate"] = surrogate_report()
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(cpu_geom, cpu_dt, cpu_nt, args.cpu_steps, threads)
    print(json.dumps(_strict(out), allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
