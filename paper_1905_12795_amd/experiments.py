"""Measurements beyond bench.py's headline line (run on an MI355X).

  python -m paper_1905_12795_amd.experiments throughput --workload batched
      one fitness call of the three-size batch (64 particles x 16 shots),
      autotuned; prints Gpt-updates/s and fitness evals/s.
  python -m paper_1905_12795_amd.experiments throughput --workload full --particles 8
      fitness of `particles` particles x 32 shots on the 601 x 1841 grid at
      5 m (a slice of the full workload's 128-particle iteration).
  python -m paper_1905_12795_amd.experiments surrogate-paired --workload realistic --pretrain pairs.npz
      plain EMPSO (128 particles) against the surrogate screen (1024
      candidates, the best-ranked 64 evaluated, a network pretrained on 20k
      FD pairs) and a random screen, on 12 paired seeds, with 95 % intervals.
  python -m paper_1905_12795_amd.experiments surrogate-ranking --workload mini
      the network's choice of one move among K candidates against a random
      choice among the same candidates (all evaluated by the FD fitness), on
      16 seeds at three states of the swarm, with 95 % intervals.
  python -m paper_1905_12795_amd.experiments surrogate --workload realistic --iters 15 --seeds 1
      plain vs surrogate-screened vs randomly screened EMPSO on the same
      seeds; FD evaluations and wall time until each reaches 1.01 x the plain
      run's final best misfit.

Every line printed is JSON; per-iteration search records are appended to
--log (JSONL) as they happen.
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1905_12795_amd import fd, search  # noqa: E402
from workloads.configs import config, true_model  # noqa: E402
from workloads.models import uniform_particles  # noqa: E402


def _emit(d):
    print(json.dumps(d), flush=True)


def throughput(workload, particles, calls):
    if workload == "batched":
        geoms = config("batched")
        probs = [fd.Problem(g) for g in geoms]
        npart = particles or geoms[0]["particles"]
        pop = [p % 3 for p in range(npart)]
        lo, hi = geoms[0]["node_lo"], geoms[0]["node_hi"]
        seed = geoms[0]["particle_seed"]
    else:
        g = config(workload)
        geoms = [g]
        probs = [fd.Problem(g)]
        npart = particles or g["particles"]
        pop = [0] * npart
        lo, hi = g["node_lo"], g["node_hi"]
        seed = g["particle_seed"]
    t0 = time.perf_counter()
    obs = [search.observed_for(g, p, true_model(g)) for p, g in zip(probs, geoms)]
    torch.cuda.synchronize()
    _emit({"stage": "observed data", "seconds": time.perf_counter() - t0})
    X = uniform_particles(npart, lo, hi, seed)
    fb = fd.FitnessBatch(probs, obs, pop)
    best, us = fb.autotune(X)
    _emit({"stage": "autotuned", "tuning": best, "us_per_step": us})
    fb(X)
    torch.cuda.synchronize()
    times = []
    for _ in range(calls):
        t0 = time.perf_counter()
        f = fb(X)
        f.cpu()
        times.append(time.perf_counter() - t0)
        _emit({"stage": "call", "seconds": times[-1]})
    s = float(np.median(times))
    _emit({"workload": workload, "particles": npart, "runs": int(sum(probs[q].nshots for q in pop)),
           "updates_per_call": fb.updates, "seconds_per_call": s, "gpt_updates_per_s": fb.updates / s / 1e9,
           "fitness_evals_per_s": npart / s, "tuning": best,
           "grids": [[p.info.Nz, p.info.Nx] for p in probs], "nt": probs[0].nt})


def surrogate(workload, iters, seeds, K, log, members=1, kappa=0.0, misfit="l2"):
    g = dict(config(workload), misfit=misfit)
    if workload in ("realistic", "irregular", "crime_free"):
        g = dict(g)
        g["particles"] = config("surrogate")["particles"]      # 64 particles x K = 16 -> 1024 candidates
    prob = fd.Problem(g)
    dobs = search.observed_for(g, prob, true_model(g))
    hist = {m: [] for m in ("plain", "screened", "random")}
    for seed in seeds:
        res = {"workload": workload, "misfit": misfit, "seed": seed, "particles": g["particles"], "K": K,
               "iterations": iters}
        hp = search.run(g, dobs, prob, iters, "plain", seed=seed, log_path=log)
        hist["plain"].append(hp)
        target = 1.01 * hp[-1]["best"]
        res.update(plain_final=hp[-1]["best"], plain_evals=hp[-1]["evaluations"], plain_wall=hp[-1]["wall_s"])
        for mode in ("screened", "random"):
            h = search.run(g, dobs, prob, iters, mode, seed=seed, K=K, log_path=log,
                           sur_kw={"members": members, "kappa": kappa} if mode == "screened" else None)
            hist[mode].append(h)
            e, t = search.evals_to_reach(h, target)
            res.update({mode + "_final": h[-1]["best"], mode + "_evals_to_plain": e, mode + "_wall_to_plain": t})
            if mode == "screened":
                rh = [r["surrogate_rho"] for r in h if "surrogate_rho" in r]
                res["screened_mean_rho"] = float(np.mean(rh)) if rh else None
        _emit(res)
    # seed-averaged best-misfit curves: a single search is chaotic
    mean = {m: search.mean_history(h) for m, h in hist.items()}
    target = 1.01 * mean["plain"][-1]["best"]
    summ = {"workload": workload, "misfit": misfit, "seeds": list(seeds), "summary": "seed-averaged best-misfit curves",
            "plain_final": mean["plain"][-1]["best"], "plain_evals": mean["plain"][-1]["evaluations"],
            "plain_wall": mean["plain"][-1]["wall_s"]}
    for mode in ("screened", "random"):
        e, t = search.evals_to_reach(mean[mode], target)
        summ.update({mode + "_final": mean[mode][-1]["best"], mode + "_evals_to_plain": e,
                     mode + "_wall_to_plain": t})
    summ["curves"] = {m: [round(r["best"], 4) for r in mean[m]] for m in mean}
    _emit(summ)


def paired_ci(d, level=0.95):
    """Mean of paired differences d and its two-sided t confidence interval."""
    from scipy import stats
    d = np.asarray(d, dtype=np.float64)
    m = float(d.mean())
    if d.size < 2:
        return m, float("nan"), float("nan")
    h = float(stats.t.ppf(0.5 + level / 2, d.size - 1) * d.std(ddof=1) / np.sqrt(d.size))
    return m, m - h, m + h


def load_pretrain_parts(paths):
    """(X, f) of pretraining pairs saved in parts (`pretrain` outputs, or one
    file): the parts are ordered by their first row and must tile the rows
    [0, n) of one seeded draw without gaps or overlaps."""
    parts = []
    for q in paths:
        d = np.load(q, allow_pickle=False)
        start = int(d["start"]) if "start" in d.files else 0
        parts.append((start, d["X"], d["f"]))
    parts.sort(key=lambda t: t[0])
    row = 0
    for start, X, _f in parts:
        if start != row:
            raise ValueError("pretraining parts do not tile the rows: expected row %d, got %d" % (row, start))
        row += len(X)
    return np.concatenate([t[1] for t in parts]), np.concatenate([t[2] for t in parts])


def surrogate_paired(workload, iters, seeds, N, K, M, pretrain_path, pretrain_n, pretrain_steps, log):
    """Plain EMPSO (N particles, all evaluated) against the surrogate screen
    (N particles x K candidate moves screened, the best-ranked M particles
    evaluated, a network pretrained on pretrain_n (particle, fitness) pairs of
    earlier FD runs) and against the same screen with a random ranking, on
    paired seeds. Per seed: FD evaluations and wall time until the best misfit
    reaches 1.01 x the plain run's final value (the screened runs stop there,
    or at the plain run's evaluation budget: censored). Summary: the mean
    paired differences with 95 % t intervals."""
    g = dict(config(workload))
    g["particles"] = N
    prob = fd.Problem(g)
    dobs = search.observed_for(g, prob, true_model(g))
    parts = pretrain_path.split(",") if pretrain_path else []
    if parts and all(os.path.exists(q) for q in parts):
        X0, f0 = load_pretrain_parts(parts)
        _emit({"stage": "pretraining pairs loaded", "paths": parts, "n": int(len(f0))})
    else:
        t0 = time.perf_counter()
        X0, f0 = search.pretrain_pairs(prob, dobs, g["node_lo"], g["node_hi"], pretrain_n, seed=1000)
        _emit({"stage": "pretraining pairs evaluated", "n": int(len(f0)), "seconds": time.perf_counter() - t0})
        if len(parts) == 1:
            np.savez(parts[0], X=X0, f=f0)
    rows = []
    tunings = {}                 # one autotuned tiling per batch size (N plain, M screened)
    for seed in seeds:
        hp = search.run(g, dobs, prob, iters, "plain", seed=seed, log_path=log, tunings=tunings)
        target = 1.01 * hp[-1]["best"]
        budget = hp[-1]["evaluations"]
        ep, tp = search.evals_to_reach(hp, target)
        row = {"seed": seed, "plain_final": hp[-1]["best"], "target": target, "budget": budget,
               "plain_evals": ep, "plain_wall": tp, "plain_wall_all": hp[-1]["wall_s"]}
        for mode in ("screened", "random"):
            h = search.run(g, dobs, prob, 10 * iters, mode, seed=seed, K=K, evaluate=M, log_path=log,
                           pretrain=(X0, f0), pretrain_steps=pretrain_steps, target=target, max_evals=budget,
                           gen=iters, tunings=tunings)
            e, t = search.evals_to_reach(h, target)
            row[mode + "_reached"] = bool(np.isfinite(e))
            row[mode + "_evals"] = e if np.isfinite(e) else h[-1]["evaluations"]
            row[mode + "_wall"] = t if np.isfinite(t) else h[-1]["wall_s"]
            row[mode + "_final"] = h[-1]["best"]
            if mode == "screened":
                rh = [r["surrogate_rho"] for r in h if "surrogate_rho" in r]
                row["screened_mean_rho"] = float(np.mean(rh)) if rh else None
        rows.append(row)
        _emit(dict(row, workload=workload))
    summ = {"workload": workload, "seeds": list(seeds), "particles": N, "K": K, "evaluated": M,
            "plain_iterations": iters, "pretrain_pairs": int(len(f0)), "pretrain_steps": pretrain_steps,
            "censored_at_budget": {m: int(sum(not r[m + "_reached"] for r in rows)) for m in ("screened", "random")}}
    for a, b in (("plain", "screened"), ("plain", "random"), ("random", "screened")):
        for q in ("evals", "wall"):
            m, lo, hi = paired_ci([r[a + "_" + q] - r[b + "_" + q] for r in rows])
            summ["%s_minus_%s_%s" % (a, b, q)] = {"mean": m, "ci95": [lo, hi]}
    for m in ("plain", "screened", "random"):
        summ[m + "_mean_evals"] = float(np.mean([r[m + "_evals"] for r in rows]))
        summ[m + "_mean_wall"] = float(np.mean([r[m + "_wall"] for r in rows]))
    _emit(summ)


def surrogate_ranking(workload, seeds, states, K, emit=True):
    """What the trained network adds where it acts: the choice of one move
    among K candidates. Per seed, plain EMPSO runs while a network trains
    online on every evaluated (position, misfit) pair (the screened search's
    schedule: 64 Adam steps per iteration); after each iteration count in
    `states`, every particle draws K candidate moves from the swarm's state,
    the FD fitness evaluates all K N of them, and the network's choice (lowest
    prediction) is compared with a uniformly random choice among the same
    candidates, whose expected log-misfit is the candidates' mean: a uniformly
    random choice among K independent draws is the move of plain EMPSO. Per
    seed, averaged over the states: the Spearman correlation of prediction and
    FD misfit over all candidates (0 for a random ranking), the mean over
    particles of E[log f(random choice)] - log f(network's choice) (positive:
    the network's moves are better) next to the same gain of the best
    candidate (the most any ranking can gain), and the fraction of particles
    whose network choice beats the candidates' median. Summary: means over
    seeds with 95 % t intervals. Returns (rows, summary)."""
    from .pso import EMPSO
    from .surrogate import Surrogate, candidate_moves
    g = config(workload)
    prob = fd.Problem(g)
    dobs = search.observed_for(g, prob, true_model(g))
    N, lo, hi = g["particles"], g["node_lo"], g["node_hi"]
    fb = fd.FitnessBatch([prob], [dobs], [0] * N)
    fb.autotune(uniform_particles(N, lo, hi, 0))
    states = sorted(int(k) for k in states)
    rows = []
    for seed in seeds:
        swarm = EMPSO(lo, hi, N, gen=max(states[-1], 10), seed=seed)
        sur = Surrogate(lo, hi, seed=seed)
        rng = np.random.Generator(np.random.PCG64(seed + 5000))
        per = []
        for it in range(1, states[-1] + 1):
            x = swarm.ask()
            f = fb(x).cpu().numpy().astype(np.float64)
            sur.add(x, f)
            sur.train()
            swarm.tell(f)
            if it not in states:
                continue
            cand = candidate_moves(swarm, K, rng)
            fc = np.stack([fb(cand[k]).cpu().numpy().astype(np.float64) for k in range(K)])     # [K][N]
            pred = sur.predict(cand.reshape(-1, swarm.D)).reshape(K, N)
            lf = np.log(fc)
            chosen = lf[np.argmin(pred, axis=0), np.arange(N)]
            per.append({"rho": search.spearman(pred.ravel(), fc.ravel()),
                        "log_gain": float(np.mean(lf.mean(axis=0) - chosen)),
                        "best_log_gain": float(np.mean(lf.mean(axis=0) - lf.min(axis=0))),
                        "beats_median": float(np.mean(chosen < np.median(lf, axis=0)))})
        row = {"seed": seed, "states": states, "K": K, "particles": N}
        for key in per[0]:
            row[key] = float(np.mean([q[key] for q in per]))
        rows.append(row)
        if emit:
            _emit(dict(row, workload=workload))
    summ = {"workload": workload, "seeds": list(seeds), "states": states, "K": K}
    for key in ("rho", "log_gain", "best_log_gain", "beats_median"):
        m, lo95, hi95 = paired_ci([r[key] for r in rows])
        summ[key] = {"mean": m, "ci95": [lo95, hi95]}
    if emit:
        _emit(summ)
    return rows, summ


def pretrain(workload, total, start, stop, out):
    """Rows [start, stop) of the seeded uniform draw of `total` particles,
    evaluated by the FD fitness, saved as (X, f) to `out` (.npz)."""
    g = config(workload)
    prob = fd.Problem(g)
    dobs = search.observed_for(g, prob, true_model(g))
    t0 = time.perf_counter()
    def progress(done, n):
        if done % 1280 == 0 or done == n:
            _emit({"stage": "pretraining pairs", "done": done, "of": n, "seconds": time.perf_counter() - t0})

    X, f = search.pretrain_pairs(prob, dobs, g["node_lo"], g["node_hi"], total, seed=1000, start=start, stop=stop,
                                 progress=progress)
    np.savez(out, X=X, f=f, start=start, stop=stop, total=total)
    _emit({"stage": "pretraining pairs", "rows": [start, stop], "seconds": time.perf_counter() - t0,
           "evals_per_s": len(f) / (time.perf_counter() - t0), "out": out})


def fwi_bands(g, prob, truth, bands):
    """Stages of a multiscale FWI on data from the workload's observing source:
    per band (f0, f_pass, f_stop, iterations), a problem with a Ricker source
    of peak f0 and the observed data low-passed to the band."""
    ob = g.get("observed")
    if not ob:
        raise ValueError("bands need a workload whose observed data come from another source")
    stages = []
    for f0, fp, fs, it in bands:
        gb = dict(g, f0=f0)
        pb = fd.Problem(gb, dt=prob.dt, nt=prob.nt)
        stages.append((pb, search.observed_data_filtered(gb, pb, truth, ob["f0"], fp, fs), int(it)))
    return stages


def local_fwi(workload, search_iters, fwi_iters, seed, misfit="l2", bands=None, particles=0, log=None):
    """The paper's workflow: the EMPSO best model starts a local FWI of the same
    data, in one band or, with `bands`, from low to high frequency."""
    from paper_1905_12795_amd import fwi
    g = dict(config(workload), misfit=misfit)
    if particles:
        g["particles"] = int(particles)
    prob = fd.Problem(g)
    truth = true_model(g)
    dobs = search.observed_for(g, prob, truth)
    h = search.run(g, dobs, prob, search_iters, "plain", seed=seed, log_path=log)
    _emit({"stage": "empso", "iterations": search_iters, "best": h[-1]["best"], "wall_s": h[-1]["wall_s"]})
    best = np.asarray(h[-1]["best_position"], dtype=np.float32)
    v0 = fd.vp_from_nodes(prob, torch.tensor(best[None, :], device="cuda"))[0].contiguous()
    t0 = time.perf_counter()
    if bands:
        v = v0
        for k, (pb, ob, it) in enumerate(fwi_bands(g, prob, truth, bands)):
            v, hb = fwi.invert(pb, ob, v, it, log=lambda r, k=k: _emit({"stage": "fwi", "band": k, **r}))
            _emit({"stage": "band", "band": k, "f0": bands[k][0], "misfit": hb[-1]["misfit"],
                   "rms_error": fwi.rms_error(v, truth)})
        v = torch.tensor(v, dtype=torch.float32, device="cuda")
        hist = [{"misfit": fwi.model_misfit(prob, v, dobs)}]
        v = v.cpu().numpy()
    else:
        v, hist = fwi.invert(prob, dobs, v0, fwi_iters, log=lambda r: _emit({"stage": "fwi", **r}))
    torch.cuda.synchronize()
    _emit({"workload": workload, "misfit": misfit, "seed": seed, "particles": g["particles"],
           "search_iterations": search_iters, "empso_misfit": h[-1]["best"],
           "true_model_misfit": fwi.model_misfit(prob, torch.tensor(truth, dtype=torch.float32, device="cuda"), dobs),
           "fwi_misfit": hist[-1]["misfit"],
           "fwi_iterations": int(sum(b[3] for b in bands)) if bands else len(hist) - 1,
           "fwi_wall_s": time.perf_counter() - t0,
           "rms_error_empso": fwi.rms_error(v0.cpu().numpy(), truth), "rms_error_fwi": fwi.rms_error(v, truth)})


def gradient_timing(workload, reps, modes=(False, True)):
    """Misfit gradients of a linear 1500-5500 m/s model over all shots of a
    workload (one untimed, `reps` timed), with and without the illumination."""
    g = config(workload)
    prob = fd.Problem(g)
    dobs = search.observed_for(g, prob, true_model(g))
    nz, nx = g["nz"], g["nx"]
    z = np.arange(nz, dtype=np.float64)[:, None] / (nz - 1)
    v0 = torch.tensor(np.repeat(1500.0 + 4000.0 * z, nx, axis=1), dtype=torch.float32, device="cuda")
    ws = fd.workspace(fd.lib.empso_gradient_workspace_bytes(prob.handle, 0))
    for illum in modes:
        fd.gradient(prob, v0, dobs, 0, ws, illumination=illum)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fd.gradient(prob, v0, dobs, 0, ws, illumination=illum)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        _emit({"workload": workload, "illumination": illum, "seconds_per_gradient": sec,
               "gpt_updates_per_s_three_passes": 3 * prob.updates_per_run * prob.nshots / sec / 1e9,
               "misfit": float(out[0])})


def bandwidth(mib, reps):
    """Achievable HBM rates of plain streaming operations on a buffer of `mib`
    MiB (context for the stencils' rooflines): device-to-device copy (read +
    write), an elementwise add of a scalar (read + write), fill (write) and
    sum (read). Median of `reps` timings with events on the current stream."""
    n = mib * (1 << 20) // 4
    a = torch.rand(n, device="cuda")
    b = torch.empty_like(a)
    ops = {"copy": (lambda: b.copy_(a), 8), "add_scalar": (lambda: torch.add(a, 1.0, out=b), 8),
           "fill": (lambda: b.fill_(1.0), 4), "sum": (lambda: a.sum(), 4)}
    out = {"bytes_per_element": {k: v[1] for k, v in ops.items()}, "mib": mib}
    for name, (fn, bpe) in ops.items():
        fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        t = float(np.median(ts))
        out[name + "_GBps"] = bpe * n / t / 1e9
        out[name + "_us"] = t * 1e6
    _emit(out)


def mlp_timing(reps):
    """Surrogate network at the surrogate workload's shape (D = 60, H = 256):
    inference on 1024 candidates and training steps of 256 rows."""
    from paper_1905_12795_amd.surrogate import Surrogate
    gs = config("surrogate")
    sur = Surrogate(gs["node_lo"], gs["node_hi"], seed=0)
    X = uniform_particles(2048, gs["node_lo"], gs["node_hi"], 0)
    sur.add(X, np.exp(np.random.default_rng(0).normal(5, 1, 2048)))
    Xc = torch.tensor(uniform_particles(1024, gs["node_lo"], gs["node_hi"], 1), dtype=torch.float32, device="cuda")
    idx = torch.arange(256, dtype=torch.int32, device="cuda")
    sur.net.predict(Xc)
    sur.net.train_step(sur.X, sur.f, idx, sur.mu, sur.sigma, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sur.net.predict(Xc)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        sur.net.train_step(sur.X, sur.f, idx, sur.mu, sur.sigma, 1e-4)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    _emit({"predict_1024_ms": (t1 - t0) / reps * 1e3, "train_step_256_ms": (t2 - t1) / reps * 1e3, "reps": reps})


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("throughput")
    t.add_argument("--workload", default="batched",
                   choices=["tiny", "realistic", "batched", "full", "irregular", "crime_free"])
    t.add_argument("--particles", type=int, default=0)
    t.add_argument("--calls", type=int, default=3)
    s = sub.add_parser("surrogate")
    s.add_argument("--workload", default="mini", choices=["mini", "realistic", "irregular", "crime_free"])
    s.add_argument("--iters", type=int, default=30)
    s.add_argument("--seeds", default="1,2,3")
    s.add_argument("--K", type=int, default=16)
    s.add_argument("--log", default=None)
    s.add_argument("--members", type=int, default=1, help="networks in the surrogate ensemble")
    s.add_argument("--kappa", type=float, default=0.0, help="score = members' mean + kappa * spread")
    s.add_argument("--misfit", default="l2", choices=["l2", "trace_normalised"])
    sp = sub.add_parser("surrogate-paired")
    sp.add_argument("--workload", default="realistic", choices=["mini", "realistic"])
    sp.add_argument("--iters", type=int, default=12, help="iterations of the plain search")
    sp.add_argument("--seeds", default="1,2,3,4,5,6,7,8,9,10,11,12")
    sp.add_argument("--particles", type=int, default=128)
    sp.add_argument("--K", type=int, default=8)
    sp.add_argument("--evaluate", type=int, default=64)
    sp.add_argument("--pretrain", default=None, help=".npz of (X, f) pairs, or a comma-separated list of `pretrain` parts: "
                         "loaded if present, else written")
    sp.add_argument("--pretrain-n", type=int, default=20000)
    sp.add_argument("--pretrain-steps", type=int, default=3000)
    sp.add_argument("--log", default=None)
    rk = sub.add_parser("surrogate-ranking")
    rk.add_argument("--workload", default="mini", choices=["mini", "realistic"])
    rk.add_argument("--seeds", default="1,2,3,4,5,6,7,8,9,10,11,12,13,14,15,16")
    rk.add_argument("--states", default="6,12,18", help="iteration counts after which the candidates are ranked")
    rk.add_argument("--K", type=int, default=16)
    pt = sub.add_parser("pretrain")
    pt.add_argument("--workload", default="realistic", choices=["mini", "realistic"])
    pt.add_argument("--total", type=int, default=20000)
    pt.add_argument("--start", type=int, default=0)
    pt.add_argument("--stop", type=int, default=None)
    pt.add_argument("--out", required=True)
    f = sub.add_parser("fwi")
    f.add_argument("--workload", default="realistic", choices=["realistic", "irregular", "crime_free"])
    f.add_argument("--search-iters", type=int, default=15)
    f.add_argument("--fwi-iters", type=int, default=10)
    f.add_argument("--seed", type=int, default=1)
    f.add_argument("--misfit", default="l2", choices=["l2", "trace_normalised"])
    f.add_argument("--particles", type=int, default=0, help="swarm size (0: the workload's)")
    f.add_argument("--log", default=None, help="per-iteration search log (JSON lines)")
    f.add_argument("--bands", default=None,
                   help="multiscale stages f0:f_pass:f_stop:iterations,... (Hz), low to high frequency")
    gr = sub.add_parser("gradient")
    gr.add_argument("--workload", default="realistic", choices=["tiny", "realistic", "irregular", "crime_free", "full"])
    gr.add_argument("--reps", type=int, default=2)
    gr.add_argument("--plain-only", action="store_true", help="skip the run that also returns the illumination")
    bw = sub.add_parser("bandwidth")
    bw.add_argument("--mib", type=int, default=1024)
    bw.add_argument("--reps", type=int, default=20)
    ml = sub.add_parser("mlp")
    ml.add_argument("--reps", type=int, default=50)
    a = ap.parse_args()
    if a.cmd == "throughput":
        throughput(a.workload, a.particles, a.calls)
    elif a.cmd == "gradient":
        gradient_timing(a.workload, a.reps, (False,) if a.plain_only else (False, True))
    elif a.cmd == "mlp":
        mlp_timing(a.reps)
    elif a.cmd == "bandwidth":
        bandwidth(a.mib, a.reps)
    elif a.cmd == "surrogate-ranking":
        surrogate_ranking(a.workload, [int(x) for x in a.seeds.split(",")], [int(x) for x in a.states.split(",")],
                          a.K)
    elif a.cmd == "pretrain":
        pretrain(a.workload, a.total, a.start, a.stop if a.stop is not None else a.total, a.out)
    elif a.cmd == "surrogate-paired":
        surrogate_paired(a.workload, a.iters, [int(x) for x in a.seeds.split(",")], a.particles, a.K, a.evaluate,
                         a.pretrain, a.pretrain_n, a.pretrain_steps, a.log)
    elif a.cmd == "fwi":
        bands = [tuple(float(x) for x in b.split(":")) for b in a.bands.split(",")] if a.bands else None
        local_fwi(a.workload, a.search_iters, a.fwi_iters, a.seed, a.misfit, bands, a.particles, a.log)
    else:
        surrogate(a.workload, a.iters, [int(x) for x in a.seeds.split(",")], a.K, a.log, a.members, a.kappa,
                  a.misfit)


if __name__ == "__main__":
    main()
