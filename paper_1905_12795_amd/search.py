"""The velocity-model search: EMPSO (or surrogate-screened EMPSO) driving the
GPU fitness evaluation, with a per-iteration log and checkpoints.

Paper: Algorithm overview section (a generation loop, fitness of every
particle per generation, statistics and the final population saved at the
end). Each iteration evaluates the N current positions with the
finite-difference fitness (`fd.FitnessBatch`), then moves the swarm on the
host in FP64. In screened mode the surrogate learns from every evaluation
and picks each particle's move among K candidates.
"""
import json
import math
import time

import numpy as np
import torch

from . import fd
from .pso import EMPSO, load_checkpoint, save_checkpoint  # noqa: F401  (re-exported)
from .surrogate import RandomRanker, ScreenedEMPSO, Surrogate


def observed_data(prob, vp_true, device="cuda"):
    """Observed traces of the true model, modelled on the GPU (input data)."""
    return fd.forward_shots(prob, torch.as_tensor(np.asarray(vp_true, np.float32), device=device))


def lowpass(traces, dt, f_pass, f_stop, axis=1, delay=0.0):
    """Zero-phase low-pass filter along the time axis (host, FP64), with an
    optional delay.

    Paper, Testing approach section: the observed data are filtered below
    6 Hz. Reading: gain 1 up to f_pass, 0 from f_stop on, a raised-cosine
    transition in between, applied in the frequency domain to each trace
    zero-padded to at least twice its length (no wrap-around), so the
    filter is real and even in time (no phase shift). `delay` (seconds,
    0 <= delay < record length) multiplies by exp(-2 pi i f delay): the
    traces of a source started `delay` later, cut to the same record.
    """
    x = np.asarray(traces, dtype=np.float64)
    n = x.shape[axis]
    if not 0.0 <= delay < n * dt:
        raise ValueError("delay must lie in [0, record length)")
    nfft = 1 << int(math.ceil(math.log2(2 * n)))
    f = np.fft.rfftfreq(nfft, dt)
    gain = np.where(f <= f_pass, 1.0, 0.0)
    mid = (f > f_pass) & (f < f_stop)
    gain[mid] = 0.5 * (1.0 + np.cos(np.pi * (f[mid] - f_pass) / (f_stop - f_pass)))
    resp = gain * np.exp(-2j * np.pi * f * delay) if delay else gain
    shape = [1] * x.ndim
    shape[axis] = resp.size
    spec = np.fft.rfft(x, nfft, axis=axis) * resp.reshape(shape)
    return np.take(np.fft.irfft(spec, nfft, axis=axis), np.arange(n), axis=axis)


def observed_data_filtered(geom, prob, vp_true, f0_obs, f_pass, f_stop, device="cuda"):
    """Observed traces without the inverse crime: modelled on the GPU with a
    Ricker source of peak frequency f0_obs (same grid, dt and nt as prob),
    delayed so that its centre matches the modelling source's (Ricker delay
    1/f0 of each), and low-passed (lowpass) on the host. The fitness models
    with prob's own source, so even the true model keeps a non-zero misfit."""
    g = dict(geom)
    g["f0"] = float(f0_obs)
    pobs = fd.Problem(g, dt=prob.dt, nt=prob.nt)
    tr = observed_data(pobs, vp_true, device).cpu().numpy()
    delay = 1.0 / float(geom["f0"]) - 1.0 / float(f0_obs)
    if delay < 0:
        raise ValueError("the observing source must have the higher peak frequency")
    out = lowpass(tr, prob.dt, f_pass, f_stop, delay=delay).astype(np.float32)
    return torch.as_tensor(out, device=device)


def observed_for(geom, prob, vp_true, device="cuda"):
    """The workload's observed data: filtered data from another source when
    the geometry asks for it ("observed" key), else the inverse-crime data."""
    ob = geom.get("observed")
    if ob:
        return observed_data_filtered(geom, prob, vp_true, ob["f0"], ob["f_pass"], ob["f_stop"], device)
    return observed_data(prob, vp_true, device)


def spearman(a, b):
    ra = np.argsort(np.argsort(a))
    rb = np.argsort(np.argsort(b))
    return float(np.corrcoef(ra, rb)[0, 1])


def run(geom, dobs, prob, iterations, mode="plain", seed=0, K=16, warmup=2, sur_kw=None, log_path=None,
        autotune=True, elitist=True, target=None, evaluate=None, pretrain=None, pretrain_steps=0, max_evals=None,
        gen=None, tunings=None):
    """Run the search; returns the list of per-iteration records.

    Record fields: iteration, best, mean, median, evaluations (FD, cumulative),
    best_position (last record only: the global best's node values),
    wall_s (cumulative, FD + host + surrogate), fd_s (cumulative seconds in
    the FD fitness, the result's copy to the host included), gpt_updates_per_s
    (this iteration's FD point-updates over its FD seconds), evaluated_fraction
    (the share of the swarm sent to the FD fitness), and in screened mode
    surrogate_rho (Spearman correlation between the surrogate's prediction and
    the FD misfit of the evaluated particles, measured before it trains on
    them) and surrogate_mae (mean absolute error of the standardised
    log-misfit). If `target` is given the run stops once best <= target, and
    with `max_evals` once the FD evaluations reach it. `gen` (default
    `iterations`) is the swarm's nominal iteration count, which sets when the
    elitist mutation starts.

    Screened and random modes: `evaluate` = M < N sends only M of the N
    particles to the FD fitness each iteration (ScreenedEMPSO); `pretrain` =
    (X, f) are (particle, fitness) pairs from earlier FD runs that the
    surrogate holds and trains on (`pretrain_steps` Adam steps) before the
    search starts (untimed; the swarm then uses it from the first iteration).
    `tunings` (a dict, batch size -> tuning) shares autotuned tilings between
    runs: a batch size found there is not tuned again, a new one is tuned
    and added.
    """
    N = geom["particles"]
    M = N if (mode == "plain" or evaluate is None) else int(evaluate)
    lo, hi = geom["node_lo"], geom["node_hi"]
    fb = fd.FitnessBatch([prob], [dobs], [0] * M)
    kw = dict(gen=gen or iterations, seed=seed, elitist=elitist)
    if mode == "plain":
        swarm = EMPSO(lo, hi, N, **kw)
        sur = None
    elif mode == "screened":
        sur = Surrogate(lo, hi, seed=seed, **(sur_kw or {}))
        if pretrain is not None:
            sur.add(pretrain[0], pretrain[1])
            sur.train(steps=pretrain_steps)
            warmup = 0
        swarm = ScreenedEMPSO(lo, hi, N, sur, K=K, warmup=warmup, evaluate=M, **kw)
    elif mode == "random":
        sur = None
        swarm = ScreenedEMPSO(lo, hi, N, RandomRanker(seed), K=K, warmup=0 if pretrain is not None else warmup,
                              evaluate=M, **kw)
    else:
        raise ValueError(mode)
    if tunings is not None and M in tunings:
        fb.tuning = tunings[M]
    elif autotune:
        fb.autotune(swarm.ask())
        if tunings is not None:
            tunings[M] = fb.tuning
    out = []
    logf = open(log_path, "a") if log_path else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fd_s = 0.0
    for it in range(iterations):
        x = swarm.ask()
        t1 = time.perf_counter()
        f = fb(x).cpu().numpy().astype(np.float64)
        t_fd = time.perf_counter() - t1
        fd_s += t_fd
        rec_extra = {}
        if isinstance(sur, Surrogate) and swarm.k >= swarm.warmup:
            pred = sur.predict(x)
            ok = np.isfinite(f)
            lf = (np.log(np.maximum(f[ok], 1e-30)) - sur.mu) / sur.sigma
            rec_extra = {"surrogate_rho": spearman(pred[ok], f[ok]),
                         "surrogate_mae": float(np.mean(np.abs(pred[ok] - lf)))}
        rec = dict(swarm.tell(f))
        rec.update(rec_extra)
        rec["wall_s"] = time.perf_counter() - t0
        rec["fd_s"] = fd_s
        rec["gpt_updates_per_s"] = fb.updates / t_fd / 1e9
        rec["evaluated_fraction"] = len(x) / N
        rec["mode"] = mode
        out.append(rec)
        if logf:
            logf.write(json.dumps(rec) + "\n")
            logf.flush()
        if target is not None and rec["best"] <= target:
            break
        if max_evals is not None and rec["evaluations"] >= max_evals:
            break
    if logf:
        logf.close()
    if out:
        out[-1]["best_position"] = [float(x) for x in swarm.g]     # gbest nodes (FP64), not logged
    return out


def pretrain_pairs(prob, dobs, lo, hi, n, seed, batch=128, start=0, stop=None, progress=None):
    """(X, fitness) of particles drawn uniformly in the search box (n of them,
    seeded), evaluated by the FD fitness in batches: the data a surrogate can
    be trained on before a search. start/stop evaluate the rows [start, stop)
    of the same draw only, so that the set can be built in parts.
    progress(done, total), if given, is called after each batch."""
    from workloads.models import uniform_particles
    X = uniform_particles(n, lo, hi, seed)[start:stop]
    n = len(X)
    fb = fd.FitnessBatch([prob], [dobs], [0] * batch)
    fb.autotune(X[:batch])
    f = np.empty(n)
    for k in range(0, n, batch):
        xb = X[k:k + batch]
        if len(xb) < batch:                       # pad the last batch with copies of its first row
            xb = np.concatenate([xb, np.repeat(xb[:1], batch - len(xb), axis=0)])
        f[k:k + batch] = fb(xb).cpu().numpy()[:min(batch, n - k)]
        if progress:
            progress(min(k + batch, n), n)
    return X, f


def evals_to_reach(history, target):
    """(FD evaluations, wall seconds) when the best misfit first reaches target, else (inf, inf)."""
    for r in history:
        if r["best"] <= target:
            return r["evaluations"], r["wall_s"]
    return math.inf, math.inf


def mean_history(histories):
    """Seed average of equally long search histories: per iteration, the mean
    best misfit so far, FD evaluations and wall seconds (runs of one mode use
    the same FD evaluations per iteration, so the averages line up)."""
    n = min(len(h) for h in histories)
    return [{"iteration": k + 1,
             "best": float(np.mean([h[k]["best"] for h in histories])),
             "evaluations": float(np.mean([h[k]["evaluations"] for h in histories])),
             "wall_s": float(np.mean([h[k]["wall_s"] for h in histories]))} for k in range(n)]
