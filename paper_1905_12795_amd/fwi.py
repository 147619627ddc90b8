"""Local full-waveform inversion from the global search's best model.

Paper, Testing approach and Results sections: the best EMPSO model is the
starting model of a local FWI of the same data with the same l2 misfit,
run from low to higher frequencies (the trace-normalised misfit, when the
problem selects it, goes through the same calls). Here: steepest descent on the grid
model with the exact gradient of the discrete misfit (empso_gradient),
Barzilai-Borwein step lengths, a backtracking (Armijo) line search and a
box projection onto [vmin, vmax]; the model update is host FP64 arithmetic
like the swarm's, every misfit and gradient is one library call. A list of
stages (problem, observed data, iterations) gives the multiscale schedule.
"""
import math
import time

import numpy as np
import torch

from . import fd


def model_misfit(prob, vp, obs):
    """The problem's misfit (l2 or trace-normalised) of a physical model
    (device FP32 [nz][nx]) over all shots."""
    tr = fd.forward_shots(prob, vp)
    return float(fd.traces_misfit(prob, tr, obs))


def invert(prob, obs, vp0, iterations, vmin=None, vmax=None, first_step=20.0, armijo=1e-4, max_trials=8,
           checkpoint_every=0, precondition=True, eps=1e-3, log=None):
    """Steepest descent with Barzilai-Borwein steps and backtracking.

    vp0: host or device [nz][nx] starting model. first_step: the first trial
    step moves the model by at most this many m/s. precondition: scale the
    gradient by 1/(illumination + eps * max illumination), the source
    illumination of the starting model (a fixed diagonal metric, so the BB
    steps stay consistent). Returns (vp host FP64, history of per-iteration
    records: misfit, step, trials, gradient time).
    """
    vmin = float(prob.vmin if vmin is None else vmin)
    vmax = float(prob.vmax if vmax is None else vmax)
    dev = obs.device
    v = np.clip(np.asarray(torch.as_tensor(vp0).cpu(), dtype=np.float64), vmin, vmax)
    ws = fd.workspace(fd.lib.empso_gradient_workspace_bytes(prob.handle, int(checkpoint_every)), dev)

    P = None

    def grad_at(x):
        nonlocal P
        t0 = time.perf_counter()
        out = fd.gradient(prob, torch.tensor(x, dtype=torch.float32, device=dev), obs, checkpoint_every, ws,
                          illumination=precondition and P is None)
        gh = out[1].cpu().numpy().astype(np.float64)
        if precondition and P is None:
            ill = out[2].cpu().numpy().astype(np.float64)
            P = 1.0 / (ill + eps * ill.max())
        return float(out[0]), gh, time.perf_counter() - t0

    J, g, tg = grad_at(v)
    if P is None:
        P = np.ones_like(g)
    hist = [{"iteration": 0, "misfit": J, "gradient_s": tg}]
    alpha = first_step / max(np.abs(P * g).max(), 1e-300)
    v_prev = g_prev = None
    for it in range(1, iterations + 1):
        if v_prev is not None:
            s = v - v_prev
            y = P * (g - g_prev)
            sy = float(np.sum(s * y))
            if sy > 0:
                alpha = float(np.sum(s * s)) / sy                 # BB1 on the preconditioned gradient P g
        trials = 0
        while True:
            trials += 1
            v_new = np.clip(v - alpha * P * g, vmin, vmax)
            J_new = model_misfit(prob, torch.tensor(v_new, dtype=torch.float32, device=dev), obs)
            if J_new <= J - armijo * float(np.sum(g * (v - v_new))) or trials >= max_trials:
                break
            alpha *= 0.5
        if J_new >= J:                                            # no descent within max_trials
            hist.append({"iteration": it, "misfit": J, "step": 0.0, "trials": trials, "stalled": True})
            break
        v_prev, g_prev = v, g
        v = v_new
        J, g, tg = grad_at(v)
        rec = {"iteration": it, "misfit": J, "step": alpha, "trials": trials, "gradient_s": tg}
        hist.append(rec)
        if log:
            log(rec)
    return v, hist


def multiscale(stages, vp0, **kw):
    """stages: [(prob, obs, iterations), ...] from low to high frequency; each
    stage starts from the previous stage's model. Returns (vp, [histories])."""
    v = vp0
    out = []
    for prob, obs, iters in stages:
        v, h = invert(prob, obs, v, iters, **kw)
        out.append(h)
    return v, out


def rms_error(v, v_true):
    return float(math.sqrt(np.mean((np.asarray(v, np.float64) - v_true) ** 2)))
