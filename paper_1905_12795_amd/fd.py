"""Python face of the fitness-evaluation library: problems, modelling, misfit, fitness.

Thin wrappers over the C ABI in include/empso.h: they check tensor dtypes,
devices and shapes, pass data pointers and the current HIP stream, and raise
EmpsoError on a non-zero status. No arithmetic of the method happens here.
"""
import ctypes
import math

import numpy as np
import torch

from ._lib import MISFITS, Geometry, ProblemInfo, Tuning, check, lib


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    """Device address of a tensor (NULL for None: an optional output)."""
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _need(t, dtype, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))


def stable_dt(vmax, dz, dx):
    """Stability limit of the scheme (library: empso_stable_dt)."""
    out = ctypes.c_double()
    check(lib.empso_stable_dt(float(vmax), float(dz), float(dx), ctypes.byref(out)))
    return out.value


def default_tuning():
    t = Tuning()
    check(lib.empso_default_tuning(ctypes.byref(t)))
    return t


def workspace(nbytes, device="cuda"):
    """A 256-byte aligned device buffer of at least nbytes (uint8 tensor)."""
    t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t[off:off + int(nbytes)]


class Problem:
    """A modelling problem (grid, time axis, acquisition, node grid) on the device.

    geom uses the keys of workloads.configs. dt defaults to dt_frac times the
    library's stability limit at vmax; nt to floor(tmax/dt) + 1.
    """

    def __init__(self, geom, dt=None, nt=None, vmin=None):
        if dt is None:
            dt = geom["dt_frac"] * stable_dt(geom["vmax"], geom["dz"], geom["dx"])
        if nt is None:
            nt = int(math.floor(geom["tmax"] / dt + 1e-9)) + 1
        self.geom = geom
        self.dt, self.nt = float(dt), int(nt)
        self._src = np.ascontiguousarray(np.asarray(geom["src"], dtype=np.float64).reshape(-1, 2))
        self._rec = np.ascontiguousarray(np.asarray(geom["rec"], dtype=np.float64).reshape(-1, 2))
        lo = np.asarray(geom["node_lo"], dtype=np.float64)
        water_rows = int(geom.get("water_rows", 0))
        v_water = float(geom.get("v_water", 1500.0))
        if vmin is None:
            vmin = float(min(lo.min(), v_water)) if water_rows else float(lo.min())
        g = Geometry()
        g.nz, g.nx = int(geom["nz"]), int(geom["nx"])
        g.dz, g.dx = float(geom["dz"]), float(geom["dx"])
        g.nbl = int(geom["nbl"])
        g.dt, g.nt, g.f0 = self.dt, self.nt, float(geom["f0"])
        g.nshots = self._src.shape[0]
        g.src_zx = self._src.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        g.nrec = self._rec.shape[0]
        g.rec_zx = self._rec.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        g.ncz, g.ncx = int(geom.get("ncz", 0)), int(geom.get("ncx", 0))
        g.vmin, g.vmax = float(vmin), float(geom["vmax"])
        self.vmin, self.vmax = g.vmin, g.vmax           # the velocity bounds the library enforces
        g.damp_R = float(geom.get("damp_R", 1e-3))
        if geom.get("node_z") is not None:          # layered node grid
            self._nz_ = np.ascontiguousarray(np.asarray(geom["node_z"], dtype=np.float64))
            self._nn_ = np.ascontiguousarray(np.asarray(geom["level_nodes"], dtype=np.int32))
            self._nx_ = np.ascontiguousarray(np.asarray(geom["node_x"], dtype=np.float64))
            g.ncz = int(self._nz_.size)
            g.node_z = self._nz_.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            g.level_nodes = self._nn_.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            g.node_x = self._nx_.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        g.water_rows, g.v_water = water_rows, v_water
        self.misfit = geom.get("misfit", "l2")
        if self.misfit not in MISFITS:
            raise ValueError("misfit must be one of %s" % sorted(MISFITS))
        g.misfit = MISFITS[self.misfit]
        h = ctypes.c_void_p()
        check(lib.empso_problem_create(ctypes.byref(g), ctypes.byref(h)))
        self.handle = h
        info = ProblemInfo()
        check(lib.empso_problem_get_info(h, ctypes.byref(info)))
        self.info = info

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lib is not None:
            try:
                lib.empso_problem_destroy(h)
            except Exception:
                pass
            self.handle = None

    @property
    def nshots(self):
        return self.info.nshots

    @property
    def nrec(self):
        return self.info.nrec

    @property
    def D(self):
        return int(self.info.D)

    @property
    def updates_per_run(self):
        return int(self.info.updates_per_run)


def vp_from_nodes(prob, nodes, out=None):
    """nodes[nm][D] FP32 (device) -> vp[nm][nz][nx] FP32 (device) (two-grid interpolation)."""
    _need(nodes, torch.float32, name="nodes")
    nm = nodes.shape[0]
    if nodes.dim() != 2 or nodes.shape[1] != prob.D:
        raise ValueError("nodes must be [nm][%d]" % prob.D)
    if out is None:
        out = torch.empty((nm, prob.info.nz, prob.info.nx), dtype=torch.float32, device=nodes.device)
    _need(out, torch.float32, (nm, prob.info.nz, prob.info.nx), "out")
    check(lib.empso_vp_from_nodes(prob.handle, nm, _ptr(nodes), _ptr(out), _stream()))
    return out


def forward_shots(prob, vp, shot0=0, nsh=None, out=None, ws=None, tuning=None):
    """Traces [nsh][nt][nrec] FP32 of shots shot0.. of the model vp[nz][nx] (device FP32)."""
    _need(vp, torch.float32, (prob.info.nz, prob.info.nx), "vp")
    if nsh is None:
        nsh = prob.nshots - shot0
    if out is None:
        out = torch.empty((nsh, prob.nt, prob.nrec), dtype=torch.float32, device=vp.device)
    _need(out, torch.float32, (nsh, prob.nt, prob.nrec), "out")
    need = lib.empso_forward_workspace_bytes(prob.handle, nsh)
    if ws is None:
        ws = workspace(need, vp.device)
    check(lib.empso_forward_shots(prob.handle, _ptr(vp), int(shot0), int(nsh), _ptr(out), _ptr(ws),
                                  ws.numel(), None if tuning is None else ctypes.byref(tuning), _stream()))
    return out


def gradient(prob, vp, obs, checkpoint_every=0, ws=None, illumination=False):
    """Misfit over all shots and its gradient with respect to the physical
    model (discrete adjoint with checkpoints, library call). vp[nz][nx] and
    obs[nshots][nt][nrec] are device FP32. Returns (misfit [1], grad [nz][nx]),
    plus the source illumination [nz][nx] when illumination=True."""
    _need(vp, torch.float32, (prob.info.nz, prob.info.nx), "vp")
    _need(obs, torch.float32, (prob.nshots, prob.nt, prob.nrec), "obs")
    need = lib.empso_gradient_workspace_bytes(prob.handle, int(checkpoint_every))
    if need == 0:
        raise ValueError("invalid gradient request")
    if ws is None:
        ws = workspace(need, vp.device)
    grad = torch.empty_like(vp)
    mis = torch.empty(1, dtype=torch.float32, device=vp.device)
    ill = torch.empty_like(vp) if illumination else None
    check(lib.empso_gradient(prob.handle, _ptr(vp), _ptr(obs), _ptr(grad), _ptr(mis), _ptr(ill),
                             int(checkpoint_every), _ptr(ws), ws.numel(), _stream()))
    return (mis, grad, ill) if illumination else (mis, grad)


def misfit(a, b, out=None, ws=None):
    """1/2 sum (a - b)^2 (FP32 inputs on the device, FP64 accumulation) -> tensor [1]."""
    _need(a, torch.float32, name="a")
    _need(b, torch.float32, tuple(a.shape), "b")
    if out is None:
        out = torch.empty(1, dtype=torch.float32, device=a.device)
    n = a.numel()
    if ws is None:
        ws = workspace(lib.empso_misfit_workspace_bytes(n), a.device)
    check(lib.empso_misfit(_ptr(a), _ptr(b), n, _ptr(out), _ptr(ws), ws.numel(), _stream()))
    return out


def traces_misfit(prob, traces, obs, out=None, ws=None):
    """The problem's misfit (l2 or trace-normalised) between recorded traces
    and observed traces, both device FP32 [nsh][nt][nrec], summed over shots
    (library call) -> tensor [1]."""
    nsh = traces.shape[0] if traces.dim() == 3 else -1
    _need(traces, torch.float32, (nsh, prob.nt, prob.nrec), "traces")
    _need(obs, torch.float32, (nsh, prob.nt, prob.nrec), "obs")
    if out is None:
        out = torch.empty(1, dtype=torch.float32, device=traces.device)
    if ws is None:
        ws = workspace(lib.empso_traces_misfit_workspace_bytes(prob.handle, nsh), traces.device)
    check(lib.empso_traces_misfit(prob.handle, _ptr(traces), _ptr(obs), nsh, _ptr(out), _ptr(ws), ws.numel(),
                                  _stream()))
    return out


def traces_misfit_noalloc(prob, traces, obs, out):
    """traces_misfit into a caller-given out [1] without any workspace: the
    library's fixed per-GPU scratch (empso_traces_misfit_noalloc; calls that
    overlap on one GPU race)."""
    nsh = traces.shape[0] if traces.dim() == 3 else -1
    _need(traces, torch.float32, (nsh, prob.nt, prob.nrec), "traces")
    _need(obs, torch.float32, (nsh, prob.nt, prob.nrec), "obs")
    _need(out, torch.float32, (1,), "out")
    check(lib.empso_traces_misfit_noalloc(prob.handle, _ptr(traces), _ptr(obs), nsh, _ptr(out), _stream()))
    return out


class FitnessBatch:
    """Reusable fitness evaluation of a fixed set of particles over one or more problems.

    probs: list of Problem; obs: list of device FP32 tensors [nshots][nt][nrec];
    prob_of_particle: problem index per particle. Holds the workspace so that
    repeated calls reuse the library's cached launch plan (and HIP graph).
    """

    def __init__(self, probs, obs, prob_of_particle, tuning=None, device="cuda"):
        self.probs = list(probs)
        self.obs = list(obs)
        for p, o in zip(self.probs, self.obs):
            _need(o, torch.float32, (p.nshots, p.nt, p.nrec), "obs")
        self.pop = np.ascontiguousarray(np.asarray(prob_of_particle, dtype=np.int32))
        self.np = int(self.pop.size)
        self._ph = (ctypes.c_void_p * len(self.probs))(*[p.handle.value for p in self.probs])
        self._oh = (ctypes.c_void_p * len(self.obs))(*[o.data_ptr() for o in self.obs])
        self.Dmax = max(p.D for p in self.probs)
        need = lib.empso_fitness_workspace_bytes(self._ph, len(self.probs), self._pop_ptr(), self.np)
        if need == 0 and self.np > 0:
            raise ValueError("invalid batch")
        self.ws = workspace(need, device)
        self.out = torch.empty(self.np, dtype=torch.float32, device=device)
        self.tuning = tuning if tuning is not None else default_tuning()

    def _pop_ptr(self):
        return self.pop.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))

    @property
    def updates(self):
        return sum(self.probs[q].updates_per_run * self.probs[q].nshots for q in self.pop)

    def autotune(self, nodes):
        """Pick the fastest tile height / temporal-blocking depth for this batch
        (library autotuner) and keep it. Returns (tuning dict, us per time step)."""
        x = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64))
        if x.shape != (self.np, self.Dmax):
            raise ValueError("nodes must be [%d][%d]" % (self.np, self.Dmax))
        best = Tuning()
        us = ctypes.c_float()
        check(lib.empso_autotune_fitness(self._ph, len(self.probs), self._oh, self._pop_ptr(), self.np,
                                         x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self.Dmax,
                                         _ptr(self.ws), self.ws.numel(), ctypes.byref(best), ctypes.byref(us),
                                         _stream()))
        self.tuning = best
        return best.as_dict(), float(us.value)

    def time_tuning(self, nodes, tuning, reps=4):
        """Microseconds per time step of one tuning over `reps` kernel launches."""
        x = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64))
        if x.shape != (self.np, self.Dmax):
            raise ValueError("nodes must be [%d][%d]" % (self.np, self.Dmax))
        us = ctypes.c_float()
        check(lib.empso_time_tuning(self._ph, len(self.probs), self._oh, self._pop_ptr(), self.np,
                                    x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self.Dmax,
                                    _ptr(self.ws), self.ws.numel(), ctypes.byref(tuning), int(reps),
                                    ctypes.byref(us), _stream()))
        return float(us.value)

    def steps(self, nodes, n_begin, n_end, tuning=None):
        """Time steps n_begin .. n_end - 1 of an evaluation of the batch
        (library: empso_fitness_batch_steps). n_begin = 0 starts one from
        `nodes` (host float64 [np][D]); later blocks continue it (nodes may be
        None); the block that ends at nt - 1 writes the fitness values, which
        the returned device tensor then holds."""
        t = tuning if tuning is not None else self.tuning
        xp = None
        if nodes is not None:
            x = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64))
            if x.shape != (self.np, self.Dmax):
                raise ValueError("nodes must be [%d][%d]" % (self.np, self.Dmax))
            self._steps_nodes = x                     # kept alive for the call
            xp = x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        check(lib.empso_fitness_batch_steps(self._ph, len(self.probs), self._oh, self._pop_ptr(), self.np, xp,
                                            self.Dmax, _ptr(self.out), int(n_begin), int(n_end), _ptr(self.ws),
                                            self.ws.numel(), ctypes.byref(t), _stream()))
        return self.out

    def __call__(self, nodes, tuning=None):
        """nodes: host float64 [np][D] (row stride Dmax). Returns the device fitness tensor."""
        x = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64))
        if x.size == 0:
            x = x.reshape(0, self.Dmax)
        if x.shape != (self.np, self.Dmax):
            raise ValueError("nodes must be [%d][%d]" % (self.np, self.Dmax))
        t = tuning if tuning is not None else self.tuning
        check(lib.empso_fitness_batch(self._ph, len(self.probs), self._oh, self._pop_ptr(), self.np,
                                      x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self.Dmax,
                                      _ptr(self.out), _ptr(self.ws), self.ws.numel(), ctypes.byref(t),
                                      _stream()))
        return self.out
