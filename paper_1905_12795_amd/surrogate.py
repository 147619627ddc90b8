"""Learned surrogate of the fitness and the screening policy built on it.

Not part of the paper. A multilayer perceptron (HIP library, BF16 MFMA with
FP32 accumulation, FP32 Adam) learns the standardised log-misfit of
control-node vectors from the (particle, misfit) pairs that the
finite-difference fitness produces during the search. Before each
finite-difference evaluation, every particle proposes several candidate
moves (independent draws of Eq. 1's random vectors) and takes the one the
network ranks best. Either every particle is then evaluated (the number of
finite-difference evaluations per iteration is unchanged, the moves that
reach the solver are better on average), or only the M particles whose new
positions rank best across the swarm are (the global screen: N K candidates
ranked, M finite-difference evaluations per iteration).
"""
import ctypes

import numpy as np
import torch

from ._lib import check, lib
from .pso import EMPSO
from workloads.models import mlp_init


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def flatten_params(layers):
    """[(W1,b1),(W2,b2),(W3,b3),(w4,b4)] -> flat FP32 vector in the library's layout."""
    parts = []
    for W, b in layers[:-1]:
        parts += [np.asarray(W, np.float32).ravel(), np.asarray(b, np.float32).ravel()]
    W4, b4 = layers[-1]
    parts += [np.asarray(W4, np.float32).ravel(), np.asarray(b4, np.float32).ravel()]
    return np.concatenate(parts)


def unflatten_params(flat, D, H):
    flat = np.asarray(flat, dtype=np.float64)
    out, k = [], 0
    for fin in (D, H, H):
        W = flat[k:k + H * fin].reshape(H, fin); k += H * fin
        b = flat[k:k + H]; k += H
        out.append((W, b))
    w4 = flat[k:k + H].reshape(1, H); k += H
    b4 = flat[k:k + 1]; k += 1
    out.append((w4, b4))
    return out


class MLP:
    """Device-resident network: FP32 parameters, BF16 weight copy, Adam moments."""

    def __init__(self, lo, hi, H=256, seed=0, device="cuda"):
        self.lo = torch.tensor(np.asarray(lo, np.float32), device=device)
        self.hi = torch.tensor(np.asarray(hi, np.float32), device=device)
        self.D, self.H = int(self.lo.numel()), int(H)
        self.P = lib.empso_mlp_param_count(self.D, self.H)
        self.PB = lib.empso_mlp_bf16_count(self.D, self.H)
        init = flatten_params(mlp_init([self.D, self.H, self.H, self.H, 1], seed))
        assert init.size == self.P
        self.params = torch.tensor(init, device=device)
        self.wbf16 = torch.empty(self.PB, dtype=torch.int16, device=device)
        self.m = torch.zeros(self.P, dtype=torch.float32, device=device)
        self.v = torch.zeros(self.P, dtype=torch.float32, device=device)
        self.step = 0
        self._ws = {}
        check(lib.empso_mlp_sync_bf16(self.D, self.H, _ptr(self.params), _ptr(self.wbf16), _stream()))

    def state_dict(self):
        """FP32 parameters, Adam moments and step count (host copies)."""
        return {"params": self.params.cpu().numpy(), "m": self.m.cpu().numpy(), "v": self.v.cpu().numpy(),
                "step": self.step}

    def load_state_dict(self, st):
        for name in ("params", "m", "v"):
            t = getattr(self, name)
            a = np.asarray(st[name], dtype=np.float32)
            if a.shape != tuple(t.shape):
                raise ValueError("%s has shape %s, want %s" % (name, a.shape, tuple(t.shape)))
            t.copy_(torch.as_tensor(a))
        self.step = int(st["step"])
        check(lib.empso_mlp_sync_bf16(self.D, self.H, _ptr(self.params), _ptr(self.wbf16), _stream()))

    def _workspace(self, n):
        if n not in self._ws:
            nb = lib.empso_mlp_workspace_bytes(self.D, self.H, n)
            if nb == 0:
                raise ValueError("bad MLP shape")
            self._ws[n] = torch.empty(nb, dtype=torch.uint8, device=self.params.device)
        return self._ws[n]

    def predict(self, X):
        """X: device FP32 [n][D] -> device FP32 [n] (standardised log-misfit)."""
        n = int(X.shape[0])
        y = torch.empty(n, dtype=torch.float32, device=X.device)
        ws = self._workspace(n)
        check(lib.empso_mlp_predict(self.D, self.H, _ptr(self.params), _ptr(self.wbf16), _ptr(self.lo),
                                    _ptr(self.hi), _ptr(X), n, _ptr(y), _ptr(ws), ws.numel(), _stream()))
        return y

    def grad(self, X, fit, idx, mu, sigma):
        n = int(idx.numel()) if idx is not None else int(X.shape[0])
        g = torch.empty(self.P, dtype=torch.float32, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        ws = self._workspace(n)
        check(lib.empso_mlp_grad(self.D, self.H, _ptr(self.params), _ptr(self.wbf16), _ptr(self.lo), _ptr(self.hi),
                                 _ptr(X), _ptr(fit), _ptr(idx), n, float(mu), float(sigma), _ptr(g), _ptr(loss),
                                 _ptr(ws), ws.numel(), _stream()))
        return loss, g

    def train_step(self, X, fit, idx, mu, sigma, lr):
        n = int(idx.numel()) if idx is not None else int(X.shape[0])
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        ws = self._workspace(n)
        self.step += 1
        check(lib.empso_mlp_train_step(self.D, self.H, _ptr(self.params), _ptr(self.wbf16), _ptr(self.m),
                                       _ptr(self.v), self.step, float(lr), _ptr(self.lo), _ptr(self.hi), _ptr(X),
                                       _ptr(fit), _ptr(idx), n, float(mu), float(sigma), _ptr(loss), _ptr(ws),
                                       ws.numel(), _stream()))
        return loss


class Surrogate:
    """MLP (or a small ensemble of them) plus the on-device dataset of
    (nodes, FD fitness) pairs it learns from.

    members > 1: independently initialised networks trained on independent
    mini-batches of the same data, each with steps_per_update / members Adam
    steps per update (the same cost as one network); a candidate is scored
    by the members' mean plus kappa times their spread, so candidates the
    members disagree on (typically far from any evaluated particle) rank
    worse.
    """

    def __init__(self, lo, hi, H=256, seed=0, lr=1e-3, batch=256, steps_per_update=64, capacity=65536,
                 members=1, kappa=0.0, device="cuda"):
        self.nets = [MLP(lo, hi, H=H, seed=seed + 1000 * m, device=device) for m in range(int(members))]
        self.net = self.nets[0]
        self.D = self.net.D
        self.kappa = float(kappa)
        self.lr, self.batch, self.steps_per_update = float(lr), int(batch), int(steps_per_update)
        self.X = torch.empty((capacity, self.D), dtype=torch.float32, device=device)
        self.f = torch.empty(capacity, dtype=torch.float32, device=device)
        self.logf = []                       # host copy of log-fitness for the target scaling
        self.count = 0
        self.rng = np.random.Generator(np.random.PCG64(seed + 1))
        self.mu, self.sigma = 0.0, 1.0

    def add(self, X, fit):
        """Append evaluated particles: X host [k][D], fit host or device [k]."""
        k = len(X)
        if self.count + k > self.X.shape[0]:
            raise ValueError("surrogate dataset full")
        self.X[self.count:self.count + k] = torch.as_tensor(np.asarray(X, np.float32), device=self.X.device)
        fit_t = torch.as_tensor(fit, dtype=torch.float32).to(self.X.device)
        self.f[self.count:self.count + k] = fit_t
        fh = np.asarray(fit_t.cpu(), dtype=np.float64)
        self.logf.extend(np.log(np.maximum(fh[np.isfinite(fh)], 1e-30)).tolist())
        self.count += k
        lf = np.asarray(self.logf)
        self.mu = float(lf.mean())
        self.sigma = float(max(lf.std(), 1e-6))

    def train(self, steps=None):
        """Adam steps on random mini-batches of the dataset (split over the
        members); returns the last loss."""
        steps = self.steps_per_update if steps is None else steps
        per = max(1, steps // len(self.nets))
        if steps <= 0 or self.count == 0:
            return None
        # every step's mini-batch indices in one upload: a host-to-device copy
        # per step would wait for the previous step's kernels each time
        b = min(self.batch, self.count)
        idx = torch.as_tensor(self.rng.integers(0, self.count, (len(self.nets) * per, b)).astype(np.int32),
                              device=self.X.device)
        loss = None
        for m, net in enumerate(self.nets):
            for k in range(per):
                loss = net.train_step(self.X, self.f, idx[m * per + k], self.mu, self.sigma, self.lr)
        return float(loss.item())

    def state_dict(self):
        """Everything a resumed search needs to continue bit for bit: every
        network's state, the dataset, the target standardisation and the
        mini-batch generator's state."""
        return {"nets": [n.state_dict() for n in self.nets], "X": self.X[:self.count].cpu().numpy(),
                "f": self.f[:self.count].cpu().numpy(), "logf": list(self.logf), "count": self.count,
                "mu": self.mu, "sigma": self.sigma, "rng": self.rng.bit_generator.state}

    def load_state_dict(self, st):
        if len(st["nets"]) != len(self.nets):
            raise ValueError("the state holds %d networks, this surrogate %d" % (len(st["nets"]), len(self.nets)))
        for n, ns in zip(self.nets, st["nets"]):
            n.load_state_dict(ns)
        k = int(st["count"])
        if k > self.X.shape[0]:
            raise ValueError("dataset of %d rows exceeds the capacity %d" % (k, self.X.shape[0]))
        self.X[:k] = torch.as_tensor(np.asarray(st["X"], np.float32), device=self.X.device)
        self.f[:k] = torch.as_tensor(np.asarray(st["f"], np.float32), device=self.X.device)
        self.count = k
        self.logf = [float(x) for x in st["logf"]]
        self.mu, self.sigma = float(st["mu"]), float(st["sigma"])
        self.rng.bit_generator.state = st["rng"]

    def predict(self, X):
        """Host [n][D] -> host score [n]: the predicted standardised log-misfit
        (members' mean + kappa * spread for an ensemble)."""
        Xd = torch.as_tensor(np.asarray(X, np.float32), device=self.X.device)
        if len(self.nets) == 1:
            return self.net.predict(Xd).cpu().numpy().astype(np.float64)
        P = np.stack([n.predict(Xd).cpu().numpy().astype(np.float64) for n in self.nets])
        return P.mean(axis=0) + self.kappa * P.std(axis=0)


class RandomRanker:
    """Ablation of the surrogate: ranks candidates at random (seeded), so the
    screened search degenerates to EMPSO with an extra choice among K draws."""

    def __init__(self, seed=0):
        self.rng = np.random.Generator(np.random.PCG64(seed + 7))
        self.count = 0
        self.mu, self.sigma = 0.0, 1.0

    def add(self, X, fit):
        self.count += len(X)

    def train(self, steps=None):
        return None

    def predict(self, X):
        return self.rng.random(len(X))


class ScreenedEMPSO(EMPSO):
    """EMPSO whose moves, and optionally whose evaluations, are chosen by the
    surrogate.

    Every iteration each particle proposes K candidate moves (independent draws
    of Eq. 1's u1, u2) and takes the one the surrogate ranks best, so N K
    candidates are screened. With evaluate = M < N only the M particles whose
    new positions rank best across the swarm go to the finite-difference
    fitness; the others move without an evaluation (their personal bests
    stand) and rank below every evaluated particle for the elitist mutation,
    among themselves in the order of their predicted misfit. With M = N every
    particle is evaluated. With K = 1 and M = N (or during the first `warmup`
    iterations with M = N) it is EMPSO. The finite-difference fitness stays
    the judge: personal and global bests change only on evaluated values.

    Draw order per iteration: K pairs (u1, u2) of [N][D] uniforms, then the
    elitist-mutation draws as in EMPSO; with M < N and an untrained surrogate
    (iterations before `warmup`) a permutation of N picks the evaluated
    particles at random.
    """

    def __init__(self, lo, hi, n, surrogate, K=16, warmup=2, evaluate=None, **kw):
        super().__init__(lo, hi, n, **kw)
        self.sur = surrogate
        self.K = int(K)
        self.warmup = int(warmup)
        self.M = self.N if evaluate is None else int(evaluate)
        if not 1 <= self.M <= self.N:
            raise ValueError("evaluate must lie in [1, N]")
        self.sel = None                      # particles evaluated at the current positions
        self.pred = np.zeros(self.N)         # predicted scores of the current positions
        self.last_rank_corr = None

    def state_dict(self):
        st = super().state_dict()
        st.update(sel=None if self.sel is None else self.sel.copy(), pred=self.pred.copy())
        return st

    def load_state_dict(self, st):
        super().load_state_dict(st)
        self.sel = None if st.get("sel") is None else np.asarray(st["sel"], dtype=np.int64)
        self.pred = np.asarray(st["pred"], dtype=np.float64)

    def _select(self):
        """Choose the M particles to evaluate at the current positions."""
        if self.M == self.N:
            self.sel = np.arange(self.N)
            return
        if self.k < self.warmup:
            self.sel = np.sort(self.rng.permutation(self.N)[:self.M])
            self.pred = np.zeros(self.N)
            return
        self.pred = self.sur.predict(self.x)
        self.sel = np.sort(np.argsort(self.pred, kind="stable")[:self.M])

    def ask(self):
        if self.sel is None:
            self._select()
        return self.x[self.sel]

    def tell(self, f):
        f = np.asarray(f, dtype=np.float64).copy()
        if self.sel is None:
            self._select()
        if f.shape != (len(self.sel),):
            raise ValueError("need %d fitness values" % len(self.sel))
        f[~np.isfinite(f)] = np.inf
        self.sur.add(self.x[self.sel], np.where(np.isfinite(f), f, np.float32(3e38)))
        self.sur.train()
        if self.M == self.N and (self.k + 1 < self.warmup or self.K <= 1):
            return super().tell(f)
        fa = np.full(self.N, np.inf)
        fa[self.sel] = f
        # bests (as in EMPSO.tell), on the evaluated particles only
        self.evaluations += len(self.sel)
        better = fa < self.fp
        self.fp = np.where(better, fa, self.fp)
        self.p = np.where(better[:, None], self.x, self.p)
        self.gi = int(np.argmin(self.fp))
        self.k += 1
        g = self.p[self.gi]
        cand_x, cand_v = [], []
        for _ in range(self.K):
            u1 = self.rng.random((self.N, self.D))
            u2 = self.rng.random((self.N, self.D))
            v = self.chi * (self.v + self.c1 * u1 * (self.p - self.x) + self.c2 * u2 * (g - self.x))
            v = np.minimum(np.maximum(v, -self.vclamp), self.vclamp)
            cand_v.append(v)
            cand_x.append(np.minimum(np.maximum(self.x + v, self.lo), self.hi))
        cx = np.stack(cand_x)                       # [K][N][D]
        if self.K > 1 and self.k >= self.warmup:
            pred = self.sur.predict(cx.reshape(-1, self.D)).reshape(self.K, self.N)
            pick = np.argmin(pred, axis=0)
        else:
            pick = np.zeros(self.N, dtype=np.int64)
        x = cx[pick, np.arange(self.N)]
        v = np.stack(cand_v)[pick, np.arange(self.N)]
        if self.elitist and self.k >= self.em_start and self.nm > 0:
            ru = self.rng.random((self.nm, self.D))
            rn = self.rng.standard_normal((self.nm, self.D))
            # worst first: unevaluated particles (by predicted score, highest
            # first), then evaluated ones by fitness; ties in index order
            evaluated = np.zeros(self.N, dtype=bool)
            evaluated[self.sel] = True
            key = np.where(evaluated, fa, np.inf)
            worst = np.lexsort((np.arange(self.N), -np.where(evaluated, 0.0, self.pred), -key))[:self.nm]
            mut = np.where(ru < self.p_em, g + 0.1 * self.vr * rn, g)
            x[worst] = np.minimum(np.maximum(mut, self.lo), self.hi)
        self.x, self.v = x, v
        self._select()
        fin = f[np.isfinite(f)]
        self.history.append({"iteration": self.k, "best": float(self.fg),
                             "mean": float(np.mean(fin)) if fin.size else float("inf"),
                             "median": float(np.median(f)), "evaluations": self.evaluations})
        return self.history[-1]


def candidate_moves(swarm, K, rng):
    """K independent draws of the Eq. 1-2 move of every particle from the
    swarm's current state (positions, velocities, personal and global bests),
    with the velocity clamp and the box clamp: [K][N][D] positions. The
    random vectors come from `rng`, so the swarm's own generator is not
    touched; the arithmetic is that of ScreenedEMPSO's candidates."""
    g = swarm.g
    out = np.empty((int(K), swarm.N, swarm.D))
    for k in range(int(K)):
        u1 = rng.random((swarm.N, swarm.D))
        u2 = rng.random((swarm.N, swarm.D))
        v = swarm.chi * (swarm.v + swarm.c1 * u1 * (swarm.p - swarm.x) + swarm.c2 * u2 * (g - swarm.x))
        v = np.minimum(np.maximum(v, -swarm.vclamp), swarm.vclamp)
        out[k] = np.minimum(np.maximum(swarm.x + v, swarm.lo), swarm.hi)
    return out


def save_surrogate(path, sur):
    """A surrogate's state (Surrogate.state_dict) in one .npz: arrays as arrays,
    the rest as JSON text; no pickles."""
    import json
    st = sur.state_dict()
    arrays = {"X": st["X"], "f": st["f"], "logf": np.asarray(st["logf"], dtype=np.float64)}
    for k, ns in enumerate(st["nets"]):
        for name in ("params", "m", "v"):
            arrays["net%d_%s" % (k, name)] = ns[name]
    meta = {"count": st["count"], "mu": st["mu"], "sigma": st["sigma"], "rng": st["rng"],
            "steps": [ns["step"] for ns in st["nets"]]}
    np.savez(path, meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8), **arrays)


def load_surrogate(path, sur):
    """Restore a surrogate saved by save_surrogate (no pickles are loaded)."""
    import json
    d = np.load(path, allow_pickle=False)
    meta = json.loads(bytes(d["meta"]).decode())
    nets = [{"params": d["net%d_params" % k], "m": d["net%d_m" % k], "v": d["net%d_v" % k], "step": step}
            for k, step in enumerate(meta["steps"])]
    sur.load_state_dict({"nets": nets, "X": d["X"], "f": d["f"], "logf": d["logf"].tolist(),
                         "count": meta["count"], "mu": meta["mu"], "sigma": meta["sigma"], "rng": meta["rng"]})
    return sur
