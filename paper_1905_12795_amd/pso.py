"""Host FP64 particle swarm with constriction factor and elitist mutation (EMPSO).

Paper, Theory section: Eq. 1 updates each particle's velocity from its own
best position p_i (cognitive term, c1) and the swarm's best g (social term,
c2, gbest topology) with independent U[0,1] vectors u1, u2 multiplied element
by element and the whole bracket scaled by the constriction factor chi of
Eq. 3; Eq. 2 moves the particle. The elitist-mutation step (figure of the
EMPSO pseudo-code) sorts particles by fitness and replaces the positions of
the NM worst by the global best, each coordinate perturbed with probability
p_em by 0.1 * VR_d * N(0, 1); their velocities are kept. Algorithm overview
section: velocities are limited to [-lambda VR, lambda VR]; Testing approach
section: variables that leave their bounds return to the box, the
mutation starts at 10 % of the iterations, c1 = 1.2, c2 = 2.9, NM = 25 %,
p_em = 0.3.

Readings (where the paper is silent): the mutation acts on the NM particles
with the largest current misfit (the search minimises), ties in index order;
bringing back = clamping to the nearest bound, velocity kept; personal bests
change on strict improvement; gbest ties go to the lowest index; the
mutation is applied after the move of the same iteration.

Random numbers: numpy Generator(PCG64(seed)). Per iteration the draws are, in
this order: u1 [N][D], u2 [N][D], and when the mutation is active the uniform
[NM][D] and then the normal [NM][D] matrices (row k for the k-th worst).
Initialisation draws x [N][D] uniform in the box, then v [N][D] uniform in
[-lambda VR, lambda VR]. Fitness values are only compared, never combined,
so any strictly increasing transform of the fitness gives the same swarm.
"""
import json
import math

import numpy as np


def constriction(c1, c2):
    """Eq. 3."""
    phi = c1 + c2
    if phi < 4.0:
        raise ValueError("phi = c1 + c2 must be >= 4")
    return 2.0 / abs(2.0 - phi - math.sqrt(phi * phi - 4.0 * phi))


class EMPSO:
    def __init__(self, lo, hi, n, c1=1.2, c2=2.9, lam=0.5, gen=100, nm_frac=0.25, p_em=0.3,
                 em_start_frac=0.1, elitist=True, seed=0):
        self.lo = np.asarray(lo, dtype=np.float64).copy()
        self.hi = np.asarray(hi, dtype=np.float64).copy()
        if self.lo.shape != self.hi.shape or np.any(self.hi < self.lo):
            raise ValueError("bad search box")
        self.N, self.D = int(n), self.lo.size
        self.c1, self.c2, self.lam = float(c1), float(c2), float(lam)
        self.chi = constriction(self.c1, self.c2)
        self.gen = int(gen)
        self.nm = int(round(nm_frac * self.N))
        self.p_em = float(p_em)
        self.em_start = int(math.ceil(em_start_frac * self.gen))
        self.elitist = bool(elitist)
        self.vr = self.hi - self.lo
        self.vclamp = self.lam * self.vr
        self.rng = np.random.Generator(np.random.PCG64(seed))
        self.x = self.lo + self.vr * self.rng.random((self.N, self.D))
        self.v = -self.vclamp + 2.0 * self.vclamp * self.rng.random((self.N, self.D))
        self.p = self.x.copy()
        self.fp = np.full(self.N, np.inf)
        self.gi = 0
        self.k = 0              # completed iterations
        self.evaluations = 0
        self.history = []

    @property
    def g(self):
        return self.p[self.gi]

    @property
    def fg(self):
        return self.fp[self.gi]

    def ask(self):
        """Positions to evaluate this iteration ([N][D] FP64)."""
        return self.x

    def tell(self, f):
        """Fitness of ask()'s positions; runs bests, Eq. 1-2 and the elitist mutation."""
        f = np.asarray(f, dtype=np.float64).copy()
        if f.shape != (self.N,):
            raise ValueError("need %d fitness values" % self.N)
        f[~np.isfinite(f)] = np.inf
        self.evaluations += self.N
        better = f < self.fp
        self.fp = np.where(better, f, self.fp)
        self.p = np.where(better[:, None], self.x, self.p)
        self.gi = int(np.argmin(self.fp))        # first minimum: ties -> lowest index
        self.k += 1
        u1 = self.rng.random((self.N, self.D))
        u2 = self.rng.random((self.N, self.D))
        g = self.p[self.gi]
        v = self.chi * (self.v + self.c1 * u1 * (self.p - self.x) + self.c2 * u2 * (g - self.x))
        v = np.minimum(np.maximum(v, -self.vclamp), self.vclamp)
        x = np.minimum(np.maximum(self.x + v, self.lo), self.hi)
        if self.elitist and self.k >= self.em_start and self.nm > 0:
            ru = self.rng.random((self.nm, self.D))
            rn = self.rng.standard_normal((self.nm, self.D))
            worst = np.argsort(-f, kind="stable")[:self.nm]
            mut = np.where(ru < self.p_em, g + 0.1 * self.vr * rn, g)
            x[worst] = np.minimum(np.maximum(mut, self.lo), self.hi)
        self.x, self.v = x, v
        self.history.append({"iteration": self.k, "best": float(self.fg),
                             "mean": float(np.mean(f[np.isfinite(f)])) if np.any(np.isfinite(f)) else math.inf,
                             "median": float(np.median(f)), "evaluations": self.evaluations})
        return self.history[-1]

    def done(self):
        return self.k >= self.gen

    # checkpoint / resume ---------------------------------------------------
    def state_dict(self):
        return {"x": self.x.copy(), "v": self.v.copy(), "p": self.p.copy(), "fp": self.fp.copy(),
                "gi": self.gi, "k": self.k, "evaluations": self.evaluations,
                "rng": self.rng.bit_generator.state, "history": list(self.history)}

    def load_state_dict(self, s):
        self.x, self.v, self.p, self.fp = (np.array(s[k], dtype=np.float64) for k in ("x", "v", "p", "fp"))
        self.gi, self.k, self.evaluations = int(s["gi"]), int(s["k"]), int(s["evaluations"])
        self.rng.bit_generator.state = s["rng"]
        self.history = list(s["history"])


def save_checkpoint(path, swarm):
    """Swarm state (positions, velocities, bests, RNG state, log, and whatever
    else a subclass's state_dict holds) in one .npz: arrays as arrays, the
    rest as JSON text."""
    s = swarm.state_dict()
    arrays = {k: v for k, v in s.items() if isinstance(v, np.ndarray)}
    meta = json.dumps({k: v for k, v in s.items() if not isinstance(v, np.ndarray)})
    np.savez(path, meta=np.frombuffer(meta.encode(), dtype=np.uint8), **arrays)


def load_checkpoint(path, swarm):
    """Restore a swarm saved by save_checkpoint (no pickles are loaded)."""
    d = np.load(path, allow_pickle=False)
    meta = json.loads(bytes(d["meta"]).decode())
    swarm.load_state_dict({**{k: d[k] for k in d.files if k != "meta"}, **meta})
    return swarm
