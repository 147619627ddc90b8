"""Host logic of the surrogate screen (ScreenedEMPSO) with a stand-in
surrogate on the CPU: with one candidate and every particle evaluated it is
EMPSO bit for bit; with M < N it evaluates the M best-predicted particles,
only those change their personal bests, and the elitist mutation takes the
unevaluated particles first, worst predicted first."""
import numpy as np

from paper_1905_12795_amd import pso
from paper_1905_12795_amd.surrogate import RandomRanker, ScreenedEMPSO


class _Exact:
    """A surrogate that predicts the sphere function exactly."""

    def __init__(self, c):
        self.c = c
        self.count = 0

    def add(self, X, f):
        self.count += len(X)

    def train(self, steps=None):
        return None

    def predict(self, X):
        return np.sum((np.asarray(X) - self.c) ** 2, axis=1)


def _box(D=6, seed=0):
    r = np.random.default_rng(seed)
    lo = r.uniform(-2, 0, D)
    hi = lo + r.uniform(1, 3, D)
    return lo, hi, r.uniform(lo, hi)


def test_one_candidate_all_evaluated_is_empso():
    lo, hi, c = _box()
    a = pso.EMPSO(lo, hi, 10, gen=8, seed=3)
    b = ScreenedEMPSO(lo, hi, 10, _Exact(c), K=1, warmup=0, gen=8, seed=3)
    for _ in range(8):
        assert np.array_equal(a.ask(), b.ask())
        f = np.sum((a.ask() - c) ** 2, axis=1)
        a.tell(f)
        b.tell(f)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.p, b.p) and a.evaluations == b.evaluations


def test_partial_evaluation_picks_the_best_predicted_and_counts():
    lo, hi, c = _box(seed=1)
    N, M = 24, 8
    sur = _Exact(c)
    sw = ScreenedEMPSO(lo, hi, N, sur, K=4, warmup=0, evaluate=M, gen=20, seed=5)
    for it in range(20):
        x = sw.ask()
        assert x.shape == (M, len(lo))
        pred = sur.predict(sw.x)
        assert set(sw.sel) == set(np.argsort(pred, kind="stable")[:M])
        p_before, fp_before = sw.p.copy(), sw.fp.copy()
        sel = sw.sel.copy()
        sw.tell(np.sum((x - c) ** 2, axis=1))
        assert sw.evaluations == M * (it + 1)
        others = np.setdiff1d(np.arange(N), sel)
        assert np.array_equal(sw.p[others], p_before[others]) and np.array_equal(sw.fp[others], fp_before[others])
    assert sw.fg < 1e-2 * np.sum((hi - lo) ** 2)


def test_mutation_takes_unevaluated_particles_worst_predicted_first():
    lo, hi, c = _box(seed=2)
    N, M = 20, 6
    sur = _Exact(c)
    sw = ScreenedEMPSO(lo, hi, N, sur, K=1, warmup=0, evaluate=M, gen=10, seed=7, p_em=0.0, em_start_frac=0.0)
    sw.ask()
    sel, pred = sw.sel.copy(), sw.pred.copy()
    sw.tell(np.sum((sw.x[sel] - c) ** 2, axis=1))
    g = sw.g
    moved_to_g = {i for i in range(N) if np.array_equal(sw.x[i], np.minimum(np.maximum(g, lo), hi))}
    unevaluated = np.setdiff1d(np.arange(N), sel)
    want = set(unevaluated[np.argsort(-pred[unevaluated], kind="stable")][:sw.nm])
    assert sw.nm < len(unevaluated)
    assert want <= moved_to_g


def test_random_ranker_screen_runs_and_counts():
    lo, hi, c = _box(seed=3)
    sw = ScreenedEMPSO(lo, hi, 16, RandomRanker(4), K=3, warmup=0, evaluate=5, gen=6, seed=9)
    for _ in range(6):
        x = sw.ask()
        sw.tell(np.sum((x - c) ** 2, axis=1))
    assert sw.evaluations == 30 and np.isfinite(sw.fg)


def test_screened_swarm_checkpoint_resumes_bitwise(tmp_path):
    lo, hi, c = _box(seed=4)
    kw = dict(K=3, warmup=0, evaluate=6, gen=12, seed=13)

    def f(x):
        return np.sum((x - c) ** 2, axis=1)

    a = ScreenedEMPSO(lo, hi, 14, _Exact(c), **kw)
    for _ in range(4):
        a.tell(f(a.ask()))
    pso.save_checkpoint(str(tmp_path / "s.npz"), a)
    b = pso.load_checkpoint(str(tmp_path / "s.npz"), ScreenedEMPSO(lo, hi, 14, _Exact(c), **kw))
    for _ in range(5):
        ra, rb = a.tell(f(a.ask())), b.tell(f(b.ask()))
        assert ra == rb
    assert np.array_equal(a.x, b.x) and np.array_equal(a.sel, b.sel) and np.array_equal(a.p, b.p)


def test_candidate_moves_draw_the_empso_move():
    """candidate_moves (the ranking study's candidates) draws Eq. 1-2 moves
    with the swarm's arithmetic: from the state tell() reaches after the
    bests update, one candidate drawn from a copy of the swarm's generator is
    the swarm's own move (mutation off); every candidate lies in the box."""
    import copy

    from paper_1905_12795_amd.surrogate import candidate_moves
    lo, hi, c = _box(D=7, seed=4)
    a = pso.EMPSO(lo, hi, 12, gen=8, seed=5, elitist=False)
    for _ in range(3):
        a.tell(np.sum((a.ask() - c) ** 2, axis=1))
    f = np.sum((a.ask() - c) ** 2, axis=1)
    b = copy.deepcopy(a)
    a.tell(f)
    better = f < b.fp
    b.fp = np.where(better, f, b.fp)
    b.p = np.where(better[:, None], b.x, b.p)
    b.gi = int(np.argmin(b.fp))
    one = candidate_moves(b, 1, copy.deepcopy(b.rng))
    assert np.array_equal(one[0], a.x)
    many = candidate_moves(b, 5, np.random.Generator(np.random.PCG64(9)))
    assert many.shape == (5, 12, 7)
    assert np.all(many >= lo) and np.all(many <= hi)
    assert not np.array_equal(many[0], many[1])
