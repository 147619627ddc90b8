"""Host FP64 swarm (product) against the oracle's Eq. 1-3 / elitist mutation, and its invariants."""
import json
import math
import os

import numpy as np
import pytest

from oracle import pso as opso
from paper_1905_12795_amd import pso

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _sphere(x, c):
    return np.sum((x - c) ** 2, axis=1)


def test_constriction_matches_oracle_and_paper():
    assert pso.constriction(1.2, 2.9) == opso.constriction(1.2, 2.9)
    assert pso.constriction(2.0, 2.0) == 1.0


def test_iterations_bitwise_equal_to_oracle_with_documented_draws():
    rng0 = np.random.default_rng(3)
    D, N, gen = 5, 12, 10
    lo = rng0.uniform(-2, 0, D)
    hi = lo + rng0.uniform(1, 3, D)
    c = rng0.uniform(lo, hi)
    sw = pso.EMPSO(lo, hi, N, gen=gen, seed=11)
    # replay the documented draw order with an independent generator
    g = np.random.Generator(np.random.PCG64(11))
    vr = hi - lo
    lam = 0.5
    x = lo + vr * g.random((N, D))
    v = -lam * vr + 2 * lam * vr * g.random((N, D))
    p = x.copy()
    fp = np.full(N, np.inf)
    chi = opso.constriction(1.2, 2.9)
    nm = int(round(0.25 * N))
    em_start = math.ceil(0.1 * gen)
    for k in range(1, gen + 1):
        assert np.array_equal(sw.ask(), x)
        f = _sphere(x, c)
        sw.tell(f)
        p, fp, gi = opso.update_bests(x, f, p, fp)
        u1 = g.random((N, D))
        u2 = g.random((N, D))
        xn, vn = opso.move(x, v, p, p[gi], u1, u2, chi, 1.2, 2.9, lam * vr, lo, hi)
        if k >= em_start:
            ru = g.random((nm, D))
            rn = g.standard_normal((nm, D))
            xn = opso.elitist_mutation(xn, f, p[gi], nm, 0.3, vr, ru, rn, lo, hi)
        x, v = xn, vn
        assert np.array_equal(sw.x, x) and np.array_equal(sw.v, v), k
        assert np.array_equal(sw.p, p) and sw.gi == gi
    assert sw.evaluations == N * gen


def test_monotone_transform_gives_identical_swarm():
    lo, hi = np.zeros(4), np.ones(4)
    a = pso.EMPSO(lo, hi, 10, gen=15, seed=5)
    b = pso.EMPSO(lo, hi, 10, gen=15, seed=5)
    c = np.full(4, 0.3)
    for _ in range(15):
        f = _sphere(a.ask(), c)
        assert np.array_equal(a.ask(), b.ask())
        a.tell(f)
        b.tell(np.exp(f) / 3.0 + 7.0)
    assert np.array_equal(a.x, b.x) and a.gi == b.gi


def test_checkpoint_resume_is_bitwise(tmp_path):
    lo, hi = -np.ones(6), np.ones(6)
    c = np.linspace(-0.5, 0.5, 6)
    ref = pso.EMPSO(lo, hi, 16, gen=20, seed=9)
    for _ in range(20):
        ref.tell(_sphere(ref.ask(), c))
    a = pso.EMPSO(lo, hi, 16, gen=20, seed=9)
    for _ in range(8):
        a.tell(_sphere(a.ask(), c))
    path = str(tmp_path / "ck.npz")
    pso.save_checkpoint(path, a)
    b = pso.load_checkpoint(path, pso.EMPSO(lo, hi, 16, gen=20, seed=123))
    for _ in range(12):
        b.tell(_sphere(b.ask(), c))
    assert np.array_equal(b.x, ref.x) and np.array_equal(b.fp, ref.fp) and b.history == ref.history


def test_converges_on_sphere_and_em_improves_on_it():
    lo, hi = -5 * np.ones(10), 5 * np.ones(10)
    c = np.full(10, 1.234)
    res = {}
    for em in (True, False):
        finals = []
        for seed in range(3):
            s = pso.EMPSO(lo, hi, 30, gen=150, seed=seed, elitist=em)
            for _ in range(150):
                s.tell(_sphere(s.ask(), c))
            finals.append(s.fg)
        res[em] = np.median(finals)
    assert res[True] < 1e-3
    assert res[True] <= res[False]


def test_paper_experiment_counts():
    exp = json.load(open(os.path.join(GOLDEN, "empso_experiment.json")))
    s = pso.EMPSO(np.zeros(3), np.ones(3), exp["particles"], gen=exp["iterations"],
                  nm_frac=exp["nm_fraction"], p_em=exp["p_em"], em_start_frac=exp["em_start_fraction"],
                  c1=exp["c1"], c2=exp["c2"], seed=0)
    assert s.nm == 90 and s.em_start == exp["em_start_iteration"]
    assert s.chi == pytest.approx(0.7298437881, abs=1e-10)
    for _ in range(exp["iterations"]):
        s.tell(np.sum(s.ask() ** 2, axis=1))
    assert s.evaluations == exp["model_evaluations"]


def test_velocity_and_box_clamps_hold():
    lo, hi = np.zeros(3), np.ones(3)
    s = pso.EMPSO(lo, hi, 20, gen=30, seed=2, lam=0.1)
    for _ in range(30):
        s.tell(np.sum((s.ask() - 2.0) ** 2, axis=1))        # optimum outside the box
        assert np.all(s.x >= lo) and np.all(s.x <= hi)
        assert np.all(np.abs(s.v) <= 0.1 + 1e-15)
    assert np.allclose(s.g, hi)


def test_nonfinite_fitness_never_becomes_best():
    s = pso.EMPSO(np.zeros(2), np.ones(2), 4, gen=3, seed=0)
    s.tell(np.array([np.nan, 1.0, np.inf, 2.0]))
    assert s.gi == 1 and np.isinf(s.fp[0]) and np.isinf(s.fp[2])
