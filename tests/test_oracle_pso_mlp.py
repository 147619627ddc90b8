"""Pins of the oracle's PSO pieces (Eq. 1-3, elitist mutation) and of the FP64 surrogate MLP."""
import json
import math
import os

import numpy as np
import pytest

from oracle import mlp, pso

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_constriction_closed_forms():
    exp = json.load(open(os.path.join(GOLDEN, "empso_experiment.json")))
    chi = pso.constriction(exp["c1"], exp["c2"])
    phi = 4.1
    assert chi == pytest.approx(2.0 / (phi - 2.0 + math.sqrt(phi * phi - 4 * phi)), rel=1e-15)
    assert chi == pytest.approx(0.7298437881, abs=1e-10)
    cfg = json.load(open(os.path.join(GOLDEN, "paper_config.json")))
    assert pso.constriction(cfg["pso"]["c1"], cfg["pso"]["c2"]) == 1.0
    with pytest.raises(ValueError):
        pso.constriction(1.0, 2.0)


def test_move_special_cases():
    # x = p = g: only the inertia survives: v' = chi v (then clamped), x' = x + v'
    x = np.array([[1.0, 2.0, 3.0]])
    v = np.array([[0.5, -0.5, 10.0]])
    u = np.full((1, 3), 0.7)
    lo, hi = np.zeros(3), np.full(3, 4.0)
    vcl = np.array([1.0, 1.0, 1.0])
    xn, vn = pso.move(x, v, x.copy(), x[0].copy(), u, u, 0.5, 1.2, 2.9, vcl, lo, hi)
    assert np.array_equal(vn, [[0.25, -0.25, 1.0]])         # last component clamped to 1
    assert np.array_equal(xn, [[1.25, 1.75, 4.0]])          # box clamp at hi, velocity kept
    # zero random draws: the attraction terms vanish
    xn2, vn2 = pso.move(x, v, x + 1, x[0] + 2, np.zeros((1, 3)), np.zeros((1, 3)), 0.5, 1.2, 2.9,
                        vcl, lo, hi)
    assert np.array_equal(vn2, vn)
    # hand-worked single coordinate
    xn3, vn3 = pso.move(np.array([[1.0]]), np.array([[0.0]]), np.array([[2.0]]), np.array([3.0]),
                        np.array([[0.5]]), np.array([[0.25]]), 0.8, 1.2, 2.9, np.array([9.0]),
                        np.array([-9.0]), np.array([9.0]))
    assert vn3[0, 0] == pytest.approx(0.8 * (0.0 + 1.2 * 0.5 * 1.0 + 2.9 * 0.25 * 2.0))
    assert xn3[0, 0] == pytest.approx(1.0 + vn3[0, 0])


def test_update_bests_strict_and_ties():
    x = np.arange(8.0).reshape(4, 2)
    p = np.zeros((4, 2))
    fp = np.array([1.0, 1.0, 5.0, 0.5])
    f = np.array([1.0, 0.9, 0.5, 0.7])
    p2, fp2, gi = pso.update_bests(x, f, p, fp)
    assert np.array_equal(fp2, [1.0, 0.9, 0.5, 0.5])
    assert np.array_equal(p2[0], [0, 0]) and np.array_equal(p2[1], x[1])   # no change on equality
    assert gi == 2                                                          # tie 0.5 -> lowest index


def test_elitist_mutation_selects_worst_and_statistics():
    exp = json.load(open(os.path.join(GOLDEN, "empso_experiment.json")))
    N, D = exp["particles"], 6
    nm = int(round(exp["nm_fraction"] * N))
    assert nm == 90
    assert exp["particles"] * exp["iterations"] == exp["model_evaluations"]
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, (N, D))
    f = rng.permutation(N).astype(float)
    g = np.full(D, 0.5)
    vr = np.full(D, 1.0)
    ru = rng.random((nm, D))
    rn = rng.standard_normal((nm, D))
    xn = pso.elitist_mutation(x, f, g, nm, exp["p_em"], vr, ru, rn,
                              np.full(D, -10.0), np.full(D, 10.0))
    worst = set(np.argsort(-f)[:nm])
    changed = {i for i in range(N) if not np.array_equal(xn[i], x[i])}
    assert changed == worst
    order = sorted(range(N), key=lambda i: (-f[i], i))
    for k in range(nm):
        for d in range(D):
            want = 0.5 + 0.1 * rn[k, d] if ru[k, d] < exp["p_em"] else 0.5
            assert xn[order[k], d] == want
    # statistics over many draws: mutated fraction ~ p_em, spread 0.1 * VR
    M = 200000
    ru = rng.random((M, 1))
    rn = rng.standard_normal((M, 1))
    xm = pso.elitist_mutation(np.zeros((M, 1)), np.arange(M, dtype=float), np.zeros(1), M, 0.3,
                              np.array([2.0]), ru, rn, np.array([-1e9]), np.array([1e9]))
    mut = xm[:, 0] != 0.0
    assert abs(mut.mean() - 0.3) < 0.005
    assert abs(np.std(xm[mut, 0]) - 0.2) < 0.003


def test_gelu_identities():
    x = np.linspace(-6, 6, 1001)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert np.allclose(mlp.gelu(-x), mlp.gelu(x) - x, atol=1e-14)
    assert abs(mlp.gelu(np.array([8.0]))[0] - 8.0) < 1e-13
    h = 1e-6
    fdg = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fdg - mlp.gelu_grad(x))) < 1e-8


def test_mlp_backward_matches_finite_differences():
    sizes = [6, 16, 16, 16, 1]
    params = mlp.init_params(sizes, seed=3)
    rng = np.random.default_rng(4)
    lo, hi = np.full(6, 1400.0), np.full(6, 2700.0)
    X = rng.uniform(1400, 2700, (20, 6))
    t = rng.standard_normal(20)
    loss, grads = mlp.loss_and_grads(params, X, t, lo, hi)
    h = 1e-6
    for k in range(len(params)):
        for which in (0, 1):
            arr = params[k][which]
            flat_idx = [0, arr.size // 2, arr.size - 1]
            for fi in flat_idx:
                idx = np.unravel_index(fi, arr.shape)
                orig = arr[idx]
                arr[idx] = orig + h
                lp, _ = mlp.loss_and_grads(params, X, t, lo, hi)
                arr[idx] = orig - h
                lm, _ = mlp.loss_and_grads(params, X, t, lo, hi)
                arr[idx] = orig
                num = (lp - lm) / (2 * h)
                ana = grads[k][which][idx]
                assert abs(num - ana) <= 1e-6 * max(1.0, abs(ana)) + 1e-9, (k, which, fi, num, ana)


def test_adam_first_step_is_signed_lr():
    params = [(np.array([[1.0, -2.0]]), np.array([0.5]))]
    grads = [(np.array([[3.0, -0.01]]), np.array([-7.0]))]
    m = mlp.zeros_like(params)
    v = mlp.zeros_like(params)
    p2, _, _ = mlp.adam_step(params, grads, m, v, 1, 1e-2)
    assert np.allclose(p2[0][0], [[1.0 - 1e-2, -2.0 + 1e-2]], atol=1e-9)
    assert np.allclose(p2[0][1], [0.5 + 1e-2], atol=1e-9)


def _adam_run(adam, grads_of_step, p0, steps, lr, eps=1e-8):
    """Parameters after `steps` Adam updates of a single-tensor model whose
    gradient at step t (from 1) is grads_of_step(t)."""
    params = [(np.array(p0, dtype=np.float64), np.zeros(1))]
    m, v = mlp.zeros_like(params), mlp.zeros_like(params)
    out = []
    for t in range(1, steps + 1):
        grads = [(grads_of_step(t), np.zeros(1))]
        params, m, v = adam(params, grads, m, v, t, lr, eps=eps)
        out.append(params[0][0].copy())
    return out


def test_adam_constant_gradient_closed_form():
    # With g fixed, m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the
    # bias-corrected moments are exactly g and g^2 at every step and each
    # step moves by -lr g / (|g| + eps): after t steps p0 - t lr g / (|g| + eps).
    g = np.array([[3.0, -0.02, 1e-8, -4e-9, 250.0]])
    p0 = np.array([[0.5, -1.0, 2.0, 0.0, 7.0]])
    lr, eps = 1e-2, 1e-8
    traj = _adam_run(mlp.adam_step, lambda t: g, p0, 8, lr, eps)
    for t, p in enumerate(traj, start=1):
        want = p0 - t * lr * g / (np.abs(g) + eps)
        assert np.allclose(p, want, rtol=1e-12, atol=1e-14), (t, p, want)


def test_adam_alternating_gradient_closed_form():
    # g_t = (-1)^(t+1) g: m_t = (1 - b1) g (-1)^(t+1) (1 - (-b1)^t) / (1 + b1)
    # (a geometric sum), v_t = (1 - b2^t) g^2, step -lr m_hat / (sqrt(v_hat) + eps).
    b1, b2, lr, eps = 0.9, 0.999, 1e-3, 1e-8
    g = np.array([[2.0, -0.5, 1e-3]])
    p0 = np.zeros((1, 3))
    traj = _adam_run(mlp.adam_step, lambda t: g * (-1.0) ** (t + 1), p0, 7, lr, eps)
    p = p0.copy()
    for t in range(1, 8):
        m = (1 - b1) * g * (-1.0) ** (t + 1) * (1 - (-b1) ** t) / (1 + b1)
        v = (1 - b2 ** t) * g * g
        p = p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
        assert np.allclose(traj[t - 1], p, rtol=1e-12, atol=1e-15), t


ADAM_MUTATIONS = {
    "bias correction frozen at step 1": ("mh = M2 / (1 - b1 ** step)", "mh = M2 / (1 - b1)"),
    "second-moment correction frozen at step 1": ("vh = V2 / (1 - b2 ** step)", "vh = V2 / (1 - b2)"),
    "first moment without (1 - b1)": ("M2 = b1 * M_ + (1 - b1) * G_", "M2 = b1 * M_ + G_"),
    "eps inside the square root": ("np.sqrt(vh) + eps", "np.sqrt(vh + eps)"),
    "moment decays swapped": ("M2 = b1 * M_ + (1 - b1) * G_", "M2 = b2 * M_ + (1 - b2) * G_"),
}


@pytest.mark.parametrize("name", sorted(ADAM_MUTATIONS))
def test_planted_adam_mistake_is_caught(monkeypatch, name):
    import inspect
    import textwrap
    old, new = ADAM_MUTATIONS[name]
    src = textwrap.dedent(inspect.getsource(mlp.adam_step))
    assert old in src, name
    ns = dict(mlp.__dict__)
    exec(compile(src.replace(old, new, 1), "<mutant>", "exec"), ns)
    monkeypatch.setattr(mlp, "adam_step", ns["adam_step"])
    caught = 0
    for pin in (test_adam_first_step_is_signed_lr, test_adam_constant_gradient_closed_form,
                test_adam_alternating_gradient_closed_form):
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught > 0, name
