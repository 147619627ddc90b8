"""Trace-normalised misfit on the GPU against the FP64 oracle (run on an MI355X).

Every trace of the modelled and of the observed data is divided by its own l2
norm before the l2 misfit, so the observed data here carry an amplitude the
modelling does not know (a different factor per shot). The geometries give
every receiver a physical arrival within the record (checked from the oracle's
traces): a trace with no arrival holds only the scheme's numerical precursor,
which normalisation would raise to full weight.

Bars: fitness within 2e-4 relative (in square-root form near the optimum,
against the sqrt of the number of traces, each of unit norm after
normalisation); gradient within 1e-3 relative L2, the bars of the l2 path.
"""
import copy
import sys

import numpy as np
import pytest
import torch

from oracle import fd as ofd
from workloads.configs import config

pytestmark = pytest.mark.gpu

REL = 2e-4
REL_G = 1e-3
SCALE = (3.7, 0.2)          # unknown source amplitude per shot of the observed data


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def gfd():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1905_12795_amd import fd
    return fd


def _geom():
    """Two x tiles at every depth, a ragged z tail, two shots, receivers every other column."""
    g = copy.deepcopy(config("tiny"))
    g.update(nz=61, nx=201, nbl=40, tmax=1.2, ncz=3, ncx=4, misfit="trace_normalised")
    g["src"] = [[0.0, 500.0], [20.0, 1500.0]]
    g["rec"] = [[0.0, 10.0 * j] for j in range(0, 201, 2)]
    return g


def _tiny():
    g = copy.deepcopy(config("tiny"))
    g.update(nz=21, nx=31, nbl=6, tmax=0.25, f0=15.0, ncz=2, ncx=3, misfit="trace_normalised")
    g["src"] = [[0.0, 100.0], [50.0, 230.0]]
    g["rec"] = [[0.0, 10.0 * j] for j in range(0, 31, 3)]
    return g


def _models(nz, nx, dz, dx):
    z = np.arange(nz)[:, None] * dz
    x = np.arange(nx)[None, :] * dx
    vp = 1800.0 + 600.0 * z / z.max() + 80.0 * np.sin(x / 90.0)
    truth = vp + 150.0 * np.exp(-((z - 0.5 * z.max()) ** 2 + (x - 0.55 * x.max()) ** 2) / (0.05 * (x.max() ** 2)))
    return vp, truth


def _observed(op, truth):
    d = ofd.forward_shots(op, truth)
    peak = np.abs(d).max(axis=1)                              # [shot][receiver]
    assert peak.min() >= 1e-4 * peak.max(), "a receiver without a physical arrival"
    return (d * np.asarray(SCALE)[:, None, None]).astype(np.float32)


def _fit_close(fg, fo, ntr):
    if fo >= 1e-2 * 0.5 * ntr:
        return abs(fg - fo) <= REL * fo
    return abs(np.sqrt(2 * fg) - np.sqrt(2 * fo)) <= REL * np.sqrt(ntr)


def test_normalised_fitness_matches_oracle_and_is_tiling_invariant(gfd):
    g = _geom()
    op = ofd.Problem(g)
    gp = gfd.Problem(g, dt=op.dt, nt=op.nt)
    rng = np.random.default_rng(21)
    truth = rng.uniform(1600, 2500, 12)
    dobs = _observed(op, ofd.vp_from_nodes(truth, 3, 4, g["nz"], g["nx"]))
    X = rng.uniform(1400, 2700, (5, 12))
    X[0] = truth
    fo, _ = ofd.fitness_batch(op, X.astype(np.float32).astype(np.float64), dobs)
    fb = gfd.FitnessBatch([gp], [torch.tensor(dobs, device="cuda")], [0] * 5)
    ntr = op.nshots * op.nrec
    ref = None
    for bz, T, graph in ((20, 1, 0), (40, 2, 1), (160, 4, 1), (320, 3, 1)):
        tu = gfd.default_tuning()
        tu.bz, tu.tsteps, tu.use_graph = bz, T, graph
        fg = fb(X, tuning=tu).cpu()
        if ref is None:
            ref = fg
            _say("normalised fitness gpu", fg.numpy(), "oracle", fo)
            for k in range(5):
                assert _fit_close(float(fg[k]), fo[k], ntr), (k, float(fg[k]), fo[k])
        else:
            assert torch.equal(fg, ref), (bz, T, graph)
    assert float(ref[0]) < 1e-6 * ntr                  # the true model fits data of any amplitude


def test_scaled_gpu_data_give_a_vanishing_misfit(gfd):
    g = _geom()
    gp = gfd.Problem(g)
    rng = np.random.default_rng(22)
    X = rng.uniform(1500, 2600, (1, 12))
    vpt = gfd.vp_from_nodes(gp, torch.tensor(X, dtype=torch.float32, device="cuda"))[0].contiguous()
    obs = gfd.forward_shots(gp, vpt) * torch.tensor(SCALE, device="cuda")[:, None, None]
    f = float(gfd.FitnessBatch([gp], [obs], [0])(X)[0])
    _say("scaled self-data misfit", f)
    assert 0.0 <= f < 1e-10 * gp.nshots * gp.nrec           # each trace's 1 - cos is clamped at 0
    mis, grad = gfd.gradient(gp, vpt, obs)
    assert float(mis) < 1e-10 * gp.nshots * gp.nrec
    assert float(grad.abs().max()) < 1e-3 * _gradient_scale(gfd, gp, vpt, obs)


def _gradient_scale(gfd, gp, vpt, obs):
    """Size of the gradient of a clearly wrong model against the same data."""
    _, g = gfd.gradient(gp, (vpt * 1.05).clamp(max=gp.vmax), obs)
    return float(g.abs().max())


@pytest.mark.parametrize("geom", [_tiny, _geom])
def test_normalised_gradient_matches_oracle_and_checkpointing_is_invariant(gfd, geom):
    g = geom()
    op = ofd.Problem(g)
    gp = gfd.Problem(g, dt=op.dt, nt=op.nt)
    vp, truth = _models(op.nz, op.nx, op.dz, op.dx)
    dobs = _observed(op, truth)
    Jo, go = ofd.gradient(op, vp.astype(np.float32).astype(np.float64), dobs)
    vpt = torch.tensor(vp, dtype=torch.float32, device="cuda")
    obs = torch.tensor(dobs, device="cuda")
    ref = None
    for K in (0, 1, 7, op.nt):
        mis, grad = gfd.gradient(gp, vpt, obs, checkpoint_every=K)
        if ref is None:
            ref = (mis.clone(), grad.clone())
            e = float(np.linalg.norm(grad.cpu().numpy() - go) / np.linalg.norm(go))
            _say(geom.__name__, "nt", op.nt, "normalised gradient rel L2", e, "misfit", float(mis), Jo)
            assert e <= REL_G
            assert float(mis) == pytest.approx(Jo, rel=REL)
        else:
            assert torch.equal(mis, ref[0]) and torch.equal(grad, ref[1]), K


def test_normalised_gradient_misfit_equals_fitness(gfd):
    g = _geom()
    gp = gfd.Problem(g)
    rng = np.random.default_rng(23)
    X = rng.uniform(1500, 2600, (1, 12))
    vpt = gfd.vp_from_nodes(gp, torch.tensor(X, dtype=torch.float32, device="cuda"))[0].contiguous()
    _, truth = _models(g["nz"], g["nx"], g["dz"], g["dx"])
    obs = gfd.forward_shots(gp, torch.tensor(truth, dtype=torch.float32, device="cuda"))
    obs = obs * torch.tensor(SCALE, device="cuda")[:, None, None]
    f = float(gfd.FitnessBatch([gp], [obs], [0])(X)[0])
    mis, _ = gfd.gradient(gp, vpt, obs)
    assert float(mis) == pytest.approx(f, rel=1e-6)


def test_l2_and_normalised_problems_in_one_process_keep_their_misfits(gfd):
    """Two problems that differ only in the misfit: each batch scores with its own."""
    g = _geom()
    gl2 = dict(g, misfit="l2")
    pn, pl = gfd.Problem(g), gfd.Problem(gl2)
    rng = np.random.default_rng(24)
    X = rng.uniform(1500, 2600, (2, 12))
    obs = torch.tensor(rng.standard_normal((2, pl.nt, pl.nrec)).astype(np.float32), device="cuda")
    fn = gfd.FitnessBatch([pn], [obs], [0, 0])(X).cpu().numpy()
    fl = gfd.FitnessBatch([pl], [obs], [0, 0])(X).cpu().numpy()
    # random observed traces are nearly orthogonal to any model's: about 1 per trace
    assert np.all(np.abs(fn / (pn.nshots * pn.nrec) - 1.0) < 0.1), fn
    assert np.all(fl > 0.4 * float((obs.double() ** 2).sum()))
    # one batch mixing both problems gives each particle its own problem's misfit, bit for bit
    Xm = np.concatenate([X, X])
    fm = gfd.FitnessBatch([pn, pl], [obs, obs], [0, 0, 1, 1])(Xm).cpu().numpy()
    assert np.array_equal(fm[:2], fn) and np.array_equal(fm[2:], fl), (fm, fn, fl)


@pytest.mark.parametrize("kind", ["l2", "trace_normalised"])
def test_traces_misfit_matches_oracle(gfd, kind):
    g = dict(_geom(), misfit=kind, tmax=0.2)
    gp = gfd.Problem(g)
    rng = np.random.default_rng(25)
    d = rng.standard_normal((3, gp.nt, gp.nrec)).astype(np.float32)
    o = (0.6 * d + rng.standard_normal(d.shape)).astype(np.float32)
    d[1, :, 7] = 0.0                                  # a zero modelled trace
    o[2, :, 11] = 0.0                                 # a zero observed trace
    o[0, :, 3] = 0.0
    d[0, :, 3] = 0.0                                  # both zero
    want = ofd.misfit_normalised(d, o) if kind == "trace_normalised" else ofd.misfit(d, o)
    got = float(gfd.traces_misfit(gp, torch.tensor(d, device="cuda"), torch.tensor(o, device="cuda")))
    assert got == pytest.approx(want, rel=1e-6)
    d[2, 5, 9] = np.inf
    assert float(gfd.traces_misfit(gp, torch.tensor(d, device="cuda"), torch.tensor(o, device="cuda"))) == np.inf
    e = torch.zeros((0, gp.nt, gp.nrec), device="cuda")
    assert float(gfd.traces_misfit(gp, e, e)) == 0.0


def test_traces_misfit_of_forward_traces_equals_fitness(gfd):
    g = _geom()
    gp = gfd.Problem(g)
    rng = np.random.default_rng(26)
    X = rng.uniform(1500, 2600, (1, 12))
    vpt = gfd.vp_from_nodes(gp, torch.tensor(X, dtype=torch.float32, device="cuda"))[0].contiguous()
    _, truth = _models(g["nz"], g["nx"], g["dz"], g["dx"])
    obs = gfd.forward_shots(gp, torch.tensor(truth, dtype=torch.float32, device="cuda")) * 0.3
    f = float(gfd.FitnessBatch([gp], [obs], [0])(X)[0])
    m = float(gfd.traces_misfit(gp, gfd.forward_shots(gp, vpt), obs))
    assert m == pytest.approx(f, rel=1e-6)


def test_traces_without_arrivals_fitness_and_gradient_match_oracle(gfd):
    """A record too short for the far receivers: their traces hold only the
    scheme's precursor (far below the floor). Fitness and gradient match the
    oracle, the gradient is finite, and neither depends on the scale of the
    observed data (1e-12 .. 1e12)."""
    g = dict(_geom(), tmax=0.3)
    op = ofd.Problem(g)
    gp = gfd.Problem(g, dt=op.dt, nt=op.nt)
    vp, truth = _models(op.nz, op.nx, op.dz, op.dx)
    d = ofd.forward_shots(op, truth)
    peak = np.abs(d).max(axis=1)
    assert np.sum(peak < 1e-12 * peak.max()) >= 10, "the geometry must have receivers without arrivals"
    dobs = (d * np.asarray(SCALE)[:, None, None]).astype(np.float32)
    ntr = op.nshots * op.nrec
    rng = np.random.default_rng(27)
    X = rng.uniform(1500, 2600, (3, 12))
    fo, _ = ofd.fitness_batch(op, X.astype(np.float32).astype(np.float64), dobs)
    obs = torch.tensor(dobs, device="cuda")
    fb = gfd.FitnessBatch([gp], [obs], [0] * 3)
    fg = fb(X).cpu()
    tu = gfd.default_tuning()
    tu.bz, tu.tsteps = 40, 2
    assert torch.equal(fb(X, tuning=tu).cpu(), fg)
    _say("no-arrival geometry fitness", fg.numpy(), fo)
    for k in range(3):
        assert _fit_close(float(fg[k]), fo[k], ntr), (k, float(fg[k]), fo[k])
    Jo, go = ofd.gradient(op, vp.astype(np.float32).astype(np.float64), dobs)
    vpt = torch.tensor(vp, dtype=torch.float32, device="cuda")
    mis, grad = gfd.gradient(gp, vpt, obs)
    assert bool(torch.isfinite(grad).all())
    e = float(np.linalg.norm(grad.cpu().numpy() - go) / np.linalg.norm(go))
    _say("no-arrival geometry gradient rel L2", e, "misfit", float(mis), Jo)
    assert e <= REL_G
    assert float(mis) == pytest.approx(Jo, rel=REL)
    for s in (1e-12, 1e12):
        ms, gs = gfd.gradient(gp, vpt, obs * s)
        fs = gfd.FitnessBatch([gp], [obs * s], [0] * 3)(X).cpu()
        assert bool(torch.isfinite(gs).all()), s
        assert float(ms) == pytest.approx(float(mis), rel=1e-5), s
        assert torch.allclose(fs, fg, rtol=1e-5), s
        assert float(torch.linalg.norm(gs - grad) / torch.linalg.norm(grad)) <= 1e-4, s


@pytest.mark.timeout(600)
def test_crime_free_full_size_directional_derivative(gfd):
    """The normalised gradient at full size on the crime-free data (16 shots,
    nt = 8114, far receivers below the floor in a linear 1.5-5.5 km/s model)
    against central differences of the GPU misfit along a smooth direction.
    The normalised misfit bends more than the l2 one over the steps used
    here, so the central differences at 10 and 20 m/s are combined by
    Richardson extrapolation (the step-squared error cancels); bar 5e-3."""
    from paper_1905_12795_amd import search
    from workloads.configs import true_model
    g = dict(config("crime_free"), misfit="trace_normalised")
    gp = gfd.Problem(g)
    obs = search.observed_for(g, gp, true_model(g))
    z = np.arange(g["nz"])[:, None] * g["dz"]
    x = np.arange(g["nx"])[None, :] * g["dx"]
    vpt = torch.tensor(1500.0 + 4000.0 * z / z.max() + 0 * x, dtype=torch.float32, device="cuda")
    mis, grad = gfd.gradient(gp, vpt, obs)
    assert bool(torch.isfinite(grad).all())
    from paper_1905_12795_amd import fwi
    d = torch.tensor(np.sin(z / 400.0) * np.cos(x / 900.0), dtype=torch.float32, device="cuda")

    def central(eps):
        return (fwi.model_misfit(gp, vpt + eps * d, obs) - fwi.model_misfit(gp, vpt - eps * d, obs)) / (2 * eps)

    c10, c20 = central(10.0), central(20.0)
    rich = (4.0 * c10 - c20) / 3.0
    dot = float(torch.sum(grad.double() * d.double()))
    _say("normalised directional derivative: adjoint %.6g; central differences %.6g (10 m/s), %.6g (20 m/s), "
         "extrapolated %.6g (misfit %.6g)" % (dot, c10, c20, rich, float(mis)))
    assert dot == pytest.approx(rich, rel=5e-3)


def test_local_fwi_with_the_normalised_misfit(gfd):
    """Data of unknown amplitude (a factor per shot): the local FWI with the
    trace-normalised misfit lowers the misfit monotonically and the model error."""
    from paper_1905_12795_amd import fwi
    g = _geom()
    gp = gfd.Problem(g)
    vp, truth = _models(g["nz"], g["nx"], g["dz"], g["dx"])
    obs = gfd.forward_shots(gp, torch.tensor(truth, dtype=torch.float32, device="cuda"))
    obs = obs * torch.tensor(SCALE, device="cuda")[:, None, None]
    v, hist = fwi.invert(gp, obs, vp, 8)
    J = [h["misfit"] for h in hist]
    _say("normalised local FWI misfits", J, "rms model error", fwi.rms_error(vp, truth), "->",
         fwi.rms_error(v, truth))
    assert all(b <= a for a, b in zip(J, J[1:]))
    assert J[-1] < 0.5 * J[0]
    assert fwi.rms_error(v, truth) < fwi.rms_error(vp, truth)
