"""Seeded random small geometries against the oracle (run on an MI355X).

Each case draws a grid (8..80 x 8..200 points, absorbing layers of 0, 1, 3,
8, 20 or 40 points in turn, equal or unequal spacing), 1..3 sources anywhere on the grid, a
receiver row at any depth with 1..60 receivers, a node grid of 2..5 x 2..8
nodes and a record long enough for the wave to cross the grid. The GPU
traces must match the oracle's (2e-4 relative L2), and the fitness of three
particles must match the oracle at two random tunings that agree bit for bit.
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


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def gfd():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1905_12795_amd import fd
    return fd


def _random_geom(seed, spacing=None):
    rng = np.random.default_rng(1000 + seed)
    g = copy.deepcopy(config("tiny"))
    nz, nx = int(rng.integers(8, 81)), int(rng.integers(8, 201))
    aniso = rng.random() < 0.4
    dz = float(rng.choice([6.0, 8.0, 12.0])) if aniso else 10.0
    dx = float(rng.choice([7.0, 10.0, 14.0])) if aniso else 10.0
    if spacing is not None:
        dz, dx = spacing
    cross = np.hypot((nz - 1) * dz, (nx - 1) * dx) / 1400.0          # slowest crossing time
    g.update(nz=nz, nx=nx, nbl=(0, 1, 3, 8, 20, 40)[seed % 6], dz=dz, dx=dx, f0=15.0,
             tmax=float(cross + 2.0 / 15.0))
    ncz, ncx = int(rng.integers(2, min(nz, 5) + 1)), int(rng.integers(2, min(nx, 8) + 1))
    g.update(ncz=ncz, ncx=ncx)
    g["src"] = [[float(rng.integers(0, nz)) * dz, float(rng.integers(0, nx)) * dx]
                for _ in range(int(rng.integers(1, 4)))]
    row = int(rng.integers(0, nz))
    cols = np.sort(rng.choice(nx, size=int(rng.integers(1, min(nx, 60) + 1)), replace=False))
    g["rec"] = [[row * dz, float(c) * dx] for c in cols]
    g["node_lo"], g["node_hi"] = np.full(ncz * ncx, 1400.0), np.full(ncz * ncx, 2700.0)
    return g, rng


def _fit_close(fg, fo, dobs_norm2):
    if fo >= 1e-2 * 0.5 * dobs_norm2:
        return abs(fg - fo) <= REL * fo
    return abs(np.sqrt(2 * fg) - np.sqrt(2 * fo)) <= REL * np.sqrt(dobs_norm2)


@pytest.mark.parametrize("seed", range(16))
def test_random_geometry_matches_oracle(gfd, seed):
    g, rng = _random_geom(seed)
    op = ofd.Problem(g)
    gp = gfd.Problem(g, dt=op.dt, nt=op.nt)
    ncz, ncx = g["ncz"], g["ncx"]
    truth = rng.uniform(1500, 2600, ncz * ncx)
    vp = ofd.vp_from_nodes(truth, ncz, ncx, g["nz"], g["nx"])
    to = ofd.forward_shots(op, vp)
    tg = gfd.forward_shots(gp, torch.tensor(vp, dtype=torch.float32, device="cuda")).cpu().numpy()
    e = float(np.linalg.norm(tg - to) / np.linalg.norm(to))
    _say("seed %d: %dx%d nbl %d d %g/%g, %d shots, %d receivers on row %d, nt %d: traces rel L2 %.3g"
         % (seed, g["nz"], g["nx"], g["nbl"], g["dz"], g["dx"], op.nshots, op.nrec,
            int(round(g["rec"][0][0] / g["dz"])), op.nt, e))
    assert e <= REL
    dobs = to.astype(np.float32)
    X = rng.uniform(1400, 2700, (3, ncz * ncx))
    X[0] = truth
    fo, _ = ofd.fitness_batch(op, X.astype(np.float32).astype(np.float64), dobs)
    fb = gfd.FitnessBatch([gp], [torch.tensor(dobs, device="cuda")], [0] * 3)
    outs = []
    for _ in range(2):
        tu = gfd.default_tuning()
        tu.bz = int(rng.choice([20, 40, 80, 160, 240, 320]))
        tu.tsteps = int(rng.integers(1, 5))
        tu.use_graph = int(rng.integers(0, 2))
        outs.append(((tu.bz, tu.tsteps, tu.use_graph), fb(X, tuning=tu).cpu()))
    assert torch.equal(outs[0][1], outs[1][1]), (outs[0][0], outs[1][0])
    fg = outs[0][1].numpy().astype(np.float64)
    n2 = float(np.sum(dobs.astype(np.float64) ** 2))
    for k in range(3):
        assert _fit_close(fg[k], fo[k], n2), (k, fg[k], fo[k], outs[0][0])


@pytest.mark.parametrize("seed", range(8))
def test_random_geometry_gradient_matches_oracle(gfd, seed):
    """The misfit gradient (l2 on even seeds, trace-normalised on odd ones, the
    observed data then scaled per shot) on random small geometries: within the
    gradient bar (1e-3 relative L2) of the oracle's discrete adjoint, misfit
    within 2e-4, and identical for two checkpoint intervals."""
    g, rng = _random_geom(100 + seed)
    if seed % 2:
        g["misfit"] = "trace_normalised"
    op = ofd.Problem(g)
    gp = gfd.Problem(g, dt=op.dt, nt=op.nt)
    ncz, ncx = g["ncz"], g["ncx"]
    truth = ofd.vp_from_nodes(rng.uniform(1500, 2600, ncz * ncx), ncz, ncx, g["nz"], g["nx"])
    vp = ofd.vp_from_nodes(rng.uniform(1500, 2600, ncz * ncx), ncz, ncx, g["nz"], g["nx"])
    vp = vp.astype(np.float32).astype(np.float64)
    dobs = ofd.forward_shots(op, truth)
    if seed % 2:
        dobs = dobs * rng.uniform(0.1, 10.0, (op.nshots, 1, 1))
    dobs = dobs.astype(np.float32)
    Jo, go = ofd.gradient(op, vp, dobs)
    vpt = torch.tensor(vp, dtype=torch.float32, device="cuda")
    obs = torch.tensor(dobs, device="cuda")
    mis, grad = gfd.gradient(gp, vpt, obs)
    e = float(np.linalg.norm(grad.cpu().numpy() - go) / np.linalg.norm(go))
    _say("seed %d (%s): %dx%d nbl %d, %d shots, nt %d: gradient rel L2 %.3g, misfit %.6g vs %.6g"
         % (seed, g.get("misfit", "l2"), g["nz"], g["nx"], g["nbl"], op.nshots, op.nt, e, float(mis), Jo))
    assert e <= 1e-3
    assert float(mis) == pytest.approx(Jo, rel=REL)
    m2, g2 = gfd.gradient(gp, vpt, obs, checkpoint_every=int(rng.integers(1, 40)))
    assert torch.equal(m2, mis) and torch.equal(g2, grad)


@pytest.mark.parametrize("seed", range(5))
def test_random_mixed_batch_equals_separate_batches(gfd, seed):
    """Three random grids (shared dt and nt) in one batch, particles assigned
    at random: the mixed batch equals the per-grid batches bit for bit at two
    random tunings, and one particle per grid matches the oracle. The grids of
    a batch share one spacing, equal (seeds 0, 2) or unequal (1, 3); seed 4
    mixes equal- and unequal-spacing grids, which the batch runs with the
    general Laplacian, so its equal-spacing runs match their own batch (the
    isotropic grouping) to rounding instead of bit for bit."""
    spacing = [(10.0, 10.0), (8.0, 12.0), (7.0, 7.0), (12.0, 6.0)]
    if seed < 4:
        geoms = [_random_geom(200 + 3 * seed + k, spacing[seed])[0] for k in range(3)]
    else:
        geoms = [_random_geom(200 + 3 * seed + k, s)[0] for k, s in enumerate([(10.0, 10.0), (8.0, 12.0), (10.0, 10.0)])]
    rng = np.random.default_rng(300 + seed)
    tmax = max(g["tmax"] for g in geoms)
    for g in geoms:
        g["tmax"] = tmax
    ops = [ofd.Problem(g) for g in geoms]
    dt = min(o.dt for o in ops)
    nt = ofd.n_steps(tmax, dt)
    ops = [ofd.Problem(g, dt=dt, nt=nt) for g in geoms]
    gps = [gfd.Problem(g, dt=dt, nt=nt) for g in geoms]
    Dmax = max(g["ncz"] * g["ncx"] for g in geoms)
    npart = 7
    pop = [int(q) for q in rng.integers(0, 3, npart)]
    pop[:3] = [0, 1, 2]                                        # every grid has a particle
    X = rng.uniform(1450, 2650, (npart, Dmax))
    dobs = []
    for o, g in zip(ops, geoms):
        vp = ofd.vp_from_nodes(rng.uniform(1500, 2600, g["ncz"] * g["ncx"]), g["ncz"], g["ncx"], g["nz"], g["nx"])
        dobs.append(ofd.forward_shots(o, vp).astype(np.float32))
    obs = [torch.tensor(d, device="cuda") for d in dobs]
    fb = gfd.FitnessBatch(gps, obs, pop)
    outs = []
    for _ in range(2):
        tu = gfd.default_tuning()
        tu.bz = int(rng.choice([20, 40, 80, 160, 240, 320]))
        tu.tsteps = int(rng.integers(1, 5))
        outs.append(fb(X, tuning=tu).cpu())
        for q in range(3):
            idx = [p for p in range(npart) if pop[p] == q]
            sep = gfd.FitnessBatch([gps[q]], [obs[q]], [0] * len(idx))(X[idx][:, :geoms[q]["ncz"] * geoms[q]["ncx"]],
                                                                      tuning=tu).cpu()
            if seed < 4:
                assert torch.equal(sep, outs[-1][idx]), (seed, q, tu.bz, tu.tsteps)
            else:
                assert torch.allclose(sep, outs[-1][idx], rtol=1e-5, atol=0), (seed, q, sep, outs[-1][idx])
    assert torch.equal(outs[0], outs[1])
    for q in range(3):
        D = geoms[q]["ncz"] * geoms[q]["ncx"]
        fo, _ = ofd.fitness_batch(ops[q], X[[q], :D].astype(np.float32).astype(np.float64), dobs[q])
        n2 = float(np.sum(dobs[q].astype(np.float64) ** 2))
        assert _fit_close(float(outs[0][q]), fo[0], n2), (seed, q, float(outs[0][q]), fo[0])
