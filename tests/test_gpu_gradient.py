"""GPU misfit gradient (discrete adjoint with checkpoints) against the FP64
oracle's (run on an MI355X).

Bar: the forward traces and misfits carry the 2e-4 FP32 bar; the gradient is a
time sum of products of a forward and an adjoint field, each within that bar,
so it is held to 1e-3 relative L2 against the oracle. Checkpoint intervals
change only the schedule, so every interval gives the same bits; data made
by the fitness path's own kernels give an exactly zero residual and gradient.
"""
import copy
import sys

import numpy as np
import pytest
import torch

from oracle import fd as ofd
from workloads.configs import config, true_model

pytestmark = pytest.mark.gpu

REL_G = 1e-3
REL = 2e-4


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def gfd():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1905_12795_amd import fd
    return fd


def _tiny():
    g = copy.deepcopy(config("tiny"))
    g.update(nz=21, nx=31, nbl=6, tmax=0.25, f0=15.0, ncz=2, ncx=3)
    g["src"] = [[0.0, 100.0], [50.0, 230.0]]
    g["rec"] = [[0.0, 10.0 * j] for j in range(0, 31, 3)]
    return g


def _wide():
    """Several x tiles, a ragged z tail, two shots, receivers every other column."""
    g = copy.deepcopy(config("tiny"))
    g.update(nz=61, nx=301, nbl=40, tmax=0.3, ncz=3, ncx=4)
    g["src"] = [[0.0, 1000.0], [20.0, 2230.0]]
    g["rec"] = [[0.0, 10.0 * j] for j in range(0, 301, 2)]
    return g


def _models(nz, nx, dz, dx):
    z = np.arange(nz)[:, None] * dz
    x = np.arange(nx)[None, :] * dx
    vp = 1800.0 + 600.0 * z / z.max() + 80.0 * np.sin(x / 90.0)        # below the 2700 m/s vmax
    truth = vp + 150.0 * np.exp(-((z - 0.5 * z.max()) ** 2 + (x - 0.55 * x.max()) ** 2) / (0.05 * (x.max() ** 2)))
    return vp, truth


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("geom", [_tiny, _wide])
def test_gradient_matches_oracle_and_checkpointing_is_invariant(gfd, geom):
    g = geom()
    op = ofd.Problem(g)
    gp = gfd.Problem(g, dt=op.dt, nt=op.nt)
    vp, truth = _models(op.nz, op.nx, op.dz, op.dx)
    dobs = ofd.forward_shots(op, truth)
    Jo, go = ofd.gradient(op, vp.astype(np.float32).astype(np.float64), dobs)
    vpt = torch.tensor(vp, dtype=torch.float32, device="cuda")
    obs = torch.tensor(dobs.astype(np.float32), device="cuda")
    ref = None
    for K in (0, 1, 7, op.nt):
        mis, grad = gfd.gradient(gp, vpt, obs, checkpoint_every=K)
        if ref is None:
            ref = (mis.clone(), grad.clone())
            e = _rel(grad.cpu().numpy(), go)
            _say(geom.__name__, "nt", op.nt, "gradient rel L2", e, "misfit", float(mis), Jo)
            assert e <= REL_G
            assert float(mis) == pytest.approx(Jo, rel=REL)
        else:
            assert torch.equal(mis, ref[0]) and torch.equal(grad, ref[1]), K


def test_data_from_the_fitness_kernels_give_zero_residual(gfd):
    g = _wide()
    gp = gfd.Problem(g)
    vp, _ = _models(g["nz"], g["nx"], g["dz"], g["dx"])
    vpt = torch.tensor(vp, dtype=torch.float32, device="cuda")
    obs = gfd.forward_shots(gp, vpt)
    mis, grad = gfd.gradient(gp, vpt, obs)
    assert float(mis) == 0.0
    assert torch.count_nonzero(grad).item() == 0


def test_gradient_misfit_equals_fitness_of_the_same_model(gfd):
    g = _wide()
    gp = gfd.Problem(g)
    rng = np.random.default_rng(3)
    X = rng.uniform(1500, 2600, (1, 12))
    vpt = gfd.vp_from_nodes(gp, torch.tensor(X, dtype=torch.float32, device="cuda"))[0].contiguous()
    _, truth = _models(g["nz"], g["nx"], g["dz"], g["dx"])
    obs = gfd.forward_shots(gp, torch.tensor(truth, dtype=torch.float32, device="cuda"))
    f = float(gfd.FitnessBatch([gp], [obs], [0])(X)[0])
    mis, _ = gfd.gradient(gp, vpt, obs)
    assert float(mis) == pytest.approx(f, rel=1e-6)


@pytest.mark.timeout(600)
def test_realistic_full_size_directional_derivative(gfd):
    """At the benchmark's full size (16 shots, nt = 8114) the oracle cannot keep
    every time level, so the gradient is checked against central differences
    of the GPU misfit itself along a smooth direction (FP32 misfits, FP64
    sums: a 1e-2 bar)."""
    import time
    g = config("realistic")
    gp = gfd.Problem(g)
    truth = true_model(g)
    obs = gfd.forward_shots(gp, torch.tensor(truth, dtype=torch.float32, device="cuda"))
    z = np.arange(g["nz"])[:, None] * g["dz"]
    x = np.arange(g["nx"])[None, :] * g["dx"]
    vp = 1500.0 + 4000.0 * z / z.max() + 0 * x
    vpt = torch.tensor(vp, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.time()
    mis, grad = gfd.gradient(gp, vpt, obs)
    torch.cuda.synchronize()
    _say("realistic gradient %.2fs, misfit %.6g" % (time.time() - t0, float(mis)))
    d = torch.tensor(np.sin(z / 400.0) * np.cos(x / 900.0), dtype=torch.float32, device="cuda")
    eps = 20.0
    mp, _ = gfd.gradient(gp, vpt + eps * d, obs)
    mm, _ = gfd.gradient(gp, vpt - eps * d, obs)
    fd_val = (float(mp) - float(mm)) / (2 * eps)
    dot = float(torch.sum(grad.double() * d.double()))
    _say("directional derivative: adjoint %.6g, central difference %.6g" % (dot, fd_val))
    assert dot == pytest.approx(fd_val, rel=1e-2)


def test_local_fwi_reduces_misfit_and_model_error(gfd):
    from paper_1905_12795_amd import fwi
    g = _wide()
    gp = gfd.Problem(g)
    vp, truth = _models(g["nz"], g["nx"], g["dz"], g["dx"])
    obs = gfd.forward_shots(gp, torch.tensor(truth, dtype=torch.float32, device="cuda"))
    v, hist = fwi.invert(gp, obs, vp, 8)
    J = [h["misfit"] for h in hist]
    _say("local FWI misfits", J, "rms model error", fwi.rms_error(vp, truth), "->", fwi.rms_error(v, truth))
    assert all(b <= a for a, b in zip(J, J[1:]))
    assert J[-1] < 0.5 * J[0]
    assert fwi.rms_error(v, truth) < fwi.rms_error(vp, truth)


def test_illumination_equals_trace_energy_on_an_interior_receiver_row(gfd):
    """With receivers on an interior row, the illumination there is the sum
    over shots and samples n >= 1 of the squared oracle traces."""
    g = _tiny()
    g["rec"] = [[50.0, 10.0 * j] for j in range(3, 28, 3)]
    op = ofd.Problem(g)
    gp = gfd.Problem(g, dt=op.dt, nt=op.nt)
    vp, _ = _models(op.nz, op.nx, op.dz, op.dx)
    vp = vp.astype(np.float32).astype(np.float64)
    to = ofd.forward_shots(op, vp)
    want = np.sum(to[:, 1:, :] ** 2, axis=(0, 1))
    obs = torch.zeros((op.nshots, op.nt, op.nrec), dtype=torch.float32, device="cuda")
    _, _, ill = gfd.gradient(gp, torch.tensor(vp, dtype=torch.float32, device="cuda"), obs, illumination=True)
    got = ill.cpu().numpy()[5, 3:28:3].astype(np.float64)
    assert np.allclose(got, want, rtol=1e-4, atol=0), (got, want)
    assert float(ill.min()) >= 0.0


def test_multiscale_fwi_two_bands(gfd):
    """The band-by-band schedule: a 5 Hz stage then a 10 Hz stage, each with its
    own problem and data; the misfit falls within each band and the model
    error ends below the starting one."""
    from paper_1905_12795_amd import fwi
    stages = []
    for f0 in (5.0, 10.0):
        g = _wide()
        g.update(f0=f0, tmax=0.6)
        gp = gfd.Problem(g)
        _, truth = _models(g["nz"], g["nx"], g["dz"], g["dx"])
        obs = gfd.forward_shots(gp, torch.tensor(truth, dtype=torch.float32, device="cuda"))
        stages.append((gp, obs, 4))
    vp, truth = _models(g["nz"], g["nx"], g["dz"], g["dx"])
    v, hists = fwi.multiscale(stages, vp)
    for h in hists:
        J = [r["misfit"] for r in h]
        _say("band misfits", J)
        assert J[-1] < J[0]
    _say("multiscale rms model error", fwi.rms_error(vp, truth), "->", fwi.rms_error(v, truth))
    assert fwi.rms_error(v, truth) < fwi.rms_error(vp, truth)


def test_illumination_leaves_gradient_and_misfit_unchanged(gfd):
    """The illumination is summed from the recomputed levels by a kernel of
    its own after each segment's adjoint, so asking for it changes neither
    the gradient nor the misfit, bit for bit, with one segment or several;
    the illumination itself does not depend on the checkpoint interval
    (the recomputed levels are the fitness kernel's at any tiling and the
    sum runs over time steps in the same order)."""
    for geom in (_tiny, _wide):
        g = geom()
        gp = gfd.Problem(g)
        vp, truth = _models(g["nz"], g["nx"], g["dz"], g["dx"])
        vpt = torch.tensor(vp, dtype=torch.float32, device="cuda")
        obs = gfd.forward_shots(gp, torch.tensor(truth, dtype=torch.float32, device="cuda"))
        ills = []
        for K in (0, 7, gp.nt):
            m1, g1 = gfd.gradient(gp, vpt, obs, K)
            m2, g2, ill = gfd.gradient(gp, vpt, obs, K, illumination=True)
            assert torch.equal(m1, m2) and torch.equal(g1, g2), (geom.__name__, K)
            assert float(ill.min()) >= 0.0 and float(ill.max()) > 0.0
            ills.append(ill)
        _say(geom.__name__, "illumination range", float(ills[0].min()), float(ills[0].max()))
        assert all(torch.equal(ills[0], x) for x in ills[1:])


def test_gradient_rejects_fields_beyond_its_32_bit_window(gfd):
    """The segment recomputation addresses six consecutive stored fields with
    32-bit byte offsets below 2^31: a grid whose stored field takes 2^31 / 6
    bytes or more (here 10,032 x 10,048 floats, 403 MB, which the fitness
    path still accepts) is refused with ENOTSUP before anything touches the
    device buffers, which are therefore only placeholders."""
    g = copy.deepcopy(config("tiny"))
    g.update(nz=10000, nx=10000, nbl=0, tmax=0.01, ncz=2, ncx=3)
    g["src"] = [[0.0, 500.0]]
    g["rec"] = [[0.0, 10.0 * j] for j in range(0, 101)]
    gp = gfd.Problem(g)
    t = gfd.workspace(1024)
    rc = gfd.lib.empso_gradient(gp.handle, gfd._ptr(t), gfd._ptr(t), gfd._ptr(t), gfd._ptr(t), None, 0,
                                gfd._ptr(t), t.numel(), None)
    assert rc == -6
    assert b"too large for the gradient" in gfd.lib.empso_last_error()


@pytest.mark.parametrize("misfit", ["l2", "trace_normalised"])
@pytest.mark.parametrize("nz,nx,nbl", [(2, 2, 0), (3, 5, 1), (9, 2, 2)])
@pytest.mark.parametrize("nt", [2, 3, 5, 6, 9])
def test_gradient_at_smallest_grids_and_shortest_records(gfd, nz, nx, nbl, nt, misfit):
    """Grids of 2 to 9 points a side and records from the shortest the
    gradient takes (nt = 2: one step) to 9 samples, with random observed
    data: misfit within 2e-4 and gradient within 1e-3 of the oracle's
    discrete adjoint, bit for bit the same at every checkpoint interval."""
    g = copy.deepcopy(config("tiny"))
    g.update(nz=nz, nx=nx, nbl=nbl, f0=25.0, ncz=2, ncx=2, misfit=misfit)
    g["src"] = [[0.0, 0.0], [(nz - 1) * 10.0, (nx - 1) * 10.0]]
    g["rec"] = [[0.0, 10.0 * j] for j in range(nx)]
    g["node_lo"], g["node_hi"] = np.full(4, 1400.0), np.full(4, 2700.0)
    op = ofd.Problem(g, nt=nt)
    gp = gfd.Problem(g, dt=op.dt, nt=nt)
    rng = np.random.default_rng(nz * 100 + nx * 10 + nt)
    vp = ofd.vp_from_nodes(rng.uniform(1500, 2600, 4), 2, 2, nz, nx).astype(np.float32).astype(np.float64)
    scale = np.float32(max(1e-4, np.abs(ofd.forward_shots(op, vp)).max()))
    dobs = rng.standard_normal((2, nt, nx)).astype(np.float32) * scale
    Jo, go = ofd.gradient(op, vp, dobs)
    vpt = torch.tensor(vp, dtype=torch.float32, device="cuda")
    obs = torch.tensor(dobs, device="cuda")
    ref = None
    for K in (0, 1, 2, nt):
        mis, grad = gfd.gradient(gp, vpt, obs, checkpoint_every=K)
        if ref is None:
            ref = (mis.clone(), grad.clone())
            gg = grad.cpu().numpy()
            if np.any(go):
                e = float(np.linalg.norm(gg - go) / np.linalg.norm(go))
                assert e <= REL_G, e
            else:
                # one step under the trace normalisation: every trace holds a
                # single nonzero sample, whose normalised value does not
                # depend on the model, so the exact gradient is zero; the
                # kernels' residue must be negligible against J / v
                e = float(np.linalg.norm(gg))
                assert misfit == "trace_normalised" and nt == 2
                assert e <= 1e-6 * Jo / 1400.0, e
            _say(misfit, nz, nx, nbl, "nt", nt, "gradient error %.3g, misfit %.7g vs %.7g" % (e, float(mis), Jo))
            assert float(mis) == pytest.approx(Jo, rel=REL)
        else:
            assert torch.equal(mis, ref[0]) and torch.equal(grad, ref[1]), K
