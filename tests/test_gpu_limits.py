"""The largest grids the library accepts, against small grids and the oracle (run on an MI355X).

The stencil kernel addresses a run's four stored fields through one buffer
resource with 32-bit byte offsets, so a stored field may take at most 2^29
bytes: 16351 x 8160 points without an absorbing layer (16383 stored rows of
8192 floats, 536,838,144 bytes) is the largest grid of that width. A source
250 points from its bottom and right edges and a record of 60 samples: a
field that starts at the source reaches ceil(di/4) + ceil(dj/4) <= n - 1
points from it by step n, so never 251 points within the record, and the
traces cannot depend on anything beyond that distance. They must equal, bit
for bit, the traces of a 501 x 501 grid with the source at its centre (every
point takes the same arithmetic whatever grid and tile it lies in), which
the oracle computes in FP64 (the oracle's own pin: a grid beyond the
record's reach leaves its traces unchanged). The big grid's rows near the
source lie at byte offsets within 0.03 % of the end of the buffer range, and
its last tiles march past the range (those reads return zero, those stores
are dropped).
"""
import sys

import numpy as np
import pytest
import torch

from oracle import fd as ofd

pytestmark = pytest.mark.gpu

REL = 2e-4
H = 10.0
NT = 60
OFFS = [(-6, dj) for dj in range(-24, 25, 4)]      # receivers 6 rows above the source


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _geom(nz, nx, si, sj):
    return {"nz": nz, "nx": nx, "dz": H, "dx": H, "nbl": 0, "vmax": 2500.0, "f0": 40.0, "damp_R": 1e-3,
            "src": [[si * H, sj * H]], "rec": [[(si + a) * H, (sj + b) * H] for a, b in OFFS],
            "ncz": 2, "ncx": 3, "node_lo": np.full(6, 1400.0), "node_hi": np.full(6, 2500.0)}


def _tuning(gfd, bz, T, graph):
    t = gfd.default_tuning()
    t.bz, t.tsteps, t.use_graph = bz, T, graph
    return t


def test_largest_accepted_grid_equals_a_small_grid_by_causality():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1905_12795_amd import fd as gfd
    dt = 0.4 * ofd.stable_dt(2500.0, H, H)
    small = _geom(501, 501, 250, 250)
    NZ, NX = 16351, 8160
    big = _geom(NZ, NX, NZ - 1 - 250, NX - 1 - 250)
    op = ofd.Problem(small, dt=dt, nt=NT)
    gs = gfd.Problem(small, dt=dt, nt=NT)
    gb = gfd.Problem(big, dt=dt, nt=NT)
    assert (gb.info.Nz, gb.info.Nx, gb.info.row_stride) == (NZ, NX, 8192)
    _say("largest grid: problem", NZ, "x", NX, "created; forward modelling at three tilings")

    to = ofd.forward_shots(op, np.full((501, 501), 2000.0))
    assert np.max(np.abs(to)) > 0
    vs = torch.full((501, 501), 2000.0, device="cuda")
    ts = gfd.forward_shots(gs, vs, tuning=_tuning(gfd, 160, 4, 1))
    e = float(np.linalg.norm(ts.cpu().numpy() - to) / np.linalg.norm(to))
    _say("small grid against the oracle: rel L2", e)
    assert e <= REL
    vb = torch.full((NZ, NX), 2000.0, device="cuda")
    for bz, T, graph in ((160, 4, 1), (20, 1, 0), (1040, 3, 1)):
        tb = gfd.forward_shots(gb, vb, tuning=_tuning(gfd, bz, T, graph))
        torch.cuda.synchronize()
        _say("largest grid, tile height", bz, "depth", T, "bitwise equal:", bool(torch.equal(tb, ts)))
        assert torch.equal(tb, ts), (bz, T)
        del tb
    del vb
    torch.cuda.empty_cache()

    # the fitness path at the same size: nodes -> coefficient field on the
    # device, observed data from a faster medium (the oracle's, FP32)
    dobs = ofd.forward_shots(op, np.full((501, 501), 2100.0)).astype(np.float32)
    X = np.full((1, 6), 2000.0)
    fo, _ = ofd.fitness_batch(op, X, dobs)
    fb = gfd.FitnessBatch([gb], [torch.tensor(dobs, device="cuda")], [0])
    fg = float(fb(X).cpu()[0])
    _say("largest grid fitness", fg, "oracle (small grid)", float(fo[0]))
    assert abs(fg - float(fo[0])) <= REL * float(fo[0])
    del fb
    torch.cuda.empty_cache()


def test_largest_gradient_grid_equals_a_small_grid_by_causality():
    """The gradient's segment recomputation addresses six consecutive stored
    fields through one buffer resource, so its stored field stays below
    2^31 / 6 bytes: 10890 x 8160 points without a layer (10922 stored rows of
    8192 floats, 357,892,096 bytes) is its largest grid of that width. With
    the source 300 points from the bottom and right edges and receivers
    within 6 rows and 8 columns of it, neither the forward field nor the
    adjoint field (which starts at the receivers) reaches 300 points from the
    source in 60 samples, so the misfit and the gradient equal those of a
    601 x 601 grid with the source at its centre bit for bit (the gradient
    zero elsewhere), at two checkpoint intervals; the small grid's gradient
    is held to 1e-3 of the oracle's."""
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1905_12795_amd import fd as gfd
    dt = 0.4 * ofd.stable_dt(2500.0, H, H)
    offs = [(-6, dj) for dj in range(-8, 9, 2)]

    def geom(nz, nx, si, sj):
        g = _geom(nz, nx, si, sj)
        g["rec"] = [[(si + a) * H, (sj + b) * H] for a, b in offs]
        return g

    NZ, NX, M = 10890, 8160, 601
    small = geom(M, M, 300, 300)
    big = geom(NZ, NX, NZ - 1 - 300, NX - 1 - 300)
    op = ofd.Problem(small, dt=dt, nt=NT)
    gs = gfd.Problem(small, dt=dt, nt=NT)
    gb = gfd.Problem(big, dt=dt, nt=NT)
    d = ofd.forward_shots(op, np.full((M, M), 2100.0))
    J, gref = ofd.gradient(op, np.full((M, M), 2000.0), d)
    dt_ = torch.tensor(d.astype(np.float32), device="cuda")
    ms, grs = gfd.gradient(gs, torch.full((M, M), 2000.0, device="cuda"), dt_)
    e = float(np.linalg.norm(grs.cpu().numpy() - gref) / np.linalg.norm(gref))
    _say("gradient, small grid against the oracle: misfit", float(ms), J, "gradient rel L2", e)
    assert abs(float(ms) - J) <= REL * J and e <= 1e-3
    vb = torch.full((NZ, NX), 2000.0, device="cuda")
    for K in (0, 7):
        mb, grb = gfd.gradient(gb, vb, dt_, checkpoint_every=K)
        torch.cuda.synchronize()
        corner = grb[NZ - M:, NX - M:]
        same = bool(torch.equal(mb, ms)) and bool(torch.equal(corner, grs))
        rest = float(grb.abs().sum()) - float(corner.abs().sum())
        _say("largest gradient grid, checkpoint interval", K, "bitwise equal:", same, "outside:", rest)
        assert same and rest == 0.0, K
        del mb, grb, corner
        torch.cuda.empty_cache()
