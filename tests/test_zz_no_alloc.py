"""The entry point that allocates nothing (empso_traces_misfit_noalloc): its
misfit equals empso_traces_misfit's bit for bit on two calls in a row, the
second over fewer shots, for both misfits; sizes beyond its fixed scratch are
refused on the host."""
import copy
import ctypes

import numpy as np
import pytest
import torch

from workloads.configs import config

pytestmark = pytest.mark.gpu


def _geom(misfit, nshots):
    g = copy.deepcopy(config("tiny"))
    g.update(nz=41, nx=121, nbl=10, tmax=0.2, misfit=misfit)
    g["src"] = [[0.0, 10.0 * (5 + 7 * (s % 15))] for s in range(nshots)]
    g["rec"] = [[0.0, 10.0 * j] for j in range(121)]
    return g


@pytest.mark.parametrize("misfit", ["l2", "trace_normalised"])
def test_noalloc_equals_the_workspace_call_twice(misfit):
    from paper_1905_12795_amd import fd
    prob = fd.Problem(_geom(misfit, 5))
    rng = np.random.default_rng(21)
    shape = (5, prob.nt, prob.nrec)
    tr = torch.tensor(rng.standard_normal(shape).astype(np.float32), device="cuda")
    ob = torch.tensor(rng.standard_normal(shape).astype(np.float32), device="cuda")
    tr[2, :, 7] = 0.0                                   # a silent trace (the floor's case)
    out = torch.full((1,), -1.0, dtype=torch.float32, device="cuda")
    for nsh in (5, 2):                                  # the second call over fewer shots
        ref = fd.traces_misfit(prob, tr[:nsh].contiguous(), ob[:nsh].contiguous())
        got = fd.traces_misfit_noalloc(prob, tr[:nsh].contiguous(), ob[:nsh].contiguous(), out)
        torch.cuda.synchronize()
        print(misfit, nsh, float(got), float(ref), flush=True)
        assert torch.isfinite(ref).all() and float(ref) > 0
        assert torch.equal(got, ref), (nsh, float(got), float(ref))


def test_noalloc_refuses_more_traces_than_its_scratch():
    from paper_1905_12795_amd import _lib, fd
    prob = fd.Problem(_geom("l2", 2200))                # 2200 shots x 121 receivers > 262144
    assert prob.nshots * prob.nrec > 262144
    dummy = torch.zeros(4, dtype=torch.float32, device="cuda")
    out = torch.full((1,), -1.0, dtype=torch.float32, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = ctypes.c_void_p(dummy.data_ptr())
    rc = _lib.lib.empso_traces_misfit_noalloc(prob.handle, p, p, prob.nshots, ctypes.c_void_p(out.data_ptr()), st)
    assert rc == -6
    assert b"scratch" in _lib.lib.empso_last_error()
    torch.cuda.synchronize()
    assert float(out) == -1.0                           # nothing enqueued
