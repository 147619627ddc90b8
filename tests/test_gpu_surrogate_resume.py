"""A surrogate-screened search checkpointed mid-run (swarm and surrogate:
weights, Adam moments and step, dataset, standardisation, generator states)
and resumed in fresh objects continues bit for bit (run on an MI355X)."""
import numpy as np
import pytest
import torch

from workloads.configs import config, true_model

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(300)
def test_screened_search_resumes_bitwise(tmp_path):
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1905_12795_amd import fd, search
    from paper_1905_12795_amd.pso import load_checkpoint, save_checkpoint
    from paper_1905_12795_amd.surrogate import ScreenedEMPSO, Surrogate, load_surrogate, save_surrogate
    g = config("mini")
    lo, hi = g["node_lo"], g["node_hi"]
    prob = fd.Problem(g)
    dobs = search.observed_data(prob, true_model(g))
    N, M = 16, 8

    def make():
        sur = Surrogate(lo, hi, seed=3, steps_per_update=8)
        return sur, ScreenedEMPSO(lo, hi, N, sur, K=4, warmup=1, evaluate=M, gen=10, seed=3)

    fb = fd.FitnessBatch([prob], [dobs], [0] * M)
    sur, sw = make()
    for _ in range(3):
        sw.tell(fb(sw.ask()).cpu().numpy())
    save_checkpoint(str(tmp_path / "swarm.npz"), sw)
    save_surrogate(str(tmp_path / "sur.npz"), sur)
    ha = [sw.tell(fb(sw.ask()).cpu().numpy()) for _ in range(3)]
    sur2, sw2 = make()
    load_checkpoint(str(tmp_path / "swarm.npz"), sw2)
    load_surrogate(str(tmp_path / "sur.npz"), sur2)
    hb = [sw2.tell(fb(sw2.ask()).cpu().numpy()) for _ in range(3)]
    print(ha, hb, flush=True)
    assert ha == hb
    assert np.array_equal(sw.x, sw2.x) and np.array_equal(sw.sel, sw2.sel)
    assert torch.equal(sur.net.params, sur2.net.params) and torch.equal(sur.net.m, sur2.net.m)
    assert sur.count == sur2.count and sur.net.step == sur2.net.step
