"""What the trained surrogate gains over the method without it (run on an MI355X).

The network acts at one place in the screened search: each particle draws K
candidate moves (independent draws of Eq. 1's random vectors) and the network
picks one. A uniformly random pick among K independent draws has the
distribution of plain EMPSO's single draw, so the network's pick against a
random pick among the same candidates is exactly the network's contribution,
measured without the chaos of whole searches (a last-bit change in one fitness
value changes a whole trajectory, which makes seed-averaged search curves
noisy; the search-level comparison is a study, not a test).

Mini problem (101 x 301 at 10 m, 4 shots, 3 x 6 nodes, 32 particles), 16
seeds: plain EMPSO runs while the network trains online on every evaluated
pair (64 Adam steps per iteration); after iterations 6, 12 and 18 every
particle draws K = 16 candidates and the FD fitness evaluates all of them.
Per seed (averaged over the three states): the Spearman correlation between
the network's prediction and the FD misfit over all 512 candidates, which is
0 in expectation for a random ranking, and the log-misfit gain of the
network's pick over a random pick (the candidates' mean log-misfit minus the
pick's). The test asserts that the 95 % t intervals of both means over the
16 seeds lie above zero (the ranking is better than chance and the moves it
picks are better than plain EMPSO's, with the seed-to-seed spread as the
noise calibration), and that the gain stays below the best candidate's (the
most any ranking can gain). The GPU fitness and the network are
deterministic, so the figures are reproducible for a given build. Parity of
these gains against the paper is unpinned (the surrogate is not in the
paper).
"""
import sys

import pytest
import torch

pytestmark = pytest.mark.gpu

SEEDS = tuple(range(1, 17))
STATES = (6, 12, 18)


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.timeout(900)
def test_network_ranks_candidate_moves_better_than_chance():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_1905_12795_amd import experiments
    rows, summ = experiments.surrogate_ranking("mini", SEEDS, STATES, 16, emit=False)
    for r in rows:
        _say("seed", r["seed"], "rho %.3f" % r["rho"], "log gain %.4f" % r["log_gain"],
             "best-candidate gain %.4f" % r["best_log_gain"], "beats median %.3f" % r["beats_median"])
    _say("summary", summ)
    assert len(rows) == len(SEEDS)
    assert summ["rho"]["ci95"][0] > 0.0, summ["rho"]
    assert summ["log_gain"]["ci95"][0] > 0.0, summ["log_gain"]
    # the network's pick can gain at most what the best candidate gains
    assert summ["log_gain"]["mean"] <= summ["best_log_gain"]["mean"]
