"""Host logic of bench.py: the strip rule it mirrors and when committed
counter summaries apply to a run."""
import math
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


class _Tu:
    def __init__(self, bz, tsteps):
        self.bz, self.tsteps = bz, tsteps


@pytest.mark.parametrize("Nz", [1, 7, 20, 33, 141, 381, 481, 681, 899])
def test_strips_cover_the_grid_with_whole_march_blocks(Nz):
    for bz in (20, 40, 80, 160, 240, 320, 480, 720, 1040, 1280):
        for T in (1, 2, 3, 4):
            h = bench.strip_rows(Nz, bz, T)
            n = math.ceil(Nz / h)
            # every strip holds rows, there are no more strips than ceil(Nz/bz),
            # and a full strip's march (fill + rows) is whole 10-step blocks
            assert h >= 1 and (n - 1) * h < Nz <= n * h
            assert n <= math.ceil(Nz / bz)
            assert (8 * (T - 1) + h) % 10 == 0


def test_realistic_grid_heights():
    # 381 padded rows: tile heights 240 and 320 give the same two strips
    assert bench.strip_rows(381, 240, 4) == bench.strip_rows(381, 320, 4) == 196
    assert bench.strip_rows(381, 160, 4) == 136


def _summary(**kw):
    d = {"kernel_source_sha256_16": bench.kernel_source_hash(), "updates_per_launch": 1000,
         "tuning": {"bz": 320, "tsteps": 4}}
    d.update(kw)
    return d


def test_counters_apply_only_to_the_same_kernel_and_tiles():
    assert bench._counters_apply(_summary(), 1000, _Tu(320, 4), 381)
    assert bench._counters_apply(_summary(), 1000, _Tu(240, 4), 381)          # same strips
    assert not bench._counters_apply(_summary(), 1000, _Tu(160, 4), 381)      # other strips
    assert not bench._counters_apply(_summary(), 1000, _Tu(320, 3), 381)      # other depth
    assert not bench._counters_apply(_summary(), 999, _Tu(320, 4), 381)       # other batch
    assert not bench._counters_apply(_summary(kernel_source_sha256_16="0" * 16), 1000, _Tu(320, 4), 381)



def test_committed_counter_picks_the_entry_of_the_launched_tiles(tmp_path, monkeypatch):
    import json
    e240 = _summary(tuning={"bz": 240, "tsteps": 4}, hbm=1.0)
    e720 = _summary(tuning={"bz": 720, "tsteps": 4}, hbm=2.0)
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "x.json").write_text(json.dumps({"entries": [e240, e720]}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: e240["kernel_source_sha256_16"])
    assert bench.committed_counter("x.json", "hbm", 1000, _Tu(240, 4), 681) == 1.0
    assert bench.committed_counter("x.json", "hbm", 1000, _Tu(720, 4), 681) == 2.0
    assert bench.committed_counter("x.json", "hbm", 1000, _Tu(160, 4), 681) is None
    assert bench.committed_counter("missing.json", "hbm", 1000, _Tu(240, 4), 681) is None


def test_algorithmic_operations_weight_the_layer():
    class _Info:
        nz, nx, Nz, Nx = 601, 1841, 681, 1921
    ops = bench.alg_ops_per_update(_Info)
    share = 1 - 601 * 1841 / (681 * 1921)
    assert abs(ops - (22 * (1 - share) + 28 * share)) < 1e-12 and 22.9 < ops < 23.0
    assert abs(bench.VALU_PEAK_GOPS - 1024 * 16 * 2.4) < 1e-9
