"""Host logic of the surrogate studies (CPU): pretraining pairs saved in parts
are put back in row order and must tile the draw; paired differences get a
t interval."""
import numpy as np
import pytest
from scipy import stats

from paper_1905_12795_amd import experiments


def _part(tmp_path, name, start, X, f):
    p = str(tmp_path / name)
    np.savez(p, X=X, f=f, start=start, stop=start + len(f), total=10)
    return p


def test_pretrain_parts_are_joined_in_row_order(tmp_path):
    X = np.arange(30, dtype=np.float64).reshape(10, 3)
    f = np.arange(10, dtype=np.float64) + 100
    a = _part(tmp_path, "a.npz", 0, X[:4], f[:4])
    b = _part(tmp_path, "b.npz", 4, X[4:], f[4:])
    X2, f2 = experiments.load_pretrain_parts([b, a])          # any order on the command line
    assert np.array_equal(X2, X) and np.array_equal(f2, f)


def test_pretrain_parts_with_a_gap_or_overlap_are_refused(tmp_path):
    X = np.zeros((10, 2))
    f = np.zeros(10)
    a = _part(tmp_path, "a.npz", 0, X[:4], f[:4])
    gap = _part(tmp_path, "gap.npz", 5, X[5:], f[5:])
    over = _part(tmp_path, "over.npz", 3, X[3:], f[3:])
    with pytest.raises(ValueError):
        experiments.load_pretrain_parts([a, gap])
    with pytest.raises(ValueError):
        experiments.load_pretrain_parts([a, over])


def test_paired_interval_is_the_t_interval_of_the_mean():
    d = np.array([3.0, -1.0, 4.0, 1.0, 5.0, 9.0, 2.0, 6.0])
    m, lo, hi = experiments.paired_ci(d)
    h = stats.t.ppf(0.975, d.size - 1) * d.std(ddof=1) / np.sqrt(d.size)
    assert m == pytest.approx(d.mean()) and lo == pytest.approx(m - h) and hi == pytest.approx(m + h)
    m1, lo1, hi1 = experiments.paired_ci([2.0])
    assert m1 == 2.0 and np.isnan(lo1) and np.isnan(hi1)
