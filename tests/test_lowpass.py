"""The observed-data low-pass filter (host): pass band, stop band, transition
gain, zero phase and trace independence, checked on wave packets whose
spectra are known in closed form."""
import numpy as np
import pytest

from paper_1905_12795_amd.search import lowpass

DT = 0.8e-3
N = 5000                                     # 4 s at 0.8 ms, as in the paper's record


def _packet(f, n=N, tc=2.0, width=0.3):
    """Gaussian wave packet: spectrum a Gaussian of standard deviation
    1/(2 pi width) Hz around f; negligible (< 1e-9) at the record's ends."""
    t = np.arange(n) * DT
    return np.exp(-0.5 * ((t - tc) / width) ** 2) * np.cos(2 * np.pi * f * (t - tc))


def test_pass_band_packet_is_unchanged():
    x = _packet(2.0)                          # 0.53 Hz wide: 3 Hz from the taper is 5.6 widths
    y = lowpass(x[None, :], DT, 5.0, 6.0)[0]
    assert np.max(np.abs(y - x)) < 1e-6


def test_stop_band_packet_is_removed():
    x = _packet(9.0)
    y = lowpass(x[None, :], DT, 5.0, 6.0)[0]
    assert np.max(np.abs(y)) < 1e-6


def test_transition_midpoint_gain_is_one_half():
    # a long, narrow-band packet at the taper's midpoint: the taper is
    # 1/2 + an odd function of (f - 5.5 Hz), whose output vanishes at the
    # packet's centre, where the envelope is flat
    n = 20000
    x = _packet(5.5, n=n, tc=8.0, width=1.2)
    y = lowpass(x[None, :], DT, 5.0, 6.0)[0]
    c = 10000
    assert y[c] == pytest.approx(0.5 * x[c], abs=1e-3)


def test_zero_phase_keeps_a_symmetric_pulse_symmetric():
    t = np.arange(N) * DT
    x = np.exp(-0.5 * ((t - 2.0) / 0.02) ** 2)     # broadband, symmetric about sample 2500
    y = lowpass(x[None, :], DT, 5.0, 6.0)[0]
    c = 2500
    assert np.argmax(y) == c
    assert np.allclose(y[c - 1000:c], y[c + 1000:c:-1], atol=1e-12)
    assert y.sum() == pytest.approx(x.sum(), rel=1e-3)          # gain 1 at 0 Hz (tails cut at the ends)


def test_shot_time_receiver_arrays_filter_trace_by_trace():
    rng = np.random.default_rng(3)
    d = rng.standard_normal((2, N, 3))
    y = lowpass(d, DT, 5.0, 6.0)
    for s in range(2):
        for r in range(3):
            assert np.allclose(y[s, :, r], lowpass(d[s, :, r][None, :], DT, 5.0, 6.0)[0], atol=1e-12)
    assert np.allclose(lowpass(2 * d, DT, 5.0, 6.0), 2 * y, atol=1e-12)


def test_delay_moves_a_pass_band_packet():
    x = _packet(2.0, tc=1.8)
    y = lowpass(x[None, :], DT, 5.0, 6.0, delay=0.4)[0]
    assert np.max(np.abs(y - _packet(2.0, tc=2.2))) < 1e-6
    with pytest.raises(ValueError):
        lowpass(x[None, :], DT, 5.0, 6.0, delay=-0.1)
