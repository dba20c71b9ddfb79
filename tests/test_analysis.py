"""The dispersion/dissipation metric on signals whose answer is known."""
import numpy as np
import pytest

from paper_2401_16322_amd.analysis import dispersion_dissipation


def _ricker(n, dt, f=15.0, t0=0.2):
    t = np.arange(n) * dt
    a = (np.pi * f * (t - t0)) ** 2
    return (1 - 2 * a) * np.exp(-a)


def test_identical_signals_have_no_error():
    r = _ricker(512, 1e-3)
    out = dispersion_dissipation(r, r, 1e-3)
    assert out["dissipation"] <= 1e-15 and out["dispersion"] <= 1e-15


@pytest.mark.parametrize("s", [0.5, 0.9, 1.1, 2.0])
def test_amplitude_scaling_is_pure_dissipation(s):
    """appr = s ref: exp(k) = 1/s at every frequency, l = 0."""
    r = _ricker(512, 1e-3)
    out = dispersion_dissipation(r, s * r, 1e-3)
    assert np.allclose(out["k"], -np.log(s), atol=1e-12)
    assert np.allclose(out["l"], 0.0, atol=1e-12)
    assert out["dissipation"] == pytest.approx(abs(np.log(s)), abs=1e-12)


@pytest.mark.parametrize("delay", [1.5e-3, -2.25e-3])
def test_time_shift_is_linear_phase(delay):
    """appr(t) = ref(t - delay), exact as a spectral shift of the periodic
    signal: F_appr = exp(-i w delay) F_ref, so l(w) = w delay and k = 0."""
    dt, n = 1e-3, 1024
    r = _ricker(n, dt, t0=0.5)
    w = 2 * np.pi * np.fft.rfftfreq(n, dt)
    a = np.fft.irfft(np.fft.rfft(r) * np.exp(-1j * w * delay), n)
    out = dispersion_dissipation(r, a, dt)
    assert np.allclose(out["l"], out["omega"] * delay, atol=1e-9)
    assert np.allclose(out["k"], 0.0, atol=1e-9)


def test_threshold_selects_band_around_the_peak_frequency():
    r = _ricker(1024, 1e-3)
    w = dispersion_dissipation(r, r, 1e-3)["omega"] / (2 * np.pi)
    assert w.min() < 15.0 < w.max() and w.max() < 60.0


def test_length_mismatch_rejected():
    with pytest.raises(ValueError):
        dispersion_dissipation(np.ones(8), np.ones(9))
