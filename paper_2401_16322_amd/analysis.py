"""Dispersion and dissipation of a recorded signal against a reference
(Sec. 4.1, numerical dispersion and dissipation by Fourier transform).

With F_ref and F_appr the Fourier transforms of the reference and the
approximated receiver signals (same uniform sampling), the method writes
F_ref(w) = exp(k(w) + i l(w)) F_appr(w): k measures the amplitude error
(dissipation) and l the phase error (dispersion). The errors are the means of
|k| and |l| over the frequencies where either spectrum exceeds a fraction
(1 %) of the peak of the reference spectrum.

Host-side analysis of receiver traces (numpy); it computes nothing of the
time integration itself.
"""
from __future__ import annotations

import numpy as np


def dispersion_dissipation(ref, appr, sample_dt=1.0, threshold=0.01):
    """Returns dict(dissipation=mean |k|, dispersion=mean |l|, omega, k, l)
    over the retained frequencies (omega in rad per unit of sample_dt)."""
    ref = np.asarray(ref, dtype=np.float64).ravel()
    appr = np.asarray(appr, dtype=np.float64).ravel()
    if ref.shape != appr.shape or ref.size < 2:
        raise ValueError("signals must have the same length (>= 2)")
    Fr = np.fft.rfft(ref)
    Fa = np.fft.rfft(appr)
    peak = np.max(np.abs(Fr))
    if not peak > 0.0:
        raise ValueError("reference signal is zero")
    keep = (np.abs(Fr) > threshold * peak) | (np.abs(Fa) > threshold * peak)
    keep &= (np.abs(Fa) > 0.0) & (np.abs(Fr) > 0.0)
    ratio = Fr[keep] / Fa[keep]
    k = np.log(np.abs(ratio))
    l = np.angle(ratio)
    omega = 2.0 * np.pi * np.fft.rfftfreq(ref.size, d=sample_dt)[keep]
    return {"dissipation": float(np.mean(np.abs(k))) if k.size else 0.0,
            "dispersion": float(np.mean(np.abs(l))) if l.size else 0.0,
            "omega": omega, "k": k, "l": l}
