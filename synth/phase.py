"""Seeded synthetic phase retrieval instances (coded diffraction patterns).

The dataset recipe of Section 7.3.3 and Appendix F.1: a signal chi drawn from
the complex standard normal distribution (real and imaginary parts
independent N(0, 1/2), so E|chi_k|^2 = 1), L = 12 modulating waveforms psi_j
whose entries are the product of a uniform draw from {1, i, -1, -i} and an
independent draw from {sqrt(2)/2, sqrt(3)} with probabilities 0.8 and 0.2,
and d = L n phaseless measurements

    b_{j, l} = |a_{j,l}^* chi|^2,   a_{j,l}^* x = (DFT_n (conj(psi_j) * x))_l,

with DFT_n the unnormalised discrete Fourier transform (entry (l, m) equal to
exp(-2 pi i l m / n)), measurement l of waveform j stored at b[j, l].  The
measurements are data acquisition, not part of the solver: they are taken
here with numpy's FFT, while the solver's measurement operator is written
independently in the oracle and in the HIP library (a test checks the
oracle's operator against these measurements).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = ["PhaseInstance", "coded_diffraction", "PHASE_SEEDS"]

# Seeds of the phase retrieval workloads: n = 10^k uses 0x5C6A5000 + k.
PHASE_SEEDS = {k: 0x5C6A5000 + k for k in range(2, 7)}


@dataclasses.dataclass
class PhaseInstance:
    n: int
    L: int
    chi: np.ndarray      # complex128[n]  the signal chi_natural
    psi: np.ndarray      # complex128[L, n]  modulating waveforms
    b: np.ndarray        # float64[L, n]  b[j, l] = |(DFT_n (conj(psi_j) chi))_l|^2

    @property
    def d(self) -> int:
        return self.L * self.n


def coded_diffraction(n: int, seed: int, L: int = 12, masks: str = "cdp") -> PhaseInstance:
    """One instance of the recipe above.  masks = "cdp" draws the waveforms of
    Appendix F.1; masks = "gaussian" draws complex normal waveforms instead
    (a different mask family with the same measurement model, for tests)."""
    rng = np.random.default_rng(seed)
    chi = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2.0)
    if masks == "cdp":
        phase = np.array([1.0, 1.0j, -1.0, -1.0j])[rng.integers(0, 4, size=(L, n))]
        mag = np.where(rng.random((L, n)) < 0.8, math.sqrt(2.0) / 2.0, math.sqrt(3.0))
        psi = phase * mag
    elif masks == "gaussian":
        psi = (rng.standard_normal((L, n)) + 1j * rng.standard_normal((L, n))) / math.sqrt(2.0)
    else:
        raise ValueError(masks)
    b = np.abs(np.fft.fft(np.conj(psi) * chi[None, :], axis=1)) ** 2
    return PhaseInstance(n=n, L=L, chi=chi, psi=psi.astype(np.complex128), b=b)
