"""MaxCut rounding of a SketchyCGAL solution (Section 7.2, sec:maxcut-rounding).

TEST INFRASTRUCTURE (see the package docstring).

The solver returns X_hat = U Lambda U^T with U (n x R) orthonormal.  The
entrywise signs of the R columns of U are signed indicators of R cuts; the
cut weights are computed and the heaviest cut is kept.

Reading: sgn(0) is taken as +1, so every vertex is placed on a side.  For
the MaxCut data C = -L/4 of eqn:comb-laplacian, the weight of the cut with
indicator chi in {-1, +1}^n is (1/4) chi^T L chi = -chi^T C chi.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def cut_indicators(U: np.ndarray) -> np.ndarray:
    """sgn(U) entrywise with sgn(0) = +1; int8, same shape as U."""
    U = np.asarray(U, dtype=np.float64)
    return np.where(U < 0.0, -1, 1).astype(np.int8)


def cut_weight(C: sp.spmatrix, chi: np.ndarray) -> float:
    """-chi^T C chi: the weight of the cut chi when C = -L/4."""
    x = np.asarray(chi, dtype=np.float64)
    return float(-(x @ (sp.csr_matrix(C, dtype=np.float64) @ x)))


def round_maxcut(U: np.ndarray, C: sp.spmatrix):
    """All R cut weights, the index of the heaviest (lowest index on ties) and its indicator."""
    chi = cut_indicators(U)
    w = np.array([cut_weight(C, chi[:, j]) for j in range(chi.shape[1])])
    best = int(np.argmax(w))
    return w, best, chi[:, best].copy()
