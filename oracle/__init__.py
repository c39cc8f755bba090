"""FP64 CPU oracle for SketchyCGAL on the MaxCut SDP.

TEST INFRASTRUCTURE.  This package is the plain, slow reference that the HIP
library is checked against.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the library never does, and it
shares no code with the library (only the seeded problem generators in
`synth` serve both).

Every function follows the paper (Yurtsever, Tropp, Fercoq, Udell, Cevher,
"Scalable Semidefinite Programming", SIAM J. Math. Data Sci. 2021,
arXiv:1912.02949) step by step, in FP64, with library routines (sparse
matrix-vector product, symmetric tridiagonal eigensolver, Cholesky, SVD)
used only as single steps.

Parity pins (see tests/test_oracle_*.py): Philox against numpy's independent
implementation; Lanczos against dense eigensolvers and Krylov bases built by
QR; the state updates against dense CGAL run on the same eigenvectors (loop
invariants of Section 6.2); reconstruction against the pseudo-inverse
definition and the exact error identity; end-to-end objective against
closed-form MaxCut SDP values and brute force.
"""
from .philox import philox4x64_10, normal_stream, uniform_pair  # noqa: F401
from .sketchycgal import (  # noqa: F401
    OracleParams, OracleResult, lanczos_q, scale_problem, approx_min_evec, approx_min_evec_regenerated,
    tridiag_min_eigpair,
    dual_step_size, NystromSketch, sketchy_cgal, start_vector, gaussian_test_matrix, maxcut_dual_bound,
)
from .rounding import cut_indicators, cut_weight, round_maxcut  # noqa: F401
