"""CPU oracle of randomized Block Krylov Iteration -- TEST INFRASTRUCTURE.

Plain, slow, float64 NumPy/LAPACK code written from the paper (Musco & Musco,
Algorithms 1 and 2, Lemma 1, eqs. (1)-(3)).  Only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg may import,
call or execute it.  It shares no code with the GPU library
(``paper_1504_05477_amd``) and never imports it; the only module both sides
use is the input generator package ``workloads``.

Pins (see tests/test_oracle_*.py): Philox known-answer vectors; brute-force
dense SVD on tiny inputs; exact recovery when the Krylov space contains the
column space; rank-k planted inputs at q = 0; agreement of three independent
span routes; Ritz-value interlacing and nestedness in q; Lemma 1; the matrix
Pythagorean identity; planted spectra with known sigma.
"""
from .philox import gaussian, philox4x32_10, philox_words
from .bki import (BKIResult, LinearOperator, RankError, StreamedDense,
                  block_krylov, block_krylov_planted, block_krylov_route_b,
                  rayleigh_ritz, rayleigh_ritz_svd, sign_normalize,
                  simultaneous_iteration, validate)
from .metrics import (frobenius_ratio, per_vector_error, principal_angle,
                      principal_angle_sin, spectral_ratio)

__all__ = [
    "gaussian", "philox4x32_10", "philox_words", "BKIResult", "LinearOperator",
    "RankError", "StreamedDense", "block_krylov", "block_krylov_planted", "block_krylov_route_b", "rayleigh_ritz",
    "rayleigh_ritz_svd", "sign_normalize", "simultaneous_iteration", "validate",
    "frobenius_ratio", "per_vector_error", "principal_angle",
    "principal_angle_sin", "spectral_ratio",
]
