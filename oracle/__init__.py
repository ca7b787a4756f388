"""CPU oracle for the walk-on-ellipsoids elliptic-measure path (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this package.  It shares
no code with the HIP library: the walk estimator is plain C (wos_oracle.c, FP64), the instance
set-up, element measures, closed forms and the SVD / truncated-SVD / Tikhonov reconstruction are
numpy / scipy.  Parity pins for every function live in tests/test_oracle_*.py.
"""
from . import walks, closed_forms, linalg  # noqa: F401
