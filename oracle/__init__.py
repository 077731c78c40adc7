"""Plain FP64 CPU oracle of DuQuad's inexact (augmented) dual first-order method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything under this package: only the test suite, the
smoke check and the benchmark's CPU-baseline leg use it.  It shares no
code with the HIP library (kernels, headers, helpers, constant
generators); both sides only share the seeded input generators.

Modules
-------
dfom      Algorithm DFOM (Sec. 3) with the inner Algorithm FOM (Sec. 2.1),
          primal last / averaged iterates (Sec. 4) and the runtime
          certificate used as outer test.
exact     Exact references used to pin the oracle: brute-force active-set
          enumeration (n <= 8) and exact box-QP inner solutions.
ipm       A textbook primal-dual interior-point QP solver, used only to
          cross-check optimal values at moderate n.

Parity status
-------------
The exact iterate sequence of DFOM has no printed reference anywhere in
the paper (all result figures are elided), so the iterate log itself is
"parity unpinned"; everything it is built from is pinned by the tests in
tests/test_oracle_*.py (exact optima, KKT, weak duality, dual ascent,
theta invariants, the feasibility identities of Sec. 4.2, rate bounds).
"""
from .dfom import (DGM, DFGM, LAST, AVG, CERT, FIXED, INNER_AUTO, INNER_GM,
                   INNER_FGM, INNER_FGM_SIGMA, Options, Result, Constants,
                   problem_constants, objective, lagrangian, dual_gradient,
                   inner_gradient, inner_certificate, fom_inner, dfom_solve)

__all__ = [
    "DGM", "DFGM", "LAST", "AVG", "CERT", "FIXED", "INNER_AUTO", "INNER_GM",
    "INNER_FGM", "INNER_FGM_SIGMA", "Options", "Result", "Constants",
    "problem_constants", "objective", "lagrangian", "dual_gradient",
    "inner_gradient", "inner_certificate", "fom_inner", "dfom_solve",
]
