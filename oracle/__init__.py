"""Oracle for the algebraic two-level Schwarz preconditioner (Al Daas, Jolivet, Rees).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 CPU
implementation of what the library computes, written from the paper.  It is
imported only by the tests, by the smoke check and by the CPU-baseline leg of
the benchmark; the library never calls it and shares no code with it.

Two tiers:
  * ``oracle.dense``    literal tier: explicit restriction matrices, dense
                        LAPACK, QZ on the restricted eigenproblem; tiny inputs.
  * ``oracle.schwarz``  scalable tier: sparse matrices, SuperLU, ARPACK; used
                        at full problem sizes and checked against the dense tier.

Readings of the paper where it is silent or ambiguous are listed in the module
docstrings (and in the design notes) and are shared by both tiers.
"""
from . import schwarz, dense  # noqa: F401
