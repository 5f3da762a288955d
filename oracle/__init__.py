"""Plain FP64 CPU oracle of the IPM hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it.
See ``ipm_oracle.h`` for what the oracle computes and how it is pinned.
"""
from .oracle import (  # noqa: F401
    Oracle, build, load, num_basis, gauss_legendre, quadrature, multi_indices,
    basis_eval, closure, entropy_grad, entropy, indicator, select_degrees, clenshaw_curtis,
    EQ, ENT, FLUX, BC, QUAD,
    STATUS,
)
