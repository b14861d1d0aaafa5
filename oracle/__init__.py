"""CPU FP64 oracle for the elastic Helmholtz hybrid MG/DD solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
this package: it is used by the tests, by ``__graft_entry__.smoke()`` and by the
``cpu_baseline`` leg of ``bench.py``.  It is written for clarity, not speed:
sparse Kronecker assembly of the staggered operator (paper section 2.1 and
eq. (14)), a direct sparse solve, and the multigrid / domain-decomposition /
FGMRES algorithms step by step in the paper's order (Algorithm 1, Algorithm 2,
section 3, section 4), with scipy/numpy primitives (sparse products, sparse LU,
batched dense solves) as the only building blocks.

It shares no code with the HIP path.  The only common inputs are the seeded
media and sources from ``workloads``.
"""
from . import discretisation, multigrid, dd, krylov, gradient, direct  # noqa: F401
