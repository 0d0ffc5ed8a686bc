"""CPU FP64 oracle for the dense Chebyshev Fermi-operator expansion.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The product path (the HIP library and its Python binding) never
imports it, and this package imports nothing from the product path: the two
share only the seeded generators in ``synth``.

What it computes is the plain definition the method reaches exactly (up to
rounding order): the degree-L Chebyshev polynomial of the scaled Hamiltonian,
``D_L = sum_{n<=L} c_n T_n(H~)``, evaluated through the eigen-decomposition
(``Q diag(p_L(lam~)) Q^T``), plus the paper's coefficient-matching algebra
(matrix A, system X, coefficients d) and the chemical-potential bisection on
the trace.  Every function cites the passage it follows.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against values the paper prints, closed forms, exact rational identities or
textbook routines, except the design choices listed as "parity unpinned" in
the module docstrings (the MLP architecture of ``oracle.mlp``).
"""
from . import chebyshev, decomposition  # noqa: F401
