"""CPU reference oracle for the probing / multi-shift Krylov log-determinant.

TEST INFRASTRUCTURE ONLY.  Nothing in the library (``paper_1105_5256_amd``)
imports, links or calls this package; only ``tests/``, the ``smoke()`` check
of ``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may use it.
It shares no code, header, table or constant with the HIP path.

Everything here is plain, slow and written to be checked by eye against
Aune & Simpson, "Parameter Estimation in High Dimensional Gaussian
Distributions" (arXiv 1105.5256), in float64 (complex128 for the shifted
systems), with SciPy/NumPy primitives (sparse products, sparse LU, dense
Cholesky/eigh, sine transforms, elliptic functions) as individual steps.

Modules
-------
lattice     Dirichlet lattice Laplacians, M = diag(kappa2) + L, Q = M @ M,
            the bilinear observation matrix A and Q_p = Q_x + tau A^T A
            (Sec. 1, eq. (1) and the posterior precision that follows eq. (3)).
exact       Exact log det Q: closed-form lattice eigenvalues, dense and
            banded Cholesky, sparse LU, dense eigh (Sec. 2, eq. (5)).
colouring   Distance-k colourings and their validator (Sec. 2.1, probing).
shifts      Conformal-map contour quadrature nodes and weights for log
            (Sec. 2.1, eq. (7)).
krylov      Textbook CG and multi-shift CG-M with per-shift vectors
            (Sec. 2.1, last paragraph).
estimator   The probing estimator sum_j v_j^T log(Q) v_j by several routes
            (Sec. 2.1, eqs. (5)-(7)).
gradient    tr(Q^{-1} dQ/deta): closed form, dense, finite differences and
            the probing estimate sum_j x_j^T dQ v_j with x_j = Q^{-1} v_j.

Every function that has an independent pin is checked by the ``-m "not gpu"``
tests under ``tests/test_oracle_*.py``; functions without one say
"parity unpinned" in their docstring.
"""
