"""Plain FP64 CPU oracles for hierarchical Tucker low-rank (HTLR) matrices.

TEST INFRASTRUCTURE ONLY.  This package exists to check the GPU library: it
may be imported, called or executed only by ``tests/``, by
``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py``.
The product path (the C-ABI library and its Python binding) never routes
through it, and the two share no code: the only common module is
``htlr_workloads`` (seeded inputs, no method arithmetic).

What each module computes, with the passage of Li & Liu, "Hierarchical Tucker
Low-Rank Matrices: Construction and Matrix-Vector Multiplication"
(arXiv 2508.05958) that it follows:

* ``kernels``   -- kernel functions k(x, y) used in Sec. 5 and by the workloads.
* ``geometry``  -- tensor grids, cells Omega_i, weights |Omega_i| and the
                   diagonal integrals of eq. (1.4) and its quasi-uniform form
                   (Sec. 3.3), by tensor Gauss-Legendre quadrature.
* ``dense``     -- O1: the dense Nystrom product of eq. (1.3) (brute force).
* ``tree``      -- cluster tree (Def. 2.1, Sec. 2.2), strong/weak
                   admissibility (Defs. 2.2-2.3), block cluster tree (Def. 2.4,
                   Def. 3.6).
* ``interp``    -- Chebyshev points and Lagrange basis (Sec. 3.1), Tucker
                   factors and cores (eq. 3.4).
* ``htlr``      -- O2: HTLR construction (Alg. 4.1) and matrix-vector product
                   (Alg. 4.2, eq. 4.3), block by block, no batching.
* ``quasi``     -- O5: the quasi-uniform grid through a uniform one, T Ahat S
                   (Sec. 3.3, eq. 3.9): 1D cell-overlap interpolation
                   matrices and their Kronecker application.
* ``gmres``     -- O3: restarted GMRES and a dense direct solve, used to check
                   the solver (the paper itself has no solver).

Every function is pinned by ``tests/test_oracle_*.py`` against values the
paper fixes (worked example, structure counts, bounds), closed forms,
library routines and brute force.  Parity status of each function is listed in
the module docstrings; none is "parity unpinned".
"""
