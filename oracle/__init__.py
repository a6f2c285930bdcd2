"""CPU oracle for non-Hermitian FEAST (Tang, Kestyn, Polizzi, "A New Highly Parallel
Non-Hermitian Eigensolver").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the GPU
library (no kernels, headers, helpers, tables or constants); the two only share
the seeded input generators in ``pencils``.

Everything here is plain, slow and FP64 complex, written step by step from the
paper:

* ``quadrature``  - contour, quadrature nodes/weights and the rational filter
                    (Section 3, eqn:ellipses, eqn:pi, eqn:quadrature_for_pi).
* ``feast``       - node factorisations, the right/left filters (eqn:Rasp,
                    eqn:Lasp), Algorithms R-FEAST and Bi-FEAST (Section 4),
                    candidate selection and stopping (Section 5 preamble), the
                    FP32-LU + FP64 refinement and FP16 emulation references.
* ``brute``       - the definition: every generalized eigenvalue by QZ, the
                    count inside the contour (Section 2).
* ``mlp``         - a NumPy FP64 reference of the m0 predictor network.

Every function is pinned by ``tests/test_oracle_*.py`` against closed forms,
invariants, brute force or library special cases.
"""
