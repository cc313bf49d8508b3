"""FP64 CPU oracle for the sine-transform-preconditioned MINRES method of
Hon, Fung, Dong and Serra-Capizzano (arXiv 2201.10062).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the tests, the smoke check of the
entry module and the ``cpu_baseline`` leg of the benchmark may import it.  It
shares no code with the GPU path (it imports nothing from the product package
and the product package imports nothing from it).  It is plain NumPy/SciPy in
float64: sparse matrices assembled explicitly, dense matrices for the pins, and
``scipy.fft.dst``/``dstn`` or the dense sine matrix for every sine transform.

Modules:
  spatial    -- finite-difference stiffness matrix K(a), averaged Toeplitz Kbar,
                Laplacian eigenvalues (Sec. 3.1.1, eqn:matrix_Km_va)
  sine       -- the orthonormal DST-I matrix S_n and P_n (eqn:matrix_tri_p)
  allatonce  -- the all-at-once matrices T_H (eq. theta) and BDF2 That
                (eqn:matrix_gen), the flip Y (eqn:main_system), right-hand
                sides and sequential time stepping (Sec. 1)
  precond    -- P_H (def:matrix_P), Phat (def:matrix_P_gen), P_theta
                (def:matrix_mod_P) exact and with a fixed-degree Chebyshev
                inner solve
  minres     -- preconditioned MINRES (Paige-Saunders), true-residual stop
  adjoint    -- adjoint solve and gradients w.r.t. f, u0 and face/nodal a

Parity status: every function here is pinned by a test in tests/ against
closed forms, the paper's printed numbers, brute-force dense algebra or an
independent library routine, except the mixed-precision comparison, which is
"parity unpinned" by design (rounding differs; only the error is reported).
"""
from . import spatial, sine, allatonce, precond, minres, adjoint, system  # noqa: F401
