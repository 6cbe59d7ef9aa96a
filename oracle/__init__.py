"""Plain FP64 CPU oracle of the reduced-space Gauss-Newton-Krylov registration method of
Mang & Biros, "Constrained H1-regularization schemes for diffeomorphic image registration"
(SIAM J. Imaging Sci. 9(3), 2016; arXiv 1503.00757).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import or call this package.  It shares no code, tables or helpers with the HIP library in
``paper_1503_00757_amd`` and never imports it; the two meet only in the seeded inputs drawn by
``synthdata``.

Modules
  spectral   pseudospectral Fourier operators (Sec. 4) and the Fourier symbols of the
             regularisation operator A, the projection K and the preconditioner (Sec. 3.3, App. E.2)
  transport  state, adjoint and incremental (Gauss-Newton) transport solves by explicit RK2 (Heun)
             with the body-force time integrals (Sec. 3.1-3.3, Sec. 4)
  reduced    objective, reduced gradient, GN Hessian matvec, preconditioner (Sec. 3.3, Sec. 4)
  solver     PCG (Alg. 2), Armijo backtracking and the outer Newton loop (Alg. 1)
  fno        the learned warm-start network (a Fourier neural operator; not part of the paper):
             forward, hand-written reverse mode, loss and Adam, in FP64 with optional bfloat16
             multiplicands

Every function is pinned by tests under ``tests/`` that check it against closed forms, invariants,
brute force on tiny grids and an independent dense-matrix construction; see the headers of the
individual modules for the readings taken where the paper is silent.
"""
from .spectral import Grid, Params  # noqa: F401
from . import spectral, transport, reduced, solver, fno  # noqa: F401
