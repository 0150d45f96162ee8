"""Plain FP64 CPU oracle of the high-order cell-centred finite-volume JFNK method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the GPU
library (``paper_2601_18417_amd``); its only common dependency is the seeded
input package ``workloads``.

Every step follows the paper's order and notation, in float64 (complex128 for
complex-step Jacobians), with numpy/scipy primitives (einsum, Householder QR,
triangular solves) as steps:

* ``geometry``  - faces, face quadrature, cell volumes/centroids, volume
                  quadrature (Sec. 3.1 "Solution Domain Discretisation").
* ``stencil``   - nearest-neighbour stencils (Sec. 3.5.2 "Interpolation Stencil").
* ``lsq``       - weighted least-squares Taylor reconstruction (Sec. 3.5.1,
                  eqs. te, qAnda, ls, maQw, lsA, weightFunc; App. B scaling).
* ``residual``  - R(u): face-point gradients (eq. faceQuadGrad), constitutive
                  laws (App. A), alpha-stabilisation (eqs. alpha, alphaJump),
                  surface/volume integrals (eqs. divStressDiscret, bodyTerm).
* ``jacobian``  - finite-difference J.v (Sec. 4.1) and brute-force Jacobians.
* ``precond``   - compact approximate Jacobian (Sec. 4.1) and its sweeps.
* ``krylov``    - right-preconditioned flexible GMRES(m).
* ``newton``    - Newton with backtracking line search and load increments.
* ``mpnn``      - the learned preconditioner correction (FP64 reference).
* ``nej``       - the near-exact Jacobian of App. C and its inner GMRES.
* ``dynamics``  - BDF2 time stepping of the momentum equation (App. D).
"""
