"""Plain FP64 CPU oracle for the corrected DGSEM Navier-Stokes hot path.

This package is TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(the HIP library and its Python binding) never imports, calls or links it, and
it shares no code, table or constant generator with that path.

Every routine is written from the paper (arXiv 2207.11571, "Accelerating high
order discontinuous Galerkin solvers using neural networks: 3D compressible
Navier-Stokes equations") and the textbook definitions it cites, in NumPy
float64, vectorised over elements, one axis at a time, with no fusion or
reordering beyond the definitions:

* ``basis``      Gauss-Legendre nodal basis of the DGSEM (Sec. 2.6).
* ``dg``         compressible Navier-Stokes fluxes (App. A), Roe flux and BR1
                 viscous treatment (Sec. 3.1), Smagorinsky closure, the weak-form
                 DG residual p(q) of Eq. (1)/(3), the TGV initial condition
                 Eq. (11), the CFL time step of Eq. (7), diagnostics Eq. (9).
* ``rk``         three-stage third-order low-storage Runge-Kutta (Sec. 2, 3.1).
* ``projection`` the filter G of Sec. 2 (nodal -> modal -> truncate -> nodal).
* ``mlp``        the fully connected forcing network (Sec. 2.2), its MSE
                 training gradient and the Adam update.
* ``forcing``    corrective forcing s = G p_HO(q_HO) - p_LO(G q_HO), Eq. (5),
                 and the corrected right-hand side of Eq. (4).

Functions without an independent pin say "parity unpinned" in their docstring.
"""
