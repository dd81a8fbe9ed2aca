"""CPU FP64 oracle for the finite-solid-angle GR radiation step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library; the only common dependency is the seeded input generator
``paper_2302_04283_amd.workloads``, which holds none of the method's
arithmetic.

The oracle follows the paper (White et al. 2023, arXiv 2302.04283) step by
step in plain, vectorised float64 torch/numpy code:

* ``angular_grid``: the geodesic angular grid (Sec. 2.6, the three-step
  icosahedral construction), solid angles, polygon edges; the
  latitude-longitude grid with its PLM stencils (Sec. 2.6, 2.3); the MAPR
  candidate-plane geometry (Sec. 2.6).
* ``geometry``: Christoffel symbols, Ricci rotation coefficients (Sec. 2.2),
  the direction four-vectors n^a, n_a and the tetrad-frame angular velocity
  on the sphere that the angular fluxes use.
* ``step``: one forward step -- ghost fill, reconstruction (Sec. 2.3),
  upwind spatial and angular fluxes (Sec. 2.4), flux divergence, primitives,
  implicit coupling with the quartic (Sec. 2.5), the |n_0| mask (Sec. 2.4),
  four-momentum bookkeeping, outgoing luminosity; plus radiation moments.
* ``quartic``: bisection root of B4 T^4 + B1 T + B0 = 0 (Sec. 2.5).
* ``fluid``: the hand-over of the coupling's four-momentum to a gamma-law
  gas (Sec. 2.5), with rho u^0 held.
* ``gradient``: the reference gradient of the luminosity functional by
  autograd through ``step``.

Parity status of each function is stated in its docstring; functions not
fixed by a pin in ``tests/`` say "parity unpinned".
"""
