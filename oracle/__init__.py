"""Plain FP64 CPU oracle for the HGKS time stage of Pan & Xu,
"High-order gas-kinetic scheme with three-dimensional WENO reconstruction for
the Euler and Navier-Stokes solutions" (arXiv:1909.01580).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the HIP library; the two meet
only through arrays produced by the seeded input generators.

The oracle follows the paper step by step, in NumPy FP64, vectorised over
cells and face Gauss points:

* ``geometry``  trilinear cells, 2x2x2 Gauss moments, bilinear faces
                (Sec. 2 last part; Sec. 3, Eqs. (10)-(11)).
* ``weno``      WENO-AO reconstruction: big stencil, 24 sub-stencils,
                least squares, smoothness indicators, nonlinear weights,
                positivity fallback (Sec. 2, Eqs. (1)-(5); Sec. 4 limiter).
* ``gks``       BGK gas-kinetic flux at one Gauss point, generic moment
                algebra and 5x5 solves (Sec. 3, Eqs. (7)-(8), (13)-(16)).
* ``characteristic``  reconstruction in characteristic variables: Euler
                eigenvectors along the face normal, projected polynomials,
                indicators and weights per characteristic field (Sec. 4).
* ``scheme``    finite-volume operator, two-stage fourth-order stepping,
                moving-mesh update, time step, step rejection and totals
                (Sec. 3, Eq. (9) and Remark 2).

Every function is pinned by CPU tests against what the paper or the
mathematics fixes (closed forms, invariants, brute-force quadrature, the
printed tables).  Parity unpinned -- readings that no printed value fixes, so
the oracle and the GPU agree on them by construction only:

* the epsilon of the nonlinear weights (Eq. (3)), default 1e-8;
* the time-step rule (only the CFL number is printed);
* the mechanism that sets the Prandtl number: the BGK flux as written has
  Pr = 1 and the paper states Pr = 0.71 without saying how; the oracle's
  heat-flux correction (the one of the gas-kinetic literature) is pinned by
  its Navier-Stokes limit (Fourier flux with kappa = c_p mu / Pr), not by a
  printed value;
* the moving-mesh conservation mechanism (Remark 2) as such, though its
  consequences (free stream to round-off, volume equal to the geometric
  volume) are pinned;
* the smooth-flow collision time tau_eps * dt of the inviscid tau (Sec. 4),
  whose printed value 0.01 matches only the coarsest row of Table 1;
* the step-rejection rule ``checked_step`` (halve dt while the step gives a
  non-physical state): a control rule the paper does not state, needed for
  the singular start of its Sedov problem.  Pinned only to its own
  definition (minimal halving, result equal to a plain step);
* the state and frame of the characteristic projection (Sec. 4 names the
  characteristic variables only as an option, without the state): the
  eigenvectors at the mean of the two cell averages sharing the face, along
  the face frame of Sec. 3 at the face centre.  Pinned through their
  consequences (eigen-decomposition of the Jacobian, linear weights giving
  the component-wise scheme, the entropy wave), not by a printed value.

Array convention inside the oracle: spatial axes are ordered (i, j, k) =
(x, y, z).  The public helpers in ``scheme`` accept and return states in the
library layout ``[5][nz][ny][nx]`` and transpose at the edge.
"""

from .scheme import (  # noqa: F401
    Params, Problem, uniform_problem, vertex_problem, residual, step,
    s2o4, max_dt, totals, gp_states, face_fluxes, physical, checked_step, kinetic_energy,
)
