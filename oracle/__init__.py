"""FP64 CPU oracle for the hybrid LAD-GBR right-hand side (arxiv 2511.18042).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library and does not import it.

The oracle is a plain, slow, vectorised-numpy transcription of what the paper
computes, in float64, step by step in the paper's order:

* ``grid``         -- node layout, ghost layers and boundary images, grid metrics
                      (governing equations, Sec. 2.1)
* ``derivatives``  -- explicit E6 / E4 and compact (tridiagonal) C4 / C6 first
                      derivatives of the primitives (Sec. 2.3, the MEG6 / MIG4
                      gradients; Sec. 4.2 LAD-E4; Sec. 3 LAD-C6)
* ``gbr``          -- characteristic transform, gradient-based linear interface
                      states, centralised interpolation, MP5 limiter, the
                      wave-appropriate selection rule, the Omega sensor and the
                      curvilinear HLLC flux (Sec. 2.3)
* ``lad``          -- localized artificial diffusivity coefficients, truncated
                      Gaussian filter, central convective + viscous fluxes in
                      E4 or compact C6 flux form (Sec. 2.2, Eq. tauij)
* ``implicit_filter`` -- the implicit Pade-type filter of LAD-C6 steps (Sec. 2.1;
                      where Alg. 1 applies it)
* ``rhs``          -- the three RHS forms (C-GBR, LAD, hybrid; Alg. 1-3), the
                      CFL time step and SSP-RK3
* ``riemann``      -- exact Riemann solver for the 1D shock-tube checks (Sec. 3.1)
* ``inflow``       -- digital-filter inflow turbulence of the 3D cases (Sec. 4)

Where the paper is silent the oracle follows the numbered readings R1..R34 that
are listed with the design; each function names the reading it relies on.

Parity pins: every function is pinned by a ``-m "not gpu"`` test against a
closed form, an invariant, brute force or a textbook value (tests/test_oracle_*.py).
"""
from . import grid, derivatives, gbr, lad, implicit_filter, rhs, riemann, inflow  # noqa: F401
