"""CPU FP64 oracle for the fractional-step MRT lattice Boltzmann two-phase method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, constant tables or helpers) and imports nothing
from it.

What it computes: one whole-lattice time step of Zhang, Guo & Li,
"A fractional step lattice Boltzmann model for two phase flows with large
density differences" (arXiv:1812.02459), written as plain whole-array
``torch.float64`` CPU operations in the paper's order and notation:

* ``lattice``     D2Q9 velocities, weights, the MRT matrix (Sec. 3.1,
                  eq:D2Q9, eq:D2Q9MRT) and the selective-filter tables (App. B).
* ``ops``         boundary extension, the isotropic gradient / Laplacian
                  (eq:dicretized), the fourth-order central difference
                  (eq:fourOrder_FDM), the explicit selective filter (eq:filter)
                  and the compact (tridiagonal) selective-filter variant.
* ``step``        equilibria, sources, MRT collision, streaming, the FD
                  correction with TVD-RK3, forces, the implicit velocity, and
                  the composed coupled / CH-only step.
* ``diagnostics`` volume, sums, pressure jump, interface height, bubble
                  centroid.
* ``analytic``    closed-form references used to pin the oracle: the tanh
                  profile, the Laplace law and Prosperetti's capillary wave.

Every elementwise expression is written with a fixed evaluation order and
without fused multiply-add, so that its rounding is fully determined.
Readings of places where the paper is silent or garbled are listed in
``step``'s module docstring; functions with no independent pin say
"parity unpinned" in their docstring.
"""

from . import lattice, ops, step, diagnostics, analytic  # noqa: F401
from .step import Params, State, init_state, set_velocity, step as step_once, run  # noqa: F401
