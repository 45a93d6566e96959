"""Plain FP64 CPU oracle for the asymptotic-preserving IMEX Runge-Kutta scheme of
Dimarco, Klar, Koefler, Pareschi (arXiv 2512.19847) applied to the six-velocity
lattice-Boltzmann-type discrete velocity model in the low-Mach diffusive scaling.

TEST INFRASTRUCTURE ONLY.  This package is the independent reference that the HIP
path is checked against.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product path never does.  It shares no code
with the HIP library: it is written directly from the paper, in NumPy, in float64,
with no blocking, fusion or reordering beyond what the definitions state.

Modules
  d2q6      velocity set, moment basis, equilibrium, BGK collision, the scaling map
            between populations and the six scaled moments, and the scaled moment
            system right-hand side (Section 2.1).
  operators spatial operators: WENO5 (Jiang-Shu) with Lax-Friedrichs splitting,
            fourth-order central differences, and the operator bundles used by the
            scheme (Section 3.2 and its high-order extension).
  tableau   IMEX Runge-Kutta double Butcher tableaux and their structural checks
            (Section 3.1 definitions; Section 4.1 tableaux).
  helmholtz exact periodic Helmholtz solve by 2D DFT diagonalisation (Algorithm 1,
            step 2).
  scheme    the fully discrete stage loop (Algorithm 1; fully discrete scheme of
            Section 3.2).

Parity status per function is stated in each module header.
"""

from . import d2q6, operators, tableau, helmholtz, scheme  # noqa: F401
