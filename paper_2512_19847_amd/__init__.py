"""MI355X (gfx950) implementation of the asymptotic-preserving IMEX Runge-Kutta scheme
for the six-velocity lattice-Boltzmann-type discrete velocity model in the low-Mach
diffusive scaling (arXiv 2512.19847).

  apdvm      ctypes binding of the C ABI (include/apdvm.h) of the HIP library
  build      compiles csrc/*.hip into libapdvm.so for gfx950
  workloads  seeded synthetic inputs (initial fields, tau, time-step rule)
"""
