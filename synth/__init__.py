"""Seeded synthetic inputs for the NMAGIC made-to-measure (M2M) per-timestep loop.

This package is the only code shared by the HIP path and the CPU oracle.  It holds
no arithmetic of the M2M method itself (no observable kernels, no chi-square, no
entropy, no weight update, no prior): it draws initial particle models and
builds target data sets, the inputs the method consumes (paper section 2: an
N-body system is trained against observables of a target galaxy with errors).

  galaxy   - density / potential closed forms used to *draw* initial conditions
             and analytic targets (Hernquist 1990, logarithmic potential, NFW)
  targets  - target observables Y_j and their errors sigma_j
  configs  - the five workload configurations and their small parity variants
"""
from . import galaxy, targets, configs  # noqa: F401
