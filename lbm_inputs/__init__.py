"""Seeded synthetic inputs for the regularised lattice Boltzmann step.

This package produces macroscopic fields, noise arrays and plain parameter
sets.  It holds none of the method's arithmetic (no equilibria, no
collision, no relaxation-rate conversion): both the FP64 oracle and the HIP
library compute those themselves from what is generated here.
"""
from .generators import (  # noqa: F401
    shock_tube_1d,
    uniform_rest,
    double_shear_layer,
    spectral_velocity,
    smooth_omega_field,
    fourier_target,
    shear_wave,
    uniform_noise,
)
from .workloads import WORKLOADS, workload  # noqa: F401
