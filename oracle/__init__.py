"""FP64 CPU oracle of the regularised lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it.  The HIP library never calls it
and shares no code with it.
"""
from .lbm_oracle import *  # noqa: F401,F403
from .lbm_oracle3d import *  # noqa: F401,F403
