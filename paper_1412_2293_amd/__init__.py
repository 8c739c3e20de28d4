"""MI355X (gfx950) noisy quantum-circuit simulator: Python binding of libqsim.

The work runs in the HIP kernels of libqsim.so behind the C ABI declared in include/qsim.h;
this package only marshals arguments.  torch provides device memory and streams.
"""
from .qsim import *  # noqa: F401,F403
from .kraus import cp_kraus, cp_kraus_improved  # noqa: F401,E402
