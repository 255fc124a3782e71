"""FP64 CPU oracle of the 3D MRT lattice-Boltzmann phase-field step
(Liang, Shi & Chai, arXiv:1507.07294).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product path never imports this
package.  The arithmetic lives in ``orc.c``; this module only marshals
arguments through ctypes.
"""
from .orc import *  # noqa: F401,F403
