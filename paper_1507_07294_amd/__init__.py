"""MI355X-native time step of the 3D MRT lattice-Boltzmann phase-field model
of Liang, Shi & Chai (arXiv:1507.07294).

The compute path is the HIP library ``libmplb.so`` (C-ABI, ``include/mplb.h``);
``paper_1507_07294_amd.mplb`` is its thin ctypes binding and
``paper_1507_07294_amd.workloads`` builds seeded synthetic inputs.
"""
