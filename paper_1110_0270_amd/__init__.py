"""MI355X (gfx950) library for the regularised lattice Boltzmann step of
arXiv:1110.0270: HIP kernels behind a C ABI (include/lbm.h) with a thin
Python binding (paper_1110_0270_amd.lbm)."""
