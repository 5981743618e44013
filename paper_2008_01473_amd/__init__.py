"""MI355X (gfx950) implementation of the forcing-based free-energy multiphase
lattice Boltzmann step of Li, Yu & Huang (arXiv:2008.01473): standard and
improved schemes on D2Q9 / D3Q19, float64 or float32-deviation storage, batched
lattices, behind the C ABI of include/lbm.h.

`runtime` loads the HIP library (liblbm.so) on first use of a handle and raises
if it has not been built; `inputs` holds the seeded synthetic initial conditions.
"""
