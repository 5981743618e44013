"""CPU oracle for the forcing-based free-energy lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 CPU implementation
of what the GPU library computes, written directly from the paper's equations
(Li, Yu & Huang, "Achieving thermodynamic consistency in a class of free-energy
multiphase lattice Boltzmann models", arXiv:2008.01473).  It exists so that the
GPU path can be checked against something that a reader can verify against the
paper by eye.  Only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark may import it; the product path never does, and the oracle imports
nothing from the product package.

Modules
-------
lattice      velocity sets, weights, the D2Q9 transformation matrix (Sec. II A)
eos          van der Waals (Eq. 30) and Carnahan-Starling bulk free energies,
             chemical potential, pressure, critical point, Maxwell construction
operators    the isotropic gradient (Eq. 17) and Laplacian on periodic lattices
model        one time step: macroscopic fields (Eq. 12), chemical potential
             (Eq. 2/30), forces (Eq. 13 and Eq. 24), Guo forcing (Eq. 14),
             equilibria (Eq. 11 and Eq. 27), correction term (Eqs. 28-29),
             moment-space collision (Eqs. 9/28) and streaming (Eq. 10)
discrete_equilibrium
             Newton solve of the lattice equation "mu uniform" that the improved
             scheme's steady state satisfies (Sec. III), used as an independent
             check of the time stepper

Parity status of each function is stated in its docstring; functions whose
results are not fixed by anything outside the oracle say "parity unpinned".
"""

from . import lattice, eos, operators, model, discrete_equilibrium  # noqa: F401
