"""FP64 CPU oracle for the volumetric curvilinear lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark do.

The oracle is a plain, slow, vectorised-over-cells NumPy implementation written
from the paper (H. Chen, "Volumetric Lattice Boltzmann Models in General
Curvilinear Coordinates: Theoretical Formulation", arXiv 2401.17183):

* lattice.py      -- discrete velocity sets, weights, T0 (Sec. 2.1, eq. (iso))
* geometry.py     -- D, beta, g_i, J, g^i, g^{ij}, Theta and its contraction A
                     (Sec. 2.1, eqs. (distance)-(gamma))
* equilibrium.py  -- curvilinear equilibrium (Sec. 2.2, eq. (equilibrium))
* collide.py      -- BGK collision, inertial force, delta-N and the implicit
                     fixed point (Sec. 2.2, eqs. (lbe), (collide),
                     (compo-constr), (delta-flux), (deltaN))
* stream.py       -- one-to-one advection (Sec. 2.2, eq. (adv)) with the wall
                     and far-field readings
* sim.py          -- initial state, time step, moments and the output mapping
                     (eq. (result)), audits
* nn.py           -- FP64 reference layers for the convolutional surrogate

Every function states the passage it follows.  Parity status of each part is
listed in the module docstrings ("parity unpinned" where nothing but
self-consistency fixes it).
"""
