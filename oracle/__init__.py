"""CPU FP64 oracle for periodic piezoelectric homogenisation.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import or run it; the
product path never does.  It shares no code with the GPU library (numpy and
scipy only) and imports nothing from it.

It follows Wegert, Roberts & Challis, "Level set-based inverse
homogenisation of three-dimensional piezoelectric materials":

* fe.py        material matrix, units, trilinear hex8 element, density map
* cell.py      periodic assembly, pinned direct solve, effective tensors,
               energy form, per-element sensitivities
* foms.py      figures of merit and their gradients (complex step)
* hj.py        one first-order upwind Hamilton-Jacobi step
* laminate.py  closed-form laminate tensors (a pin, not the method)
* krylov.py    textbook right-preconditioned GMRES with the block
               lower-triangular Schur preconditioner of Sec. 2.5.3
* tricg.py     TriCG for the quasi-definite block system (Sec. 2.5.2)
* optim.py     the optimisation step: reinitialisation, Hilbertian
               extension and projection, stopping rule (Sec. 2.6)
* fullsize.py  the operator, residual and tensors element by element, for
               checks at sizes the direct solve cannot reach

Where the paper is silent the readings are stated in the docstrings:
standard Galerkin weak form with E = -grad(phi); scales C0 = 1e9 Pa,
e0 = 1 C/m^2; ersatz factor s = eps_v + (1 - eps_v) rho on all three tensors;
density from a sinusoidal smoothed Heaviside of the element-mean level set.
"""
from . import fe, cell, foms, hj, laminate, krylov  # noqa: F401
from .cell import homogenise  # noqa: F401
