"""FP64 CPU oracle of the ternary electrohydrodynamic lattice-Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it.

It is a plain, slow, whole-array implementation written from the paper's Methods
section (Eqs. 8-21) in plain PyTorch CPU float64 ops, with no blocking, fusion
or closed-form shortcuts: the multiple-relaxation-time collisions are applied
literally in raw-moment space (m* = (I - S) m + S m_eq + (I - S/2) M C, then
f* = M^-1 m*), and the electric potential is obtained by solving the discrete
Gauss law (2D: sparse LU; 3D: Jacobi-preconditioned conjugate gradients to a
relative residual of 1e-15).  Because every operation is a differentiable torch
op (the solve carries its own adjoint), reverse-mode autograd through this
oracle is the FP64 CPU adjoint of the discrete step.

Where the paper is silent, each module states the reading it takes.
"""
from .lattice import Lattice  # noqa: F401
from .geometry import Geometry  # noqa: F401
from .step import Oracle, State  # noqa: F401
