"""CPU oracle for the nodal DG velocity-stress elastic-wave solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
FP64 (and complex128, for complex-step checks) implementation written from the
mathematics of the method: strong-form nodal DG on affine tetrahedra with
element-constant isotropic material, the exact (upwind) Riemann flux, and the
five-stage fourth-order low-storage Runge-Kutta scheme of Carpenter and
Kennedy.  It shares no code with the GPU library.  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product path
never calls it.

Modules
-------
refelem   exact rational reference operators (Dr, Ds, Dt, mass, LIFT)
setup     connectivity, face node maps, affine geometry, point location
solver    right-hand side, LSERK4, source, receivers, energy, misfit
adjoint   discrete adjoint gradient (reverse mode through the discrete
          forward, with checkpointed recomputation)
pml       convolutional perfectly matched layer (memory variables driven by
          the scheme's directional derivatives)

Every operator and formula here is stated in the docstrings of those modules;
which statement pins which function is recorded in the tests.
"""

from . import refelem, setup, solver, adjoint, pml  # noqa: F401
