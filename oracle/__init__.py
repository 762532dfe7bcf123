"""CPU oracle for the many-body Galerkin solver of active spheres (FP64).

TEST INFRASTRUCTURE ONLY. Nothing on the product path imports, calls or links
anything in this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it. It shares no code, constants or helpers
with the HIP implementation; the two meet only at the seeded input generator.

Contents
--------
basis      orthonormal 5-component basis of symmetric traceless tensors
greens     pair blocks by exact symbolic differentiation of the Stokes
           Green's function under the finite-size operators (section III)
galerkin   dense assembly of the stresslet equations, direct LAPACK solve,
           rigid-body outputs (generalized Stokes laws), superposition
krylov     matrix-free restarted GMRES (modified Gram-Schmidt), FP64
stepper    Adams-Bashforth rigid-body/trap integrator
mlp        reference forward/backward of the warm-start network
"""
