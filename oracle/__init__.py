"""CPU FP64 oracle for the fully implicit Runge-Kutta stage solve.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link or
execute anything in this package; only the tests, the smoke check and the CPU
baseline leg of the benchmark do. It shares no code with the GPU library: the
only common dependency is :mod:`synth`, which draws the seeded inputs.

Modules
  fem       Q1 mass and stiffness matrices on the uniform grid (assembled CSR).
  tableaux  Butcher tableaux by the collocation recipe, printed tableaux,
            stability function.
  step      the exact stage-coupled step: dense brute force, full coupled sparse
            LU, eigen-decoupled sparse LU, closed form for sine modes.
  mg        a plain CSR statement of the geometric multigrid V-cycle and of the
            block Jacobi / block Gauss-Seidel stage preconditioners.
  adjoint   discrete adjoint of the time-step map and the gradient with respect
            to per-element log-diffusivity.
  revolve   the optimal binomial checkpointing cost, by dynamic programming and
            by the closed form.

Every function cites the paper passage (section / equation) it follows. Where the
paper is silent the reading adopted is stated in the docstring.
"""
