"""Plain, slow FP64 reference implementation of the fitness evaluation.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package. The product path
(the HIP library and its Python binding) never imports it, and this package
imports nothing from the product: the two share no code. Both sides take their
seeded inputs from the separate ``workloads`` package.

Modules:
  fd        stencil weights, stability limit, Ricker wavelet, damping profile,
            bilinear two-grid interpolation, forward modelling, misfit, fitness
            (the C time loop in oracle_fd.c does the stepping).
  pso       constriction PSO update and elitist mutation, written from the paper.
  mlp       FP64 multilayer perceptron with hand-written backward pass and Adam
            (the learned surrogate; not part of the paper).
  build     compiles oracle_fd.c with gcc.

Parity status of each function is stated in its docstring ("pinned by" or
"parity unpinned").
"""
