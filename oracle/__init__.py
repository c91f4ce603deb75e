"""CPU oracle for the wedge-localised FIO apply -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's cpu_baseline leg may import
or call anything in this package.  The product library (the HIP path under
paper_math_0610051_amd/) never imports it, and it never imports the product
library: the two share no code, tables or helpers.  The only module both
sides use is `fio_inputs`, which holds seeded random inputs and no method
arithmetic.

Contents:
  * direct.c / direct.py -- plain FP64 direct summation of eq. (dfio),
    OpenMP over output points (the definition itself, against which every
    parity test compares);
  * reference.py -- NumPy FP64: phase families, the dense operator matrix
    for tiny N, the wedge partition of Section 1.3, the residual phase,
    the randomized separation of Section 3.2, a step-by-step model of the
    evaluation of Section 3.4 that uses direct nonuniform sums instead of a
    NUFFT, and the error estimators of Section 4;
  * mlp.py -- FP64 NumPy model of the factor network (forward, backward,
    Adam) used to check the GPU training kernels.
"""
