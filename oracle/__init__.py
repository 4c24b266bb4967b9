"""FP64 CPU oracle for the two-scale micro batch (TEST INFRASTRUCTURE).

Plain, slow and meant to be checked by eye against the paper.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
this package; the GPU library never calls it and shares no code with it.

Modules
-------
deformation  the pullback quantities F, J, K, C and the boundary weight
             (Section 3.1, equations for K and J and the change of variables)
fem          Q1 reference element, Gauss rules, micro and macro assembly
             (Section 3.1, discrete weak form on the reference cell)
twoscale     the coupled implicit-Euler step: exact Schur route, the paper's
             fixed-point coupling (Section 3.3) and a dense monolithic solve
adjoint      discrete adjoint of the time-stepped system (no counterpart in
             the paper; the derivation is written out in the module)
stationary   the paper's stationary three-field system (Section 2.1) with
             Robin exchange on parts of each cell boundary, solved as one
             sparse system
"""
