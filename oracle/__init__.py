"""Plain FP64 CPU oracle of the truncated-unity fRG flow right-hand side.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never calls it, and it shares no code,
tables or helpers with that path; both sides receive their inputs from the
seeded generators in ``synth``.

Modules
-------
cutoff      regulator functions J, K = dJ/dLambda and the loop kernels L-/L+
            (Sec. 3.1, the loop definition and the Fermi-function bubbles).
bands       Bloch Hamiltonian, FP64 Hermitian eigendecomposition, projectors.
tufrg       orbital-basis TU-fRG: loop matrices, real-space transforms, the
            cross projections of Sec. 3.3, bundle products, Euler and
            Dormand-Prince integrators, stop test and critical scale.
bruteforce  momentum-space vertex on tiny lattices: the channel projections of
            Sec. 2 as double sums, their converse expansions, and the band-basis
            one-loop right-hand side of Sec. 3.1 (the plain definition that TU
            reproduces exactly with a complete form-factor set).
mlp         the loop surrogate: features of a loop block, a GELU multilayer
            perceptron, its mean-squared loss, gradient and Adam update (no
            counterpart in the paper; pinned by finite differences and closed
            forms).
"""
