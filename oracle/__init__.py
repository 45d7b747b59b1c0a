"""Plain FP64 CPU oracle for the spaQR least-squares hot path.

TEST INFRASTRUCTURE ONLY.  This package is a slow, obviously-correct
re-statement of the method of Gnanasekaran & Darve, "Hierarchical Orthogonal
Factorization: Sparse Least Squares problems" (arXiv 2102.09878): column
scaling and partitioning (Sections 2.2 and 2.7), block Householder
elimination with row reassignment (Section 2.3), interface scaling
(Section 2.4), two-step sparsification (Section 2.5), merging (Section 2.6),
the level loop of Algorithm 1, and CGLS preconditioned by the resulting
factor (Section 4).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import it.  The GPU library never calls into it and shares no code with
it; the two meet only through the seeded input generator in ``synth``.
"""

