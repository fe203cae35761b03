"""Plain FP64 CPU oracle for the kinetic Monte-Carlo hysteresis-loop method of
Tan, Carrey and Respaud (arXiv:1407.2737), Sec. II.1, Eqs. 1-5.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import this package:
only the test suite, the smoke check and the benchmark's CPU-baseline leg use it.
It shares no code with the GPU library; the only thing the two sides share is the
seeded input generator module, which holds none of the method's arithmetic.

Modules
-------
philox   counter-based Philox-4x64-10 uniforms (published definition), vectorised
sw       Stoner-Wohlfarth stationary points, Eq. 2, by dense scan + bisection
kmc      one synchronous kMC step (steps ii-vii) and whole loop runs (Sec. III.1)
master   deterministic mean-magnetisation loop of non-interacting particles, the
         paper's validation method (Sec. II.3)
swloop   T=0 random-axis Stoner-Wohlfarth loop by 1-D quadrature (closed-form pin)

Parity status: every function here is pinned by a test in tests/test_oracle_*.py
against a closed form, a printed number of the paper, a library routine, an
invariant or brute force, except the interacting-assembly SAR values, for which the
paper prints no number (parity unpinned beyond oracle-versus-GPU agreement).
"""
