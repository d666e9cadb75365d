"""CPU oracle for the multibody (Axilrod-Teller) potential.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the benchmark's ``cpu_baseline`` leg may import, call or link anything here.
The oracle and the GPU library share no code; the only common dependency is
the seeded input generators in ``workloads``, which hold none of the
method's arithmetic.

Modules:
  * ``direct``     - the exact sum Phi(x) (Section 1), plain C triple loop
                     with compensated sums, plus a tiny-N brute force.
  * ``kdtree``     - BuildKdTree (Algorithm 1).
  * ``multitree``  - the triple-tree traversal with deterministic (Section 4,
                     Section 4.1) and Monte Carlo (Algorithms 3-5) pruning.
  * ``philox``     - the Philox4x32-10 counter-based generator, from its
                     published definition, that the Monte Carlo step draws
                     its random tuples from.
  * ``factorized`` - the law-of-cosines expansion of phi into products of
                     pairwise powers, evaluated with dense FP64 matrices.
"""
