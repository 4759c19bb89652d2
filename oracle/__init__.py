"""CPU FP64 oracle for the D3Q27 CHM-MRT lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code, headers, tables or
helpers with the HIP library.

Two independent tiers, both written from the paper's equations:

* ``o1_dense`` (numpy) -- the definition tier: the equilibrium as the Hermite
  series of Eq. (3), the central Hermite transform as a dense 27x27 matrix per
  node, the collision of Eq. (6) solved with a linear solve, then plain
  collide-then-push streaming with the boundary rules.  Slow; small cases only.
* ``o2`` (plain C + OpenMP, ``o2_fast.c``) -- the fast tier used at full
  sizes: factored per-axis transforms, same push streaming.  Checked against
  ``o1_dense`` by brute force on tiny random inputs.
* ``o3_net`` (numpy) -- the learned corrector's network in FP64: 3x3x3
  convolution and its gradients, pooling, upsampling, the trilinear base, the
  masked loss, Adam, and the whole U-net forward and backward (with an
  optional rounding hook at the points where a reduced-precision
  implementation stores values).
"""
