"""FP64 CPU oracle for the Neural Bootstrapping Method (NBM) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package; only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library: the only common dependency is `nbm_inputs`, which holds seeded input
data and no arithmetic of the method.

Parts (paper, Sec. 3 and Sec. 4.1; the loss equation of Sec. 3 is missing from
the text, so the discretisation is this project's reading, stated in `scheme`):
  geometry  - level sets, projection onto the interface, simplex clipping
  problems  - coefficients, forcing, jump data and exact solutions
  scheme    - cut-cell finite-volume residual at arbitrary cell centres
  grid      - the same scheme assembled on a uniform grid, solved by PCG
  mlp       - FP64 two-network MLP, point evaluation, reverse mode
  nbm       - NBM loss, gradient and Adam (plain definitions)
  philox    - Philox4x32-10 counter-based generator and point sampling

Pins (tests marked "not gpu") tie each part to closed forms, invariants,
finite differences and published test vectors; see tests/test_oracle_*.py.
"""
