"""Oracle for algorithmic Matsubara integration (AMI): TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU implementation of what the device path
computes, written from the paper (Burke & LeBlanc, "TorchAmi", arXiv
2311.17189).  Only the test suite, the smoke check of the package entry file
and the CPU-baseline leg of the benchmark may import or call anything here;
the product path never does.  It shares no code with the HIP library.

* :mod:`oracle.construct` -- repeated residue theorem (Sec. 2.2, Eqs. (1)-(4)),
  canonical term list, factorized Fermi tree (Sec. 2.1, Fig. 1).
* :mod:`oracle.evaluate`  -- evaluation of the term list over energy and
  frequency batches (Sec. 2.2 Eq. (6), Sec. 2.3), energies from momenta
  (Sec. 5.2),
  analytic gradients.
* :mod:`oracle.brute`     -- the plain definition Eq. (1): truncated Matsubara
  sums with analytic tails, used to pin the two modules above.

Parity status: every function is pinned by tests under ``tests/`` against
closed forms, brute-force sums, exact integer examples printed in the paper or
invariants, except the shape of the factorized tree (the paper does not fix
which terms are grouped); only its expansion and its values are pinned.
"""
