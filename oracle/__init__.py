"""CPU oracle for exact PEPS amplitudes of random quantum circuits.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, FP64 reference
that the GPU path is checked against.  Only tests/, the smoke() function of
__graft_entry__ and the cpu_baseline leg of bench.py may import it; the
library (paper_1905_08394_amd) never does, and this package imports nothing
from the library.  The two share no code: the only common dependency is the
seeded input generator `rqcgen`, which emits symbolic gates and bitstrings.

Modules
  gates        gate matrices written out from their definitions
  bruteforce   O1: full 2^N x 2^N operators built from Kronecker products
  statevector  O2: state-vector simulation (the plain definition <tau|G...G|0>)
  peps         O3: PEPS evolution (eqs. 3-6) and exact contraction by the
               generic row scheme (eqs. S2-S6) and the square partition
               (eqs. S9-S10), with loop slicing ("cut") for large lattices
  stats        O4: Porter-Thomas statistics
  complexity   closed forms of eqs. (8)-(10), (S7)-(S12) and exact step counts
"""
