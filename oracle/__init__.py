"""CPU oracle for the categorical STP-DAS sigma build and Davidson solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package; only the test suite, the smoke check and
the CPU-baseline leg of the benchmark use it.  It shares no code with the GPU
library: determinants are explicit occupation bitstrings, matrix elements come
from the textbook Slater-Condon rules, and every sign is obtained by applying
fermion operators to a bitstring.

Modules
  space      explicit enumeration of a windowed determinant space
  csc        the plain-C row-driven Slater-Condon sigma (sc_sigma.c), built
             with gcc on first use
  fock       Jordan-Wigner Fock-space Hamiltonian (the definition of H,
             used to pin the Slater-Condon code on tiny spaces)
  dense      dense projected H for small spaces, exact diagonalisation
  davidson   a plain Davidson iteration with the paper's preconditioners
  bounds     gap-theorem error bound and the rigorous gap lower bound
  spinfree   spatial -> spin-orbital integral expansion

Parity status: every function here is pinned by tests under tests/ against
closed forms, invariants, brute force or library routines (see the test
module docstrings); none is "parity unpinned".
"""
