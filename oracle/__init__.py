"""CPU oracle for the CT-HYB local trace — TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check of the package entry file and the
benchmark's CPU-baseline leg may import, call or execute anything here.  The
product library never does, and this package never imports the product.

What it computes is the plain definition of the local weight (Sec. 2.2, the
w_loc equation, with the time ordering already applied as in the naive form
of Sec. 3.3.1):

    w_loc(C) = Tr[ P(beta - tau_n) O_n P(tau_n - tau_{n-1}) ... O_1 P(tau_1) ],
    P(x) = exp(-x H_loc),

on the FULL occupation-number space (dimension 2^n_flavors), with no sector
structure at all.  Operators come from Kronecker (Jordan-Wigner) products;
H_loc is assembled from its one- and two-body coefficients (Sec. 2.1).  All
arithmetic is float64 / complex128.

Modules:
  fock       Jordan-Wigner operators as sparse Kronecker products
  hamiltonian full-space H_loc from (h1, U)
  trace      dense full-space trace, eigenbasis route and expm route
  densdens   exact trace for occupation-diagonal H by enumerating states
  labels     quantum-number labels and the label walk of sector strings
"""

from .trace import DenseTrace, expm_trace  # noqa: F401
from .densdens import densdens_trace  # noqa: F401
from .labels import label_walk  # noqa: F401
