"""Jordan-Wigner fermion operators on the full occupation-number space.

Each flavor f is a tensor factor with basis (|0>, |1>).  Flavor 0 is the most
significant factor.  The annihilator is

    c_f = Z (x) ... (x) Z (x) a (x) 1 (x) ... (x) 1,     a = [[0, 1], [0, 0]],
    Z = diag(1, -1) on every factor before f,

which satisfies {c_f, c+_g} = delta_fg and {c_f, c_g} = 0.
"""

from __future__ import annotations

import functools

import numpy as np
import scipy.sparse as sp

_A = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))
_Z = sp.csr_matrix(np.diag([1.0, -1.0]))
_I = sp.identity(2, format="csr")


@functools.lru_cache(maxsize=None)
def annihilators(n_flavors: int) -> tuple:
    """Sparse CSR matrices c_0 .. c_{n-1} (real)."""
    out = []
    for f in range(n_flavors):
        m = sp.identity(1, format="csr")
        for g in range(n_flavors):
            fac = _Z if g < f else (_A if g == f else _I)
            m = sp.kron(m, fac, format="csr")
        out.append(m.tocsr())
    return tuple(out)


def occupations(n_flavors: int) -> np.ndarray:
    """occ[s, f] = occupation of flavor f in basis state s (flavor 0 = most significant)."""
    s = np.arange(1 << n_flavors)
    return ((s[:, None] >> (n_flavors - 1 - np.arange(n_flavors))[None, :]) & 1).astype(np.int64)


def operator(n_flavors: int, code: int):
    """Sparse matrix of operator code = 2*flavor + dagger."""
    c = annihilators(n_flavors)[code // 2]
    return c.T.tocsr() if code % 2 else c
