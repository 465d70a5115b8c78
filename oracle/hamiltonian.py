"""Full-space local Hamiltonian (Sec. 2.1, the local-Hamiltonian equation):

    H_loc = sum_ij c+_i h1_ij c_j + 1/2 sum_ijkl c+_i c+_j U_ijkl c_k c_l ,

with h1 = t - mu*1 as provided by the impurity definition.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fock import annihilators


def hamiltonian_sparse(h1: np.ndarray, U: np.ndarray) -> sp.csr_matrix:
    nf = h1.shape[0]
    c = annihilators(nf)
    cd = [x.T.tocsr() for x in c]
    dtype = np.result_type(h1.dtype, U.dtype, np.float64)
    D = 1 << nf
    H = sp.csr_matrix((D, D), dtype=dtype)
    for i in range(nf):
        for j in range(nf):
            if h1[i, j] != 0:
                H = H + h1[i, j] * (cd[i] @ c[j])
    # two-body part, grouped as 1/2 sum_ij (c+_i c+_j) (sum_kl U_ijkl c_k c_l)
    for i in range(nf):
        for j in range(nf):
            block = U[i, j]
            nz = np.nonzero(np.abs(block) > 1e-14)
            if len(nz[0]) == 0:
                continue
            right = sp.csr_matrix((D, D), dtype=dtype)
            for k, l in zip(*nz):
                right = right + block[k, l] * (c[k] @ c[l])
            H = H + 0.5 * ((cd[i] @ cd[j]) @ right)
    H.eliminate_zeros()
    return H.tocsr()


def hamiltonian_dense(h1: np.ndarray, U: np.ndarray) -> np.ndarray:
    return hamiltonian_sparse(h1, U).toarray()
