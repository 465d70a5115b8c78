"""Block-sparse trace in NumPy on the product's sector tables (tests only).

Evaluates the block form of Sec. 3.3.1 directly, sum over start sectors q0
of Tr[P F ... F P], with no rotation, no panels and no bounds.  It isolates
the host sector builder from the GPU kernels: if this agrees with the oracle
and the GPU does not, the kernels are wrong."""

import math

import numpy as np


def block_trace(tab, tau, op):
    nf = tab.n_flavors
    beta = tab.beta
    E0 = tab.e0()
    total = []
    for q0 in range(tab.n_sectors):
        q = q0
        X = np.eye(tab.dims[q0], dtype=np.complex128 if tab.is_complex else np.float64)
        e2 = 0
        shift = 0.0
        prev = 0.0
        ok = True
        for t, o in zip(tau, op):
            emin = float(np.min(tab.energies[q]))
            X = np.exp(-(t - prev) * (tab.energies[q] - emin))[:, None] * X
            shift += (t - prev) * (emin - E0)
            f, dag = int(o) // 2, int(o) % 2
            nq = tab.next[q, o]
            if nq < 0:
                ok = False
                break
            F = tab.blocks[q][f] if not dag else tab.blocks[nq][f].conj().T
            X = F @ X
            q = nq
            m = np.max(np.abs(X))
            if m == 0:
                ok = False
                break
            e = math.frexp(m)[1]
            X = X * 2.0 ** -e
            e2 += e
            prev = float(t)
        if not ok or q != q0:
            continue
        emin = float(np.min(tab.energies[q]))
        X = np.exp(-(beta - prev) * (tab.energies[q] - emin))[:, None] * X
        shift += (beta - prev) * (emin - E0)
        total.append((np.trace(X), e2 * math.log(2.0) - shift - beta * E0))
    if not total:
        return 0.0, 0.0
    M = max(l for _, l in total)
    return sum(complex(m) * math.exp(l - M) for m, l in total), M
