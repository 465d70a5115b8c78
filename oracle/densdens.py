"""Exact local trace when H_loc is diagonal in the occupation-number basis.

Sec. 3.3.1 notes that with a diagonal one-body term and an Ising-type
(density-density) interaction every sector is one-dimensional.  Then each
occupation state |s> is an eigenstate with energy

    E(s) = sum_f h1_ff n_f + 1/2 sum_{i != j} (U_ijji - U_ijij) n_i n_j ,

every operator maps a state to at most one state with a +-1 factor, and

    w_loc = sum_s  sign(s) * exp( - sum_segments  dt_seg * E(state on segment) ).

States are enumerated as integers (bit f = occupation of flavor f) and the
sign of c_f on |s> is (-1)^(number of occupied flavors below f).  This is an
independent construction from the Kronecker operators used elsewhere in the
oracle; both represent the same fermion algebra, so traces agree.
"""

from __future__ import annotations

import numpy as np


def _energies(imp) -> np.ndarray:
    h1 = np.asarray(imp.h1)
    U = np.asarray(imp.U)
    nf = imp.n_flavors
    if np.max(np.abs(h1 - np.diag(np.diag(h1)))) > 0:
        raise ValueError("h1 is not diagonal")
    V = np.zeros((nf, nf), dtype=U.dtype)
    nz = np.argwhere(np.abs(U) > 1e-14)
    for i, j, k, l in nz:
        if i != j and k == j and l == i:
            V[i, j] += U[i, j, k, l]
        elif i != j and k == i and l == j:
            V[i, j] -= U[i, j, k, l]
        else:
            raise ValueError("U is not of density-density form")
    s = np.arange(1 << nf)
    occ = ((s[:, None] >> np.arange(nf)[None, :]) & 1).astype(np.float64)
    E = occ @ np.real(np.diag(h1)) + 0.5 * np.einsum("si,ij,sj->s", occ, np.real(V), occ)
    return E


def densdens_trace(imp, tau, op, moduli=False):
    """(mantissa, log_scale) of w_loc for a density-density impurity.  With
    moduli=True the signs are dropped: the sum of |terms| (cancellation
    scale)."""
    tau = np.asarray(tau, dtype=np.float64)
    op = np.asarray(op, dtype=np.int64)
    nf = imp.n_flavors
    beta = float(imp.beta)
    E = _energies(imp)
    D = 1 << nf
    state = np.arange(D, dtype=np.int64)
    start = state.copy()
    alive = np.ones(D, dtype=bool)
    sign = np.ones(D)
    logw = np.zeros(D)
    prev = 0.0
    for t, o in zip(tau, op):
        logw -= (t - prev) * E[state]
        f, dag = int(o) // 2, int(o) % 2
        bit = 1 << f
        occ = (state & bit) != 0
        alive &= ~occ if dag else occ
        below = state & (bit - 1)
        parity = _popcount(below) & 1
        sign *= np.where(parity == 1, -1.0, 1.0)
        state = state ^ bit
        prev = float(t)
    logw -= (beta - prev) * E[state]
    alive &= state == start
    if not np.any(alive):
        return 0.0, 0.0
    m = float(np.max(logw[alive]))
    sg = np.abs(sign[alive]) if moduli else sign[alive]
    total = float(np.sum(sg * np.exp(logw[alive] - m)))
    return total, m


def _popcount(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.int64)
    c = np.zeros_like(x)
    while np.any(x):
        c += x & 1
        x = x >> 1
    return c


def densdens_partition_function(imp):
    E = _energies(imp)
    e0 = float(np.min(E))
    return float(np.sum(np.exp(-imp.beta * (E - e0)))), -imp.beta * e0
