"""Dense full-space local trace (the naive evaluation of Sec. 3.3.1).

    w_loc = Tr[ P(beta - tau_n) O_n P(tau_n - tau_{n-1}) ... O_1 P(tau_1) ],
    P(x) = exp(-x H_loc).

Two independent routes:
  * DenseTrace: diagonalise H_loc once (LAPACK eigh on each connected
    component of its nonzero pattern, assembled into one full-space unitary
    V), carry every operator to the eigenbasis (V^H C V, a full 2^n x 2^n
    matrix), where P(x) is diagonal;
  * expm_trace: stay in the occupation-number basis and form every P(x) with
    scipy's matrix exponential (no eigendecomposition), for tiny spaces.

Magnitudes: every column of the running product X carries its own log scale.
Propagators take out the factor of the column's lowest occupied energy, and
after every operator the column is divided by a power of two (exact).  The
result is returned as (mantissa, log_scale) with w_loc = mantissa *
exp(log_scale).
"""

from __future__ import annotations

import math
import os

import numpy as np
import scipy.linalg
from scipy.sparse.csgraph import connected_components

from .fock import operator
from .hamiltonian import hamiltonian_dense, hamiltonian_sparse

LN2 = math.log(2.0)


def _eigh_keeping_zeros(H):
    """Eigen-decomposition H = V diag(E) V^H of the full-space matrix.

    The eigenvectors are computed separately on every connected component of
    the graph of H's nonzero entries (the smallest subspaces H leaves
    invariant), so V has exact zeros wherever H's powers do.  A single dense
    eigh of the whole matrix may mix degenerate levels that belong to
    different invariant subspaces; the trace is unchanged in exact arithmetic,
    but rounding then couples contributions that differ by many orders of
    magnitude at low temperature and the small ones are lost."""
    D = H.shape[0]
    pattern = (abs(H) > 0).astype(np.int8)
    n_comp, comp = connected_components(pattern, directed=False)
    E = np.zeros(D)
    V = np.zeros((D, D), dtype=H.dtype)
    pos = 0
    for k in range(n_comp):
        idx = np.nonzero(comp == k)[0]
        e, v = scipy.linalg.eigh(H[idx][:, idx].toarray())
        E[pos:pos + idx.size] = e
        V[idx, pos:pos + idx.size] = v
        pos += idx.size
    order = np.argsort(E, kind="stable")
    return E[order], V[:, order]


def _check_string(tau, op, beta, n_flavors):
    tau = np.asarray(tau, dtype=np.float64)
    op = np.asarray(op, dtype=np.int64)
    if tau.shape != op.shape:
        raise ValueError("tau and op differ in length")
    if tau.size and (tau[0] < 0 or tau[-1] >= beta or np.any(np.diff(tau) < 0)):
        raise ValueError("times must be sorted in [0, beta)")
    if op.size and (op.min() < 0 or op.max() >= 2 * n_flavors):
        raise ValueError("operator code out of range")
    return tau, op


def _propagate(X, E, x, logs):
    """X <- exp(-x H) X for H = diag(E), one column at a time.

    Column c is X applied to basis vector c and its nonzero rows lie in one
    invariant subspace.  The factor exp(-x s_c), with s_c the lowest energy
    among the column's nonzero rows, is taken out and added to the column's
    log scale, so the remaining factors exp(-x (E_i - s_c)) are <= 1 with the
    largest equal to 1: no column underflows as a whole, however far above
    the ground state its subspace lies."""
    live = X != 0
    s = np.min(np.where(live, E[:, None], np.inf), axis=0)
    s = np.where(np.isfinite(s), s, 0.0)
    arg = np.where(live, -x * (E[:, None] - s[None, :]), -np.inf)
    return np.exp(arg) * X, logs - x * s


def _rescale(X, logs):
    """Divide every column by a power of two (exact) so that its largest
    modulus lies in [1/2, 1); the factor goes into the column's log scale."""
    m = np.max(np.abs(X), axis=0)
    e = np.where(m > 0, np.frexp(m)[1], 0)
    return X * np.ldexp(1.0, -e)[None, :], logs + e * LN2


def _close(X, logs):
    """Tr of the column-scaled X as (mantissa, log_scale)."""
    d = np.diagonal(X)
    live = d != 0
    if not np.any(live):
        return 0.0, 0.0
    lmax = float(np.max(logs[live]))
    tr = np.sum(d[live] * np.exp(logs[live] - lmax))
    return (complex(tr) if np.iscomplexobj(tr) else float(tr)), lmax


def _chain(X, E, ops, tau, beta):
    """Apply the time-ordered string to X (columns = start basis vectors)."""
    logs = np.zeros(X.shape[1])
    prev = 0.0
    for t, O in zip(tau, ops):
        X, logs = _propagate(X, E, float(t) - prev, logs)
        X = O @ X
        X, logs = _rescale(X, logs)
        prev = float(t)
    X, logs = _propagate(X, E, beta - prev, logs)
    return _close(X, logs)


def _chain_live(D, dtype, E, get_op, tau, beta):
    """trace() and abs_scale() of the same string in one pass, carrying only
    the columns of the running products that are not yet zero.

    Every step acts on each column alone (propagator, operator, rescale), so a
    column that an operator maps to zero stays zero and can be dropped; the
    trace sums the diagonal entries of the columns that are left.  The live
    set follows the modulus chain: |X| <= A entrywise for the running
    products X and A of the two chains, so a zero column of A is a zero
    column of X.  get_op(j) returns operator j of the string as a dense
    matrix."""
    idx = np.arange(D)
    X = np.eye(D, dtype=dtype)
    A = np.eye(D)
    logs = np.zeros(D)
    loga = np.zeros(D)
    prev = 0.0
    for j, t in enumerate(tau):
        X, logs = _propagate(X, E, float(t) - prev, logs)
        A, loga = _propagate(A, E, float(t) - prev, loga)
        O = get_op(j)
        X = O @ X
        A = np.abs(O) @ A
        del O
        keep = np.any(A != 0, axis=0)
        if not np.all(keep):
            idx, X, A, logs, loga = idx[keep], X[:, keep], A[:, keep], logs[keep], loga[keep]
        X, logs = _rescale(X, logs)
        A, loga = _rescale(A, loga)
        prev = float(t)
        if idx.size == 0:
            return (0.0, 0.0), (0.0, 0.0)
    X, logs = _propagate(X, E, beta - prev, logs)
    A, loga = _propagate(A, E, beta - prev, loga)

    def close(M, lg):
        d = M[idx, np.arange(idx.size)]
        live = d != 0
        if not np.any(live):
            return 0.0, 0.0
        lmax = float(np.max(lg[live]))
        tr = np.sum(d[live] * np.exp(lg[live] - lmax))
        return (complex(tr) if np.iscomplexobj(tr) else float(tr)), lmax

    return close(X, logs), close(A, loga)


class DenseTrace:
    """Full-space trace of one impurity in the eigenbasis of H_loc.

    op_store: optional directory.  The annihilator matrices in the eigenbasis
    are then written there as .npy files once and memory-mapped back on use
    instead of being kept in memory (a 2^14-state complex operator takes
    4 GiB); a creator is the conjugate transpose of its annihilator (the
    Jordan-Wigner matrices are real, so c+ = c^T)."""

    def __init__(self, imp, op_store: str | None = None):
        self.imp = imp
        self.op_store = op_store
        self.nf = imp.n_flavors
        self.beta = float(imp.beta)
        H = hamiltonian_sparse(imp.h1, imp.U)
        if abs(H - H.conj().T).max() > 1e-12:
            raise ValueError("H_loc is not Hermitian")
        self.E, self.V = _eigh_keeping_zeros(H)
        self.E0 = float(self.E[0])
        self.dtype = self.V.dtype
        self._ops = {}

    def op_matrix(self, code: int) -> np.ndarray:
        """Operator 'code' in the eigenbasis: <a| O |b> = (V^H O V)_ab."""
        if self.op_store is not None:
            path = os.path.join(self.op_store, f"c{code // 2}.npy")
            if not os.path.exists(path):
                C = operator(self.nf, code - code % 2)
                np.save(path + ".tmp.npy", self.V.conj().T @ (C @ self.V))
                os.replace(path + ".tmp.npy", path)
            M = np.load(path, mmap_mode="r")
            return np.array(M) if code % 2 == 0 else M.conj().T
        if code not in self._ops:
            C = operator(self.nf, code)
            self._ops[code] = self.V.conj().T @ (C @ self.V)
        return self._ops[code]

    def trace(self, tau, op):
        """(mantissa, log_scale) of w_loc for the time-ordered string (tau, op)."""
        tau, op = _check_string(tau, op, self.beta, self.nf)
        D = self.E.shape[0]
        return _chain(np.eye(D, dtype=self.dtype), self.E, [self.op_matrix(int(o)) for o in op], tau, self.beta)

    def abs_scale(self, tau, op):
        """(mantissa, log_scale) of A = the same chain with every operator
        matrix replaced by its elementwise modulus in the eigenbasis: the sum
        of |terms| of the Lehmann expansion of w_loc.  Rounding error of any
        evaluation scales with A, not with |w_loc|; when |w_loc| << A the
        trace is cancellation dominated."""
        tau, op = _check_string(tau, op, self.beta, self.nf)
        D = self.E.shape[0]
        return _chain(np.eye(D), self.E, [np.abs(self.op_matrix(int(o))) for o in op], tau, self.beta)

    def trace_and_scale(self, tau, op):
        """(trace(tau, op), abs_scale(tau, op)) from one pass over the string
        that drops the columns of the running products once they are zero
        (same per-column arithmetic; see _chain_live).  Used for the
        full-size impurities, where a column of the product costs 2^14 rows."""
        tau, op = _check_string(tau, op, self.beta, self.nf)
        D = self.E.shape[0]
        return _chain_live(D, self.dtype, self.E, lambda j: self.op_matrix(int(op[j])), tau, self.beta)

    def partition_function(self):
        """Order zero: Z = Tr exp(-beta H) as (mantissa, log_scale)."""
        return float(np.sum(np.exp(-self.beta * (self.E - self.E0)))), -self.beta * self.E0


def expm_trace(imp, tau, op):
    """Same trace with P(x) = expm(-x (H - s)) in the occupation basis, where s
    is a Gershgorin lower bound of the spectrum (no eigendecomposition)."""
    tau, op = _check_string(tau, op, imp.beta, imp.n_flavors)
    H = hamiltonian_dense(imp.h1, imp.U)
    D = H.shape[0]
    off = np.sum(np.abs(H), axis=1) - np.abs(np.diag(H))
    s = float(np.min(np.real(np.diag(H)) - off))
    Hs = H - s * np.eye(D)
    X = np.eye(D, dtype=H.dtype)
    logs = np.zeros(D)
    prev = 0.0
    for t, o in zip(tau, op):
        X = scipy.linalg.expm(-(t - prev) * Hs) @ X
        X = operator(imp.n_flavors, int(o)) @ X
        prev = float(t)
        X, logs = _rescale(X, logs)
    X = scipy.linalg.expm(-(imp.beta - prev) * Hs) @ X
    m, l = _close(X, logs)
    return m, l - imp.beta * s
