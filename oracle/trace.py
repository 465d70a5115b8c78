"""Dense full-space local trace (the naive evaluation of Sec. 3.3.1).

    w_loc = Tr[ P(beta - tau_n) O_n P(tau_n - tau_{n-1}) ... O_1 P(tau_1) ],
    P(x) = exp(-x H_loc).

Two independent routes:
  * DenseTrace: diagonalise H_loc once (LAPACK eigh), carry every operator to
    the eigenbasis (V^H C V), where P(x) is diagonal;
  * expm_trace: stay in the occupation-number basis and form every P(x) with
    scipy's matrix exponential (no eigendecomposition), for tiny spaces.

Magnitudes: after every operator the running product X is divided by a power
of two (2^e, e from frexp of max|X|); the exponents are summed.  The result is
returned as (mantissa, log_scale) with w_loc = mantissa * exp(log_scale).
"""

from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from .fock import operator
from .hamiltonian import hamiltonian_dense

LN2 = math.log(2.0)


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


def _rescale(X):
    m = float(np.max(np.abs(X))) if X.size else 0.0
    if m == 0.0:
        return X, 0, True
    e = math.frexp(m)[1]
    return X * (2.0 ** -e), e, False


class DenseTrace:
    """Full-space trace of one impurity in the eigenbasis of H_loc."""

    def __init__(self, imp):
        self.imp = imp
        self.nf = imp.n_flavors
        self.beta = float(imp.beta)
        H = hamiltonian_dense(imp.h1, imp.U)
        if not np.allclose(H, H.conj().T, atol=1e-12):
            raise ValueError("H_loc is not Hermitian")
        self.E, self.V = scipy.linalg.eigh(H)
        self.E0 = float(self.E[0])
        self.dtype = self.V.dtype
        self._ops = {}

    def op_matrix(self, code: int) -> np.ndarray:
        """Operator 'code' in the eigenbasis: <a| O |b> = (V^H O V)_ab."""
        if code not in self._ops:
            C = operator(self.nf, code)
            self._ops[code] = self.V.conj().T @ (C @ self.V)
        return self._ops[code]

    def propagator(self, x: float) -> np.ndarray:
        """Diagonal of exp(-x (H - E0)) in the eigenbasis."""
        return np.exp(-x * (self.E - self.E0))

    def trace(self, tau, op):
        """(mantissa, log_scale) of w_loc for the time-ordered string (tau, op)."""
        tau, op = _check_string(tau, op, self.beta, self.nf)
        D = self.E.shape[0]
        X = np.eye(D, dtype=self.dtype)
        exp2 = 0
        prev = 0.0
        for t, o in zip(tau, op):
            X = self.propagator(t - prev)[:, None] * X
            X = self.op_matrix(int(o)) @ X
            prev = float(t)
            X, e, zero = _rescale(X)
            if zero:
                return 0.0, 0.0
            exp2 += e
        X = self.propagator(self.beta - prev)[:, None] * X
        return complex(np.trace(X)) if np.iscomplexobj(X) else float(np.trace(X)), \
            exp2 * LN2 - self.beta * self.E0

    def abs_scale(self, tau, op):
        """(mantissa, log_scale) of A = the same chain with every operator
        matrix replaced by its elementwise modulus in the eigenbasis: the sum
        of |terms| of the Lehmann expansion of w_loc.  Rounding error of any
        evaluation scales with A, not with |w_loc|; when |w_loc| << A the
        trace is cancellation dominated."""
        tau, op = _check_string(tau, op, self.beta, self.nf)
        X = np.eye(self.E.shape[0])
        exp2 = 0
        prev = 0.0
        for t, o in zip(tau, op):
            X = self.propagator(t - prev)[:, None] * X
            X = np.abs(self.op_matrix(int(o))) @ X
            prev = float(t)
            X, e, zero = _rescale(X)
            if zero:
                return 0.0, 0.0
            exp2 += e
        X = self.propagator(self.beta - prev)[:, None] * X
        return float(np.trace(X)), exp2 * LN2 - self.beta * self.E0

    def partition_function(self):
        """Order zero: Z = Tr exp(-beta H) as (mantissa, log_scale)."""
        return float(np.sum(self.propagator(self.beta))), -self.beta * self.E0


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
    exp2 = 0
    prev = 0.0
    for t, o in zip(tau, op):
        X = scipy.linalg.expm(-(t - prev) * Hs) @ X
        X = operator(imp.n_flavors, int(o)) @ X
        prev = float(t)
        X, e, zero = _rescale(X)
        if zero:
            return 0.0, 0.0
        exp2 += e
    X = scipy.linalg.expm(-(imp.beta - prev) * Hs) @ X
    tr = np.trace(X)
    return (complex(tr) if np.iscomplexobj(X) else float(tr)), exp2 * LN2 - imp.beta * s
