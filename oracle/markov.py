"""The Markov step around the local trace (Sec. 2.3.1 sampling, App. C
Metropolis-Hastings, App. D Pauli-aware pair moves, Sec. 2.2 hybridisation
weight) -- TEST INFRASTRUCTURE ONLY, like the rest of oracle/.

Everything here is the plain definition, evaluated from scratch at every
step: the hybridisation weight is a determinant computed by LAPACK on the
whole matrix, the local weight is the dense full-space trace.

Bath.  Flavor f couples to discrete levels eps_fk with amplitudes V_fk, so
that for 0 < tau < beta

    Delta_f(tau) = - sum_k V_fk^2 exp(-tau eps_fk) / (1 + exp(-beta eps_fk)),

extended antiperiodically, Delta_f(tau - beta) = -Delta_f(tau).  With the
hybridisation diagonal in flavor, w_hyb = prod_f det M_f, M_f[r][s] =
Delta_f(tc_r - ta_s) over the creator times tc and annihilator times ta of
flavor f (Sec. 2.2, the w_hyb equation).

Moves (App. D; the reading of the proposal weights is derived here from
detailed balance for the draws below).  Random numbers u[0..5] in [0, 1)
are inputs:
  u0 < 1/2: insert a pair, else remove one;  u1: flavor f = floor(u1 n_f);
  L = the operators of flavor f in time order, N = |L|.
  Insert, N = 0: creator at u2 beta, annihilator at u3 beta;
      proposal ratio q = beta^2.
  Insert, N > 0: o = L[floor(u2 N)], d = distance from o to the next operator
      of flavor f (on the circle of circumference beta); times o + u3 d and
      o + u5 d (wrapped below beta); the earlier one gets the type that
      keeps the flavor alternating (an annihilator after a creator);
      q = N d^2 / (2 (N + 2)).
  Remove: o = L[floor(u2 N)] and the next operator of flavor f are removed;
      q = 1 / beta^2 if N = 2, else 2 N / ((N - 2) d^2) with d the distance
      from the operator before o to the operator after the removed pair.
  Accept iff q |w_hyb'/w_hyb| |w_loc'| >= u4 |w_loc| (the uniform drawn
  first; the sampled weight is |w_loc w_hyb|).
A proposal that would put two operators at the same time is no proposal.
"""

from __future__ import annotations

import math

import numpy as np

from .hamiltonian import hamiltonian_dense


def bath_delta(beta, eps, v, tau):
    """Delta(tau) of one flavor for tau in (-beta, beta), tau != 0."""
    eps = np.asarray(eps, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    sign = 1.0
    if tau < 0:
        tau += beta
        sign = -1.0
    total = 0.0
    for e, a in zip(eps, v):
        # the same fraction written so that no exponent is positive
        term = math.exp(-tau * e) / (1.0 + math.exp(-beta * e)) if e >= 0 else \
            math.exp((beta - tau) * e) / (math.exp(beta * e) + 1.0)
        total += a * a * term
    return -sign * total


def hyb_matrices(beta, baths, tau, op, n_flavors):
    """M_f for every flavor, rows = creators, columns = annihilators, both in time order."""
    out = []
    for f in range(n_flavors):
        tc = [t for t, o in zip(tau, op) if o // 2 == f and o % 2 == 1]
        ta = [t for t, o in zip(tau, op) if o // 2 == f and o % 2 == 0]
        if len(tc) != len(ta):
            raise ValueError("unbalanced flavor")
        eps, v = baths[f]
        M = np.array([[bath_delta(beta, eps, v, a - b) for b in ta] for a in tc]).reshape(len(tc), len(ta))
        out.append(M)
    return out


def log_abs_hyb(beta, baths, tau, op, n_flavors):
    """log |w_hyb| (-inf if a determinant vanishes)."""
    total = 0.0
    for M in hyb_matrices(beta, baths, tau, op, n_flavors):
        if M.size == 0:
            continue
        d = abs(np.linalg.det(M))
        if d == 0:
            return -math.inf
        total += math.log(d)
    return total


def propose(tau, op, u, n_flavors, beta):
    """(new_tau, new_op, q) for the move drawn by u, or None (no proposal)."""
    tau = list(tau)
    op = list(op)
    f = min(n_flavors - 1, int(u[1] * n_flavors))
    L = [i for i, o in enumerate(op) if o // 2 == f]
    N = len(L)
    if u[0] < 0.5:
        if N == 0:
            tc, ta = u[2] * beta, u[3] * beta
            new = [(tc, 2 * f + 1), (ta, 2 * f)]
            q = beta * beta
        else:
            k = min(N - 1, int(u[2] * N))
            o, nx = L[k], L[(k + 1) % N]
            d = tau[nx] - tau[o]
            if d <= 0:
                d += beta
            x1, x2 = u[3] * d, u[5] * d
            if x1 == x2:
                return None
            lo, hi = min(x1, x2), max(x1, x2)
            t_lo, t_hi = tau[o] + lo, tau[o] + hi
            if t_lo >= beta:
                t_lo -= beta
            if t_hi >= beta:
                t_hi -= beta
            first_is_creator = op[o] % 2 == 0   # after an annihilator the flavor is empty
            new = [(t_lo, 2 * f + (1 if first_is_creator else 0)), (t_hi, 2 * f + (0 if first_is_creator else 1))]
            q = N * d * d / (2.0 * (N + 2))
        times = set(tau)
        if new[0][0] == new[1][0] or new[0][0] in times or new[1][0] in times:
            return None
        items = sorted(list(zip(tau, op)) + new, key=lambda x: x[0])
        return [t for t, _ in items], [o for _, o in items], q
    if N == 0:
        return None
    k = min(N - 1, int(u[2] * N))
    o, nx = L[k], L[(k + 1) % N]
    if N == 2:
        q = 1.0 / (beta * beta)
    else:
        prev, after = L[(k - 1) % N], L[(k + 2) % N]
        d = tau[after] - tau[prev]
        if d <= 0:
            d += beta
        q = 2.0 * N / ((N - 2) * d * d)
    keep = [i for i in range(len(op)) if i != o and i != nx]
    return [tau[i] for i in keep], [op[i] for i in keep], q


class OracleChain:
    """One Markov chain over configurations (tau, op), weights from scratch."""

    def __init__(self, dense_trace, baths, tau=(), op=()):
        self.dt = dense_trace
        self.baths = baths
        self.nf = dense_trace.nf
        self.beta = dense_trace.beta
        self.tau = list(tau)
        self.op = list(op)
        self.la_loc = self._la_loc(self.tau, self.op)
        self.la_hyb = log_abs_hyb(self.beta, baths, self.tau, self.op, self.nf)

    def _la_loc(self, tau, op):
        m, l = self.dt.trace(np.asarray(tau, dtype=np.float64), np.asarray(op, dtype=np.int64))
        return math.log(abs(m)) + l if m != 0 else -math.inf

    def step(self, u):
        """Returns (decision, margin): decision 1 accepted, 0 rejected, -1 no
        proposal; margin = log of (accept ratio / u4), the distance of the
        decision from its threshold (inf when there was no proposal)."""
        p = propose(self.tau, self.op, u, self.nf, self.beta)
        if p is None:
            return -1, math.inf
        nt, no, q = p
        la_hyb = log_abs_hyb(self.beta, self.baths, nt, no, self.nf)
        if la_hyb == -math.inf:
            return 0, math.inf
        la_loc = self._la_loc(nt, no)
        if la_loc == -math.inf:
            return 0, math.inf
        log_r = math.log(u[4]) if u[4] > 0 else -math.inf
        margin = math.log(q) + (la_hyb - self.la_hyb) + la_loc - (log_r + self.la_loc)
        if margin >= 0:
            self.tau, self.op, self.la_loc, self.la_hyb = nt, no, la_loc, la_hyb
            return 1, margin
        return 0, margin


def anderson_occupation(imp, baths):
    """Exact <sum_f n_f> of the impurity coupled to its discrete bath: the
    impurity orbitals plus one orbital per bath level, H_imp + sum eps b+b +
    V (c+ b + b+ c), thermal average by dense diagonalisation."""
    nf = imp.n_flavors
    levels = [(f, e, v) for f in range(nf) for e, v in zip(*baths[f])]
    n = nf + len(levels)
    h1 = np.zeros((n, n), dtype=np.result_type(imp.h1, np.float64))
    h1[:nf, :nf] = imp.h1
    for j, (f, e, v) in enumerate(levels):
        h1[nf + j, nf + j] = e
        h1[f, nf + j] = h1[nf + j, f] = v
    U = np.zeros((n,) * 4, dtype=np.result_type(imp.U, np.float64))
    U[:nf, :nf, :nf, :nf] = imp.U
    H = hamiltonian_dense(h1, U)
    E, V = np.linalg.eigh(H)
    w = np.exp(-imp.beta * (E - E[0]))
    s = np.arange(1 << n)
    # flavor 0 is the most significant bit of the occupation-basis index
    n_imp = sum(((s >> (n - 1 - f)) & 1) for f in range(nf)).astype(np.float64)
    occ = np.einsum("i,ik,k->", n_imp, np.abs(V) ** 2, w)
    return float(occ / np.sum(w))
