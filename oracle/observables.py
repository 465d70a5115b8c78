"""Histogram of a conserved label from the reduced-density-matrix estimator
(Sec. 2.3.2, the impurity density-matrix estimator; Sec. 4.2, the valence
histogram of delta-Pu) -- TEST INFRASTRUCTURE ONLY, like the rest of oracle/.

For a configuration C and a projector P_l onto the states whose label (a
function of the occupation state that commutes with H_loc, such as N) equals
l, the per-configuration estimator is

    h_l(C) = beta^-1  int_0^beta  w_loc(C, P_l(tau)) d tau  /  w_loc(C),

where w_loc(C, P_l(tau)) is the local trace with P_l inserted at time tau
among the operators of C.  Because P_l commutes with H_loc, the integrand
is constant on every interval between two consecutive operator times, so the
integral is the sum over the n + 1 intervals [0, tau_1), [tau_1, tau_2),
..., [tau_n, beta) of (interval length) x (trace with P_l inserted there).
Each of those traces is evaluated here as a plain dense full-space chain with
the projector matrix as one more factor, at the interval's start.

The labels sum to the identity, so sum_l h_l(C) = 1 whenever w_loc(C) != 0.
"""

from __future__ import annotations

import numpy as np

from .trace import _chain, _check_string


def label_projectors(dt, state_label, n_labels):
    """Projector of every label in the eigenbasis of dt, (V^H diag(1[label == l]) V).
    Raises if a projector does not commute with H_loc (then the histogram
    estimator above is not defined by interval sums)."""
    state_label = np.asarray(state_label, dtype=np.int64)
    D = dt.E.shape[0]
    if state_label.shape != (D,):
        raise ValueError("one label per occupation state")
    if state_label.min() < 0 or state_label.max() >= n_labels:
        raise ValueError("label out of range")
    out = []
    for l in range(n_labels):
        mask = (state_label == l).astype(np.float64)
        P = dt.V.conj().T @ (mask[:, None] * dt.V)
        # in the eigenbasis H is diag(E): commuting means P_ab (E_a - E_b) = 0
        comm = P * (dt.E[:, None] - dt.E[None, :])
        if np.max(np.abs(comm)) > 1e-9 * max(1.0, float(np.max(np.abs(dt.E)))):
            raise ValueError(f"label {l} does not commute with H_loc")
        P[np.abs(P) < 1e-13] = 0.0
        out.append(P)
    return out


def _inserted(dt, tau, op, pos, t_ins, P):
    """(mantissa, log_scale) of the trace with P inserted after the first
    `pos` operators, at time t_ins."""
    mats = [dt.op_matrix(int(o)) for o in op]
    mats.insert(pos, P)
    times = list(tau)
    times.insert(pos, t_ins)
    return _chain(np.eye(dt.E.shape[0], dtype=dt.dtype), dt.E, mats, np.asarray(times), dt.beta)


def label_histogram(dt, tau, op, projectors):
    """(h, w) for one configuration: h[l] = h_l(C) as defined above (complex
    array), w = (mantissa, log_scale) of w_loc(C).  h is all zeros when
    w_loc(C) = 0."""
    tau, op = _check_string(tau, op, dt.beta, dt.nf)
    n = tau.size
    wm, wl = dt.trace(tau, op)
    h = np.zeros(len(projectors), dtype=np.complex128)
    if wm == 0:
        return h, (wm, wl)
    edges = np.concatenate([[0.0], tau, [dt.beta]])
    for l, P in enumerate(projectors):
        acc = 0.0 + 0.0j
        for g in range(n + 1):
            length = edges[g + 1] - edges[g]
            if length == 0.0:
                continue
            m, ls = _inserted(dt, tau, op, g, edges[g], P)
            if m != 0:
                acc += length * m * np.exp(ls - wl)
        h[l] = acc / (dt.beta * wm)
    return h, (wm, wl)


def label_histogram_abs(dt, tau, op, projectors):
    """Cancellation scale of every h_l: the same interval sums with every
    factor replaced by its elementwise modulus, divided by |w_loc(C)|.  The
    rounding error of any evaluation of h_l scales with this, not with |h_l|."""
    tau, op = _check_string(tau, op, dt.beta, dt.nf)
    n = tau.size
    wm, wl = dt.trace(tau, op)
    out = np.zeros(len(projectors))
    if wm == 0:
        return out
    edges = np.concatenate([[0.0], tau, [dt.beta]])
    D = dt.E.shape[0]
    for l, P in enumerate(projectors):
        acc = 0.0
        for g in range(n + 1):
            length = edges[g + 1] - edges[g]
            if length == 0.0:
                continue
            mats = [np.abs(dt.op_matrix(int(o))) for o in op]
            mats.insert(g, np.abs(P))
            times = list(tau)
            times.insert(g, edges[g])
            m, ls = _chain(np.eye(D), dt.E, mats, np.asarray(times), dt.beta)
            acc += length * abs(m) * np.exp(ls - wl)
        out[l] = acc / (dt.beta * abs(wm))
    return out
