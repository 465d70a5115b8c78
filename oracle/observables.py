"""The impurity density-matrix estimator (Sec. 2.3.2) and the histogram of a
conserved label derived from it (Sec. 4.2, the valence histogram of
delta-Pu) -- TEST INFRASTRUCTURE ONLY, like the rest of oracle/.

density_matrix() returns the whole tau-integrated estimator; the functions
below it take the histogram route described here.

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


def _interval_kernel(a, b, D):
    """int_0^D exp(-t a) exp(-(D - t) b) dt for every pair (a_u, b_v), in closed
    form: (e^{-D b} - e^{-D a}) / (a - b), and D e^{-D a} where a = b."""
    A = a[:, None]
    B = b[None, :]
    diff = A - B
    same = np.abs(diff) <= 1e-12 * np.maximum(1.0, np.maximum(np.abs(A), np.abs(B)))
    safe = np.where(same, 1.0, diff)
    k = (np.exp(-D * B) - np.exp(-D * A)) / safe
    return np.where(same, D * np.exp(-D * 0.5 * (A + B)), k)


def density_matrix(dt, tau, op):
    """(R, w) for one configuration: the tau-integrated estimator of the
    impurity density matrix (Sec. 2.3.2) in the eigenbasis of H_loc,

        R = (beta w)^-1 int_0^beta A(tau) dtau,

    where A(tau) is the time-ordered product cut at tau and closed the other
    way round: with W = P(beta - tau_n) O_n ... O_1 P(tau_1) = W_>(tau) W_<(tau)
    (W_< the part before tau), A(tau) = W_<(tau) W_>(tau), so Tr A(tau) = w for
    every tau and Tr R = 1.  On interval g = [tau_g, tau_{g+1}) (tau_0 = 0,
    tau_{n+1} = beta) A(tau)_uv = e^{-(tau - tau_g) E_u} M_g[u, v]
    e^{-(tau_{g+1} - tau) E_v} with M_g = (O_g P ... O_1 P(tau_1))
    (P(beta - tau_n) O_n ... P O_{g+1}); the tau integral over the interval is
    done in closed form (_interval_kernel).  Energies are taken relative to the
    ground state.  Returns R (2^n x 2^n complex) and w = (mantissa, log_scale);
    R is zero when w is.  Dense full-space matrices with one scale per product:
    for the small impurities of the tests."""
    tau, op = _check_string(tau, op, dt.beta, dt.nf)
    n = tau.size
    D = dt.E.shape[0]
    E = dt.E - dt.E0
    mats = [dt.op_matrix(int(o)) for o in op]
    edges = np.concatenate([[0.0], tau, [dt.beta]])

    def prop(x):
        return np.exp(-x * E)

    # prefix_g = O_g P(tau_g - tau_{g-1}) ... O_1 P(tau_1), with one log scale each
    pre, pre_l = [np.eye(D, dtype=complex)], [0.0]
    for g in range(1, n + 1):
        M = mats[g - 1] @ (prop(edges[g] - edges[g - 1])[:, None] * pre[-1])
        m = np.max(np.abs(M))
        s = m if m > 0 else 1.0
        pre.append(M / s)
        pre_l.append(pre_l[-1] + np.log(s))
    # suffix_g = P(beta - tau_n) O_n ... P(tau_{g+2} - tau_{g+1}) O_{g+1}; suffix_n = 1
    suf, suf_l = [None] * (n + 1), [0.0] * (n + 1)
    suf[n] = np.eye(D, dtype=complex)
    for g in range(n - 1, -1, -1):
        M = (suf[g + 1] * prop(edges[g + 2] - edges[g + 1])[None, :]) @ mats[g]
        m = np.max(np.abs(M))
        s = m if m > 0 else 1.0
        suf[g] = M / s
        suf_l[g] = suf_l[g + 1] + np.log(s)
    W = suf[0] * prop(edges[1])[None, :]
    wm = complex(np.trace(W))
    wl = suf_l[0]
    R = np.zeros((D, D), dtype=complex)
    if wm == 0:
        return R, (0.0, 0.0)
    for g in range(n + 1):
        length = edges[g + 1] - edges[g]
        if length == 0.0:
            continue
        Mg = pre[g] @ suf[g]
        R += _interval_kernel(E, E, length) * Mg * np.exp(pre_l[g] + suf_l[g] - wl)
    R /= dt.beta * wm
    return R, (wm, wl - dt.beta * dt.E0)
