"""Resident subproducts for Markov updates, in NumPy on the product's sector
tables (tests and cost counts only; nothing here runs on the device).

Sec. 3.3.1 keeps subproducts of the operator chain between Monte Carlo steps
(a skip list), so that a local update costs a few products instead of the
whole chain.  Two ways of keeping them are written out here, next to the
full re-evaluation the GPU path does for every proposal:

* panels: every surviving sector string, rooted at its narrowest sector
  (width w), keeps its forward products F_m (d_m x w, the steps 1..m applied
  to the identity) and backward products B_m (w x d_m, steps m+1..k), with a
  log scale per column / row.  Tr[B_m F_m] is the string's trace for every m.
  A proposal that leaves the first m1 and the last t steps of the string
  untouched costs only its changed middle: Y = steps m1+1..k'-t applied to
  F_m1, then Tr[B_(k-t) Y].  An accepted proposal rebuilds the panels from
  the changed steps on (one pass over the string).
* tree: a balanced binary tree over the string's steps whose nodes hold the
  full d_out x d_in product of their range (the skip list's subproducts); a
  proposal recomputes the nodes whose range meets the changed steps, and the
  accepted tree is the recomputed one.

A "step" is one interval's propagator followed by the operator that ends it.
Rotated order: a string rooted at interval r (after operator r) runs through
operators r+1, ..., k-1, 0, ..., r, and the propagator of step m is that of
the interval before its operator, so every interval appears exactly once.
The tree cost counts multiply-adds only (complex ones count once).
"""

from __future__ import annotations

import math

import numpy as np


def _op_block(tab, q, o):
    """(next sector, block d(next) x d(q)) of operator code o from sector q,
    or (-1, None) where the string dies."""
    nq = int(tab.next[q, o])
    if nq < 0:
        return -1, None
    f, dag = int(o) // 2, int(o) % 2
    return nq, (tab.blocks[q][f] if not dag else tab.blocks[nq][f].conj().T)


def steps_from(tau, op, beta, root):
    """(op code, preceding interval length, op index) of every step of the
    rotated string rooted at the interval after operator `root`."""
    k = len(op)
    out = []
    for m in range(1, k + 1):
        j = (root + m) % k
        i = (j - 1) % k
        dt = (tau[j] - tau[i]) if j > 0 else (tau[0] + beta - tau[k - 1])
        out.append((int(op[j]), float(dt), j))
    return out


def walk(tab, steps, s0):
    """Sectors after every step from s0 ([s0, s_1, ..., s_k]) if the string
    survives and returns to s0, else None."""
    path = [s0]
    q = s0
    for o, _, _ in steps:
        q = int(tab.next[q, o])
        if q < 0:
            return None
        path.append(q)
    return path if q == s0 else None


def strings(tab, tau, op):
    """Every surviving string of a configuration of order >= 1 as (root
    operator index, sector path from that root), rooted at its narrowest
    interval (the first one on ties)."""
    k = len(op)
    base = steps_from(tau, op, tab.beta, k - 1)  # rooted at the interval through beta / 0
    out = []
    for s0 in range(tab.n_sectors):
        path = walk(tab, base, s0)
        if path is None:
            continue
        dims = [int(tab.dims[q]) for q in path[:-1]]
        m = int(np.argmin(dims))        # interval after step m of the base order = after operator m - 1
        root = (k - 1 + m) % k
        out.append((root, walk(tab, steps_from(tau, op, tab.beta, root), path[m])))
    return out


def _shifted(tab, q):
    return tab.energies[q] - tab.e0()


def _forward(tab, X, lg, q, step):
    """One step applied to the columns of X (sector q): propagator, operator,
    per-column rescale.  Returns (X, lg, next sector)."""
    o, dt, _ = step
    X = np.exp(-dt * _shifted(tab, q))[:, None] * X
    nq, F = _op_block(tab, q, o)
    X = F @ X
    m = np.max(np.abs(X), axis=0)
    s = np.where(m > 0, m, 1.0)
    return X / s[None, :], lg + np.log(s), nq


def _backward(tab, Bm, lg, q_before, step):
    """B_(m-1) = B_m (operator) (propagator) on the rows of B_m, where the
    step starts in sector q_before."""
    o, dt, _ = step
    nq, F = _op_block(tab, q_before, o)
    Bm = (Bm @ F) * np.exp(-dt * _shifted(tab, q_before))[None, :]
    m = np.max(np.abs(Bm), axis=1)
    s = np.where(m > 0, m, 1.0)
    return Bm / s[:, None], lg + np.log(s)


def _trace(B, bl, Y, yl):
    """Tr[B Y] with row logs bl of B and column logs yl of Y, as (mantissa,
    log scale)."""
    d = np.einsum("ij,ji->i", B, Y)   # the diagonal only: w x d multiply-adds
    lg = bl + yl
    live = d != 0
    if not np.any(live):
        return 0.0, 0.0
    M = float(np.max(lg[live]))
    return complex(np.sum(d[live] * np.exp(lg[live] - M))), M


class Resident:
    """Panels of one string: root operator index, steps, sector path, F and
    B with their logs (energies relative to the ground state, as in
    full_string)."""

    def __init__(self, tab, tau, op, root, path):
        self.root = root
        self.steps = steps_from(tau, op, tab.beta, root)
        self.path = path
        k = len(self.steps)
        w = int(tab.dims[path[0]])
        dtype = np.complex128 if tab.is_complex else np.float64
        self.F = [np.eye(w, dtype=dtype)]
        self.Fl = [np.zeros(w)]
        X, lg = self.F[0], self.Fl[0]
        for m in range(k):
            X, lg, _ = _forward(tab, X, lg, path[m], self.steps[m])
            self.F.append(X)
            self.Fl.append(lg)
        self.B = [None] * (k + 1)
        self.Bl = [None] * (k + 1)
        self.B[k] = np.eye(w, dtype=dtype)
        self.Bl[k] = np.zeros(w)
        for m in range(k, 0, -1):
            self.B[m - 1], self.Bl[m - 1] = _backward(tab, self.B[m], self.Bl[m], path[m - 1], self.steps[m - 1])

    def value(self, m=None):
        k = len(self.steps)
        m = k if m is None else m
        return _trace(self.B[m], self.Bl[m], self.F[m], self.Fl[m])


def full_string(tab, tau, op, root, path):
    """The string's trace by one forward pass (what every proposal costs
    without resident products), with energies relative to the ground state
    (a factor e^(beta E0) from the trace)."""
    w = int(tab.dims[path[0]])
    X = np.eye(w, dtype=np.complex128 if tab.is_complex else np.float64)
    lg = np.zeros(w)
    for m, st in enumerate(steps_from(tau, op, tab.beta, root)):
        X, lg, _ = _forward(tab, X, lg, path[m], st)
    return _trace(np.eye(w), np.zeros(w), X, lg)


def common_ends(old_steps, new_steps):
    """(m1, t): the leading and trailing steps two rotated strings share
    (same operator code and preceding interval from the same root)."""
    k, kn = len(old_steps), len(new_steps)
    m1 = 0
    while m1 < min(k, kn) and old_steps[m1][:2] == new_steps[m1][:2]:
        m1 += 1
    t = 0
    while t < min(k, kn) - m1 and old_steps[k - 1 - t][:2] == new_steps[kn - 1 - t][:2]:
        t += 1
    return m1, t


def _macs(tab, w, path, lo, hi):
    return w * sum(int(tab.dims[path[m]]) * int(tab.dims[path[m + 1]]) for m in range(lo, hi))


def plan_proposal(tab, old_tau, old_op, old, new_tau, new_op):
    """Match every surviving string of a proposed configuration with a
    current string (old: list of (root, path)) that shares its root
    operator and start sector: one entry (index into old or None, root,
    path, steps, m1, t, full multiply-adds) per new string.  A match is
    re-rooted at the current string's root (same trace, the current width),
    which may no longer be the narrowest interval of the new string."""
    keyed = {}
    for i, (root, path) in enumerate(old):
        t_r, o_r = old_tau[root], int(old_op[root])
        hit = np.nonzero((new_tau == t_r) & (new_op == o_r))[0]
        if hit.size == 1:
            keyed[(int(hit[0]), path[0])] = i
    out = []
    for root, path in strings(tab, new_tau, new_op):
        steps = steps_from(new_tau, new_op, tab.beta, root)
        full = _macs(tab, int(tab.dims[path[0]]), path, 0, len(steps))
        i = keyed.get((root, path[0]))
        if i is None:
            for (r, s0), cand in keyed.items():
                st = steps_from(new_tau, new_op, tab.beta, r)
                p = walk(tab, st, s0)
                if p is not None and _same_cycle(p, path, steps, st):
                    i, root, path, steps = cand, r, p, st
                    break
        if i is None:
            out.append((None, root, path, steps, 0, 0, full))
            continue
        old_steps = steps_from(old_tau, old_op, tab.beta, old[i][0])
        m1, t = common_ends(old_steps, steps)
        assert old[i][1][len(old_steps) - t] == path[len(steps) - t]
        out.append((i, root, path, steps, m1, t, full))
    return out


def propose(tab, old_tau, old_op, residents, new_tau, new_op):
    """Trace of a proposed configuration from the resident panels of the
    current one: strings matched to a resident (plan_proposal) take their
    changed middle only, all others (root operator removed, strings that did
    not survive before) a full pass.  Returns ((mantissa, log scale),
    multiply-adds spent, multiply-adds of a full re-evaluation)."""
    plan = plan_proposal(tab, old_tau, old_op, [(r.root, r.path) for r in residents], new_tau, new_op)
    vals, spent, full = [], 0, 0
    for i, root, path, steps, m1, t, f in plan:
        full += f
        if i is None:
            vals.append(full_string(tab, new_tau, new_op, root, path))
            spent += f
            continue
        res = residents[i]
        k, kn = len(res.steps), len(steps)
        w = int(tab.dims[path[0]])
        X, lg = res.F[m1], res.Fl[m1]
        for m in range(m1, kn - t):
            X, lg, _ = _forward(tab, X, lg, path[m], steps[m])
        spent += _macs(tab, w, path, m1, kn - t) + w * int(tab.dims[path[kn - t]])
        vals.append(_trace(res.B[k - t], res.Bl[k - t], X, lg))
    if not any(m != 0 for m, _ in vals):
        return (0.0, 0.0), spent, full
    M = max(l for m, l in vals if m != 0)
    # the chains propagate with energies relative to the ground state
    return (sum(m * math.exp(l - M) for m, l in vals if m != 0), M - tab.beta * tab.e0()), spent, full


def proposal_costs(tab, old_tau, old_op, old, new_tau, new_op):
    """Multiply-adds of one proposal by the three routes, with no numerics:
    dict with 'full' (re-evaluation from the narrowest sectors), 'panel'
    (the changed middles, full passes for unmatched strings), 'panel_accept'
    (rebuilding the panels of the new configuration if accepted: one pass
    each way outside the middle already computed, i.e. one full pass), 'tree'
    (the tree nodes that meet the changed steps; a whole tree for unmatched
    strings).  old: the current strings as (root, path)."""
    c = {"full": 0, "panel": 0, "panel_accept": 0, "tree": 0}
    for i, root, path, steps, m1, t, f in plan_proposal(tab, old_tau, old_op, old, new_tau, new_op):
        c["full"] += f
        kn = len(steps)
        w = int(tab.dims[path[0]])
        dims = [int(tab.dims[q]) for q in path]
        if i is None:
            c["panel"] += f
            c["panel_accept"] += f
            c["tree"] += tree_macs(dims, None)
            continue
        c["panel"] += _macs(tab, w, path, m1, kn - t) + w * dims[kn - t]
        c["panel_accept"] += _macs(tab, w, path, 0, kn)
        c["tree"] += tree_macs(dims, (m1, kn - t))
    return c


def _same_cycle(p, path, steps, st):
    """Whether two rooted walks are the same cyclic string (same operator
    index and sector after every operator)."""
    a = {steps[m][2]: path[m + 1] for m in range(len(steps))}
    b = {st[m][2]: p[m + 1] for m in range(len(st))}
    return a == b


def residents_of(tab, tau, op):
    return [Resident(tab, tau, op, root, path) for root, path in strings(tab, tau, op)]


# ---------------------------------------------------------------------------
# cost counts (multiply-adds and stored elements), no numerics
# ---------------------------------------------------------------------------

def string_costs(tab, tau, op):
    """Per surviving string of a configuration: (width, dims along the rotated
    path) -- all the cost counts below need."""
    out = []
    for root, path in strings(tab, tau, op):
        out.append((root, path, steps_from(tau, op, tab.beta, root)))
    return out


def full_macs(tab, tau, op):
    """Multiply-adds of a full re-evaluation (every string from its narrowest
    interval, panel width w)."""
    tot = 0
    for _, path, steps in string_costs(tab, tau, op):
        w = int(tab.dims[path[0]])
        tot += w * sum(int(tab.dims[path[m]]) * int(tab.dims[path[m + 1]]) for m in range(len(steps)))
    return tot


def panel_elements(tab, tau, op):
    """Stored elements of the panels of every string (F and B)."""
    tot = 0
    for _, path, _ in string_costs(tab, tau, op):
        w = int(tab.dims[path[0]])
        tot += 2 * w * sum(int(tab.dims[q]) for q in path)
    return tot


def _tree_nodes(lo, hi, out):
    """Ranges [lo, hi) of a balanced binary tree over steps lo..hi-1 (internal
    nodes with their split point)."""
    if hi - lo <= 1:
        return
    mid = (lo + hi) // 2
    out.append((lo, mid, hi))
    _tree_nodes(lo, mid, out)
    _tree_nodes(mid, hi, out)


def tree_macs(dims_path, changed):
    """Multiply-adds to recompute the tree nodes of one string whose range
    meets the changed steps [a, b) (all nodes when changed is None); dims_path
    holds the sector dimension before every step and after the last.  A node
    over steps [lo, hi) split at mid is d(hi) x d(mid) x d(lo)."""
    k = len(dims_path) - 1
    nodes = []
    _tree_nodes(0, k, nodes)
    tot = 0
    for lo, mid, hi in nodes:
        if changed is not None and (hi <= changed[0] or lo >= changed[1]):
            continue
        tot += dims_path[hi] * dims_path[mid] * dims_path[lo]
    return tot


def tree_elements(dims_path):
    k = len(dims_path) - 1
    nodes = []
    _tree_nodes(0, k, nodes)
    return sum(dims_path[hi] * dims_path[lo] for lo, _, hi in nodes) + sum(
        dims_path[m + 1] * dims_path[m] for m in range(k))
