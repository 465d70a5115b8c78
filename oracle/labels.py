"""Quantum-number labels and the sector-string walk (Sec. 3.3.1, the sector
map s_alpha(q) and the "zero sector").

Every occupation state carries the label (sum_f q_f n_f for each abelian
charge).  For operator code o and label L, next[L][o] is the label reached by
o from states with label L if the full-space matrix of o has any nonzero
entry leaving a state with label L; otherwise the string dies (the zero
sector).  A start label survives a string iff the walk never dies and returns
to it.
"""

from __future__ import annotations

import numpy as np

from .fock import occupations, operator


def state_labels(imp) -> np.ndarray:
    occ = occupations(imp.n_flavors)          # [D, nf]
    return occ @ np.asarray(imp.qn).T         # [D, n_qn]


def label_table(imp):
    """(labels list of tuples, next dict: (label, code) -> label or None)."""
    lab = state_labels(imp)
    keys = sorted({tuple(int(v) for v in row) for row in lab})
    groups = {k: np.nonzero(np.all(lab == np.array(k)[None, :], axis=1))[0] for k in keys}
    nxt = {}
    for code in range(2 * imp.n_flavors):
        M = operator(imp.n_flavors, code).tocsc()
        for k in keys:
            cols = groups[k]
            sub = M[:, cols]
            rows = sub.nonzero()[0]
            if rows.size == 0:
                nxt[(k, code)] = None
            else:
                targets = {tuple(int(v) for v in lab[r]) for r in rows}
                assert len(targets) == 1, "operator does not map a label to a unique label"
                nxt[(k, code)] = targets.pop()
    return keys, nxt


def label_walk(imp, op, table=None):
    """Sorted list of start labels whose sector string survives op."""
    keys, nxt = table if table is not None else label_table(imp)
    out = []
    for k0 in keys:
        k = k0
        ok = True
        for o in op:
            k = nxt[(k, int(o))]
            if k is None:
                ok = False
                break
        if ok and k == k0:
            out.append(k0)
    return out
