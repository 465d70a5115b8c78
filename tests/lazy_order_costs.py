"""Counts how much chain work the lazy trace could skip if a configuration's
strings were evaluated in descending order of their bounds (Sec. 3.3.1),
against evaluating all of them, on the benchmark's pair-insertion proposals.

    python tests/lazy_order_costs.py [impurity] [config_id] [n]

Each of the first n configurations gets one pair insertion (App. D move,
PCG64(4242), the bench's lazy leg); the threshold is r times the summed
string moduli of the current configuration, r ~ U(0, 1) drawn after the
proposals.  Per string of the proposal: its exact modulus (tests/panelref.py,
a NumPy chain), its bound (width times the exact propagator norms; every
block has norm 1) and its multiply-adds (width times the products along the
rotated string).  Prints the fraction of proposals that are rejectable, that
the plan's summed bound rejects, that the largest-bound string's exact value
plus the other bounds rejects, and the fraction of the work done when
(a) only the largest-bound string goes first and (b) strings go one by one in
descending bound, each stopping once the exact prefix plus the remaining
bounds falls below the threshold."""

from __future__ import annotations

import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import panelref as P  # noqa: E402
from paper_2010_08482_amd.sectors import build_sectors  # noqa: E402
from workloads import make_impurity  # noqa: E402
from workloads.configs import insert_pair, make_configs  # noqa: E402


def strings_with_bounds(tab, s, emin, E0):
    """(|value|, bound, multiply-adds) of every surviving string, with
    energies relative to the ground state."""
    out = []
    for root, path in P.strings(tab, s.tau, s.op):
        steps = P.steps_from(s.tau, s.op, tab.beta, root)
        m, l = P.full_string(tab, s.tau, s.op, root, path)
        w = int(tab.dims[path[0]])
        log_b = math.log(w) - sum(dt * (emin[path[k]] - E0) for k, (_, dt, _) in enumerate(steps))
        macs = w * sum(int(tab.dims[path[k]]) * int(tab.dims[path[k + 1]]) for k in range(len(steps)))
        out.append((abs(m) * math.exp(l) if m != 0 else 0.0, math.exp(log_b), macs))
    return out


def main():
    name = sys.argv[1] if len(sys.argv) > 1 else "dshell"
    cid = int(sys.argv[2]) if len(sys.argv) > 2 else 1
    n = int(sys.argv[3]) if len(sys.argv) > 3 else 400
    imp = make_impurity(name)
    tab = build_sectors(imp)
    E0 = tab.e0()
    emin = [float(np.min(e)) for e in tab.energies]
    rng = np.random.Generator(np.random.PCG64(4242))
    cfgs = make_configs(cid, n)
    props = [insert_pair(rng, s, imp.n_flavors, imp.beta) for s in cfgs]
    r = rng.uniform(0.0, 1.0, size=len(props))
    rejectable = plan = first = 0
    full = work_first = work_desc = 0.0
    for s, p, ri in zip(cfgs, props, r):
        T = ri * sum(v for v, _, _ in strings_with_bounds(tab, s, emin, E0))
        new = sorted(strings_with_bounds(tab, p, emin, E0), key=lambda x: -x[1])
        total = sum(f for _, _, f in new)
        full += total
        bsum = sum(b for _, b, _ in new)
        rejectable += sum(v for v, _, _ in new) < T
        if bsum < T:
            plan += 1
            continue
        if new[0][0] + bsum - new[0][1] < T:
            first += 1
            work_first += new[0][2]
        else:
            work_first += total
        exact, rest = 0.0, bsum
        for v, b, f in new:
            work_desc += f
            exact += v
            rest -= b
            if exact + rest < T:
                break
    print(f"{name}: {n} proposals, rejectable {rejectable / n:.3f}, plan bound rejects {plan / n:.3f}, "
          f"largest-bound string first rejects {(plan + first) / n:.3f}; work done: largest first "
          f"{work_first / full:.3f}, descending bound {work_desc / full:.3f} of evaluating every string")


if __name__ == "__main__":
    main()
