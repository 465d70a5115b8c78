"""Counts, over Markov proposals on the benchmark workloads, the multiply-adds
and resident memory of three ways to evaluate a proposal: full re-evaluation
(what the GPU path does), resident panels and a subproduct tree (panelref).

    python tests/panel_reuse_costs.py [n_configs] [proposals_per_config]

Each chain starts from one of the workload's first n_configs configurations
and makes proposals_per_config pair insertions or removals (App. D moves,
half each), accepting each with the probability given per workload (the
acceptance rates the Markov runs measured); an accepted proposal becomes the
chain's configuration.  No trace is evaluated: the counts follow from the
sector dimensions along every surviving string.  Prints one JSON line per
workload."""

from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import panelref as P  # noqa: E402
from paper_2010_08482_amd.sectors import build_sectors  # noqa: E402
from workloads import make_impurity  # noqa: E402
from workloads.configs import insert_pair, make_configs, remove_pair  # noqa: E402

WORKLOADS = [("dshell", 1, 0.42), ("fshell", 2, 0.47), ("fshell_cf", 3, 0.47)]


def run(name, config_id, accept, n_cfg, n_prop, seed=11):
    imp = make_impurity(name)
    tab = build_sectors(imp)
    elem = 16 if tab.is_complex else 8
    rng = np.random.Generator(np.random.PCG64(seed))
    tot = {"full": 0, "panel": 0, "panel_accept": 0, "tree": 0}
    per_move = {"full": 0.0, "panel": 0.0, "tree": 0.0}
    mem_panel, mem_tree, n_states, moves, accepted, unmatched_share = [], [], 0, 0, 0, []
    for s in make_configs(config_id, n_cfg):
        old = [(r, p) for r, p in P.strings(tab, s.tau, s.op)]
        for _ in range(n_prop):
            if s.n <= 2 or rng.uniform() < 0.5:
                t = insert_pair(rng, s, imp.n_flavors, imp.beta)
            else:
                t = remove_pair(rng, s, imp.n_flavors)
            c = P.proposal_costs(tab, s.tau, s.op, old, t.tau, t.op)
            acc = rng.uniform() < accept
            for k in tot:
                tot[k] += c[k]
            per_move["full"] += c["full"]
            per_move["panel"] += c["panel"] + (c["panel_accept"] if acc else 0)
            per_move["tree"] += c["tree"]
            moves += 1
            if acc:
                accepted += 1
                s = t
                old = [(r, p) for r, p in P.strings(tab, s.tau, s.op)]
            if old:
                mem_panel.append(P.panel_elements(tab, s.tau, s.op) * elem)
                mem_tree.append(sum(P.tree_elements([int(tab.dims[q]) for q in p]) for _, p in old) * elem)
                n_states += 1
    f = per_move["full"]
    return {
        "workload": f"{name} (configurations of benchmark {config_id})", "chains": n_cfg, "proposals": moves,
        "accepted": accepted, "complex": bool(tab.is_complex),
        "macs_per_proposal": {k: v / moves for k, v in tot.items()},
        "macs_per_move": {k: v / moves for k, v in per_move.items()},
        "per_move_vs_full": {k: v / f for k, v in per_move.items()},
        "resident_bytes_per_chain": {"panels_mean": float(np.mean(mem_panel)), "panels_max": float(np.max(mem_panel)),
                                     "tree_mean": float(np.mean(mem_tree)), "tree_max": float(np.max(mem_tree))},
    }


def main():
    n_cfg = int(sys.argv[1]) if len(sys.argv) > 1 else 40
    n_prop = int(sys.argv[2]) if len(sys.argv) > 2 else 25
    for name, cid, acc in WORKLOADS:
        print(json.dumps(run(name, cid, acc, n_cfg, n_prop)), flush=True)


if __name__ == "__main__":
    main()
