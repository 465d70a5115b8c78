"""The resident-panel route for Markov proposals (tests/panelref.py) against
the oracle, and its cost counts on hand-checkable cases (CPU only)."""

import math

import numpy as np
import pytest

import tests.panelref as P
from oracle import DenseTrace
from paper_2010_08482_amd.sectors import build_sectors
from tests.tracecmp import close_enough
from workloads import make_impurity
from workloads.configs import insert_pair, random_string, remove_pair


@pytest.mark.parametrize("name,seed", [("kanamori2", 3), ("pshell", 4)])
def test_panel_proposals_match_the_oracle(name, seed):
    """A chain of pair insertions and removals, half of them accepted: every
    proposal evaluated from the current configuration's panels equals the
    oracle's trace of the proposed configuration, and Tr[B_m F_m] is the
    same for every cut m of every resident string."""
    imp = make_impurity(name)
    tab = build_sectors(imp)
    dt = DenseTrace(imp)
    rng = np.random.Generator(np.random.PCG64(seed))
    s = random_string(rng, imp.n_flavors, imp.beta, 16, "alternating")
    res = P.residents_of(tab, s.tau, s.op)
    n_nonzero, saved = 0, 0
    for _ in range(40):
        if s.n <= 2 or rng.uniform() < 0.5:
            t = insert_pair(rng, s, imp.n_flavors, imp.beta)
        else:
            t = remove_pair(rng, s, imp.n_flavors)
        (m, l), spent, full = P.propose(tab, s.tau, s.op, res, t.tau, t.op)
        ref = dt.trace(t.tau, t.op)
        if ref[0] == 0:
            assert m == 0
        else:
            A = dt.abs_scale(t.tau, t.op)
            assert close_enough((m, l), ref, A), (m, l, ref)
            n_nonzero += 1
        saved += full - spent
        if rng.uniform() < 0.5:
            s, res = t, P.residents_of(tab, t.tau, t.op)
            for r in res:
                v0 = r.value()
                for cut in range(len(r.steps) + 1):
                    v = r.value(cut)
                    assert abs(v[0] * math.exp(v[1] - v0[1]) - v0[0]) <= 1e-12 * abs(v0[0])
    assert n_nonzero >= 20 and saved > 0


def test_panel_and_tree_counts_by_hand():
    """Cost counts on a string whose sector dimensions are written out: the
    tree over four steps with dimensions 2,3,4,5,2 has nodes [0,4) split at 2
    (2*4*2), [0,2) (4*3*2) and [2,4) (2*5*4); a change in step 3 touches
    [0,4) and [2,4) only."""
    dims = [2, 3, 4, 5, 2]
    assert P.tree_macs(dims, None) == 2 * 4 * 2 + 4 * 3 * 2 + 2 * 5 * 4
    assert P.tree_macs(dims, (3, 4)) == 2 * 4 * 2 + 2 * 5 * 4
    assert P.tree_macs(dims, (0, 1)) == 2 * 4 * 2 + 4 * 3 * 2
    # leaves (one block per step) plus the three nodes' d_out x d_in
    assert P.tree_elements(dims) == (3 * 2 + 4 * 3 + 5 * 4 + 2 * 5) + (2 * 2 + 4 * 2 + 2 * 4)


def test_unchanged_proposal_costs_only_the_closing_trace():
    """Proposing the current configuration again: every string is matched,
    nothing in the middle is recomputed, the panel route spends w x d per
    string (the closing trace) against a full pass."""
    imp = make_impurity("pshell")
    tab = build_sectors(imp)
    rng = np.random.Generator(np.random.PCG64(9))
    s = random_string(rng, imp.n_flavors, imp.beta, 12, "alternating")
    old = P.strings(tab, s.tau, s.op)
    assert old
    c = P.proposal_costs(tab, s.tau, s.op, old, s.tau, s.op)
    assert c["panel"] == sum(int(tab.dims[p[0]]) * int(tab.dims[p[0]]) for _, p in old)
    assert c["tree"] == 0 and c["panel_accept"] == c["full"] > c["panel"]


@pytest.mark.parametrize("name,cid,count", [("kanamori2", 0, 40), ("pshell_cf", None, 12), ("dshell", 1, 4)])
def test_block_reference_matches_the_oracle(name, cid, count):
    """The NumPy block-sparse reference (the bench's CPU block-sparse
    baseline, tests/blockref.py) against the oracle's dense trace."""
    from tests.blockref import block_trace
    from workloads import make_configs

    imp = make_impurity(name)
    tab = build_sectors(imp)
    dt = DenseTrace(imp)
    if cid is None:
        rng = np.random.Generator(np.random.PCG64(17))
        strings = [random_string(rng, imp.n_flavors, imp.beta, 2 * int(rng.integers(1, 15)), "alternating")
                   for _ in range(count)]
    else:
        strings = make_configs(cid, count)
    nonzero = 0
    for s in strings:
        got, ref = block_trace(tab, s.tau, s.op), dt.trace(s.tau, s.op)
        if ref[0] == 0:
            assert got[0] == 0
            continue
        assert close_enough(got, ref, dt.abs_scale(s.tau, s.op))
        nonzero += 1
    assert nonzero >= count // 3
