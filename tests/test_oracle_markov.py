"""Pins of the oracle's Markov step (pair moves of App. D, hybridisation
determinant of Sec. 2.2, Metropolis of App. C) against facts that do not
come from the oracle.  CPU only."""

import math

import numpy as np
import pytest

from oracle import DenseTrace
from oracle.fock import occupations
from oracle.markov import OracleChain, anderson_occupation, bath_delta, propose
from oracle.observables import label_histogram, label_projectors
from workloads.impurity import Impurity


def resonant_level():
    imp = Impurity("rlm", 1, 5.0, np.array([[0.4]]), np.zeros((1,) * 4), np.array([[1]]), ("N",), {})
    return imp, [([-0.6, 0.9], [0.7, 0.5])]


def anderson_two_flavor():
    U = 2.0
    T = np.zeros((2,) * 4)
    T[0, 1, 1, 0] = T[1, 0, 0, 1] = U
    imp = Impurity("aim", 2, 5.0, -0.5 * np.eye(2), T, np.array([[1, 1], [-1, 1]]), ("N", "2Sz"), {})
    return imp, [([-0.7, 0.8], [0.6, 0.5])] * 2


def test_M1_bath_function_closed_forms():
    """Delta(0+) + Delta(beta-) = -sum V^2 and Delta(tau - beta) = -Delta(tau);
    a single level at eps = 0 gives the constant -V^2/2."""
    beta, eps, v = 5.0, [-0.6, 0.9, 2.5], [0.7, 0.5, 0.2]
    tiny = 1e-12
    assert abs(bath_delta(beta, eps, v, tiny) + bath_delta(beta, eps, v, beta - tiny) + np.sum(np.square(v))) < 1e-10
    for t in (0.3, 1.7, 4.9):
        assert abs(bath_delta(beta, eps, v, t - beta) + bath_delta(beta, eps, v, t)) < 1e-15
    assert abs(bath_delta(beta, [0.0], [0.8], 2.2) + 0.32) < 1e-15
    # large |eps beta| stays finite
    assert np.isfinite(bath_delta(400.0, [-3.0, 3.0], [1.0, 1.0], 200.0))


def _reverse_u(tau, op, new_tau, new_op, f, nf):
    """Random numbers of the removal that undoes an insertion: the flavor, and
    the index of the first inserted operator among the flavor's operators."""
    L = [i for i, o in enumerate(new_op) if o // 2 == f]
    added = [i for i in L if (new_tau[i], new_op[i]) not in set(zip(tau, op))]
    pos = [L.index(i) for i in added]
    N = len(L)
    first = pos[0] if (pos[0] + 1) % N == pos[1] else pos[1]
    return [0.75, (f + 0.5) / nf, (first + 0.5) / N, 0.0, 0.5, 0.0]


def test_M2_pair_moves_are_each_others_reverse_with_inverse_weights():
    """Detailed balance of the proposals: the removal that undoes an insertion
    exists, gives back the old configuration, and its proposal ratio is the
    inverse of the insertion's."""
    rng = np.random.Generator(np.random.PCG64(501))
    nf, beta = 3, 7.0
    tau, op = [], []
    checked = 0
    for _ in range(400):
        u = rng.uniform(size=6)
        u[0] = 0.25
        p = propose(tau, op, u, nf, beta)
        if p is None:
            continue
        nt, no, q = p
        f = min(nf - 1, int(u[1] * nf))
        back = propose(nt, no, _reverse_u(tau, op, nt, no, f, nf), nf, beta)
        assert back is not None
        bt, bo, qb = back
        assert bt == list(tau) and bo == list(op)
        assert abs(q * qb - 1.0) < 1e-12
        checked += 1
        if rng.uniform() < 0.7 or len(op) > 16:
            tau, op = nt, no   # walk on to configurations of higher order
        if len(op) > 24:
            tau, op = [], []
    assert checked > 300


def test_M3_alternation_is_kept():
    """Pauli-aware moves never create or annihilate a flavor twice in a row."""
    rng = np.random.Generator(np.random.PCG64(502))
    nf, beta = 2, 4.0
    tau, op = [], []
    for _ in range(3000):
        p = propose(tau, op, rng.uniform(size=6), nf, beta)
        if p is None:
            continue
        tau, op, _ = p
        for f in range(nf):
            kinds = [o % 2 for o in op if o // 2 == f]
            assert all(kinds[i] != kinds[(i + 1) % len(kinds)] for i in range(len(kinds))) or not kinds


def _run_chain(imp, baths, steps, seed):
    dt = DenseTrace(imp)
    P = label_projectors(dt, occupations(imp.n_flavors).sum(axis=1), imp.n_flavors + 1)
    rng = np.random.Generator(np.random.PCG64(seed))
    ch = OracleChain(dt, baths)
    vals = []
    for i in range(steps):
        ch.step(rng.uniform(size=6))
        if i >= 1000 and i % 10 == 0:
            h, _ = label_histogram(dt, ch.tau, ch.op, P)
            vals.append(float(np.real(np.arange(len(h)) @ h)))
    vals = np.array(vals)
    nb = 20
    bm = vals[: len(vals) // nb * nb].reshape(nb, -1).mean(axis=1)
    return vals.mean(), bm.std(ddof=1) / math.sqrt(nb)


@pytest.mark.parametrize("model,steps", [(resonant_level, 20000), (anderson_two_flavor, 24000)])
def test_M4_sampled_occupation_matches_exact_diagonalisation(model, steps):
    """The chain samples |w_loc w_hyb|; the N histogram averaged over it must
    give the occupation of the impurity coupled to its bath, computed by
    diagonalising impurity plus bath levels (4 sigma of batch means).  A
    proposal ratio off by a factor 2, or the hybridisation argument
    reversed, moves the estimate by 7 and 20 sigma on the resonant level."""
    imp, baths = model()
    exact = anderson_occupation(imp, baths)
    est, err = _run_chain(imp, baths, steps, 503)
    assert abs(est - exact) < 4 * err + 1e-3, (est, err, exact)
