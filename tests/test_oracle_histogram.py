"""Pins of the oracle's label histogram (the density-matrix estimator of
Sec. 2.3.2 summed over the states of one conserved label, as in the valence
histogram of Sec. 4.2) against facts that do not come from the oracle.  CPU only."""

import math

import numpy as np
import pytest
import scipy.linalg

from oracle import DenseTrace
from oracle.fock import occupations, operator
from oracle.hamiltonian import hamiltonian_dense
from oracle.observables import label_histogram, label_histogram_abs, label_projectors
from workloads import make_impurity
from workloads.configs import random_string
from workloads.impurity import _density_density


def _n_labels(imp):
    return occupations(imp.n_flavors).sum(axis=1).astype(np.int64)


@pytest.fixture(scope="module")
def k2():
    imp = make_impurity("kanamori2")
    dt = DenseTrace(imp)
    return imp, dt, label_projectors(dt, _n_labels(imp), imp.n_flavors + 1)


def test_H1_order_zero_is_the_boltzmann_distribution_over_N(k2):
    """Empty configuration: h_N = Tr[P_N e^{-beta H}] / Z.  Kanamori atom
    (U=4, J=0.5, mu=4.75) levels relative to E0=-7: N=0,4 one state at +7,
    N=1,3 four at +2.25, N=2 three at 0, two at +1, one at +2."""
    imp, dt, P = k2
    b = imp.beta
    w = np.array([math.exp(-7 * b), 4 * math.exp(-2.25 * b), 3 + 2 * math.exp(-b) + math.exp(-2 * b),
                  4 * math.exp(-2.25 * b), math.exp(-7 * b)])
    h, _ = label_histogram(dt, [], [], P)
    assert np.max(np.abs(h - w / w.sum())) < 1e-14


def test_H2_labels_sum_to_one(k2):
    """sum_l P_l = 1, hence sum_l h_l = 1 for every nonzero configuration."""
    imp, dt, P = k2
    rng = np.random.Generator(np.random.PCG64(301))
    seen = 0
    for _ in range(12):
        s = random_string(rng, imp.n_flavors, imp.beta, 2 * int(rng.integers(1, 5)), "alternating")
        h, w = label_histogram(dt, s.tau, s.op, P)
        if w[0] == 0:
            assert np.all(h == 0)
            continue
        seen += 1
        assert abs(h.sum() - 1.0) < 1e-11
    assert seen >= 6


def _expm_histogram(imp, tau, op, state_label, n_labels, rng):
    """Independent route: occupation basis, P(x) = expm(-x H) (no
    eigendecomposition), the projector diag(1[label == l]) inserted at a
    RANDOM time inside every interval between operator times."""
    H = hamiltonian_dense(imp.h1, imp.U)
    D = H.shape[0]
    ops = [operator(imp.n_flavors, int(o)).toarray() for o in op]
    edges = np.concatenate([[0.0], tau, [imp.beta]])
    n_gaps = len(tau) + 1
    # one random insertion time per interval, shared by all labels: the
    # interval's propagator and its two pieces around that time
    whole, before, after = [], [], []
    for g in range(n_gaps):
        length = edges[g + 1] - edges[g]
        t_ins = edges[g] + rng.uniform(0.05, 0.95) * length
        whole.append(scipy.linalg.expm(-length * H))
        before.append(scipy.linalg.expm(-(t_ins - edges[g]) * H))
        after.append(scipy.linalg.expm(-(edges[g + 1] - t_ins) * H))

    def chain(g_ins, P):
        X = np.eye(D, dtype=complex)
        for g in range(n_gaps):
            X = (after[g] @ (P @ (before[g] @ X))) if g == g_ins else whole[g] @ X
            if g < len(tau):
                X = ops[g] @ X
        return np.trace(X)

    w = chain(-1, None)
    h = np.zeros(n_labels, dtype=complex)
    for l in range(n_labels):
        P = np.diag((state_label == l).astype(float))
        for g in range(n_gaps):
            h[l] += (edges[g + 1] - edges[g]) * chain(g, P)
    return h / (imp.beta * w)


@pytest.mark.parametrize("name", ["kanamori2", "pshell"])
def test_H3_random_insertion_times_with_expm(name):
    """The integrand is constant between operator times (P_l commutes with
    H_loc): inserting the projector at random times inside each interval, in
    the occupation basis with scipy's expm, gives the same histogram."""
    imp = make_impurity(name)
    dt = DenseTrace(imp)
    lab = _n_labels(imp)
    P = label_projectors(dt, lab, imp.n_flavors + 1)
    rng = np.random.Generator(np.random.PCG64(302))
    checked = 0
    for _ in range(6):
        s = random_string(rng, imp.n_flavors, imp.beta, 2 * int(rng.integers(1, 3)), "alternating")
        h, w = label_histogram(dt, s.tau, s.op, P)
        if w[0] == 0 or abs(w[0]) * math.exp(w[1]) < 1e-200:
            continue
        scale = label_histogram_abs(dt, s.tau, s.op, P)
        ref = _expm_histogram(imp, s.tau, s.op, lab, imp.n_flavors + 1, rng)
        assert np.all(np.abs(h - ref) <= 1e-8 * np.maximum(scale, 1.0))
        checked += 1
    assert checked >= 3


def _brute_histogram(imp, tau, op, n_labels):
    """Density-density impurity: every occupation state is an eigenstate, each
    operator maps a state to one state with a sign, so the trace is a sum over
    start states and the time each path spends at each N is read off the
    path."""
    nf = imp.n_flavors
    eps = np.real(np.diag(np.asarray(imp.h1)))
    V = np.asarray(imp.params["V"])
    num = np.zeros(n_labels)
    den = 0.0
    for s0 in range(1 << nf):
        s, sign, t_prev = s0, 1.0, 0.0
        segs = []
        alive = True
        for t, o in zip(tau, op):
            segs.append((t - t_prev, s))
            f, dag = int(o) // 2, int(o) % 2
            if ((s >> f) & 1) == dag:
                alive = False
                break
            if bin(s & ((1 << f) - 1)).count("1") % 2:
                sign = -sign
            s ^= 1 << f
            t_prev = t
        if not alive or s != s0:
            continue
        segs.append((imp.beta - t_prev, s))
        expo = 0.0
        for dtau, st in segs:
            n = np.array([(st >> f) & 1 for f in range(nf)], dtype=float)
            expo += dtau * (eps @ n + 0.5 * n @ V @ n)
        wgt = sign * math.exp(-expo)
        den += wgt
        for dtau, st in segs:
            num[bin(st).count("1")] += wgt * dtau
    return num / (imp.beta * den)


def test_H4_density_density_brute_force():
    imp = _density_density("dd_pshell", 3, 8.0, 311, "NS", False)
    dt = DenseTrace(imp)
    P = label_projectors(dt, _n_labels(imp), imp.n_flavors + 1)
    rng = np.random.Generator(np.random.PCG64(303))
    checked = 0
    for _ in range(10):
        s = random_string(rng, imp.n_flavors, imp.beta, 2 * int(rng.integers(1, 4)), "alternating")
        h, w = label_histogram(dt, s.tau, s.op, P)
        if w[0] == 0:
            continue
        ref = _brute_histogram(imp, s.tau, s.op, imp.n_flavors + 1)
        assert np.max(np.abs(h - ref)) < 1e-10
        checked += 1
    assert checked >= 4


def test_H5_non_conserved_label_is_refused(k2):
    """A label that does not commute with H_loc (here: occupation of flavor 0
    in the Kanamori atom, which spin flips and pair hopping change) has no
    interval-sum estimator."""
    imp, dt, _ = k2
    occ0 = occupations(imp.n_flavors)[:, 0].astype(np.int64)
    with pytest.raises(ValueError):
        label_projectors(dt, occ0, 2)
