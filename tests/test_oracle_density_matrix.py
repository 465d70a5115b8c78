"""Pins of the oracle's density-matrix estimator (Sec. 2.3.2, tau-integrated,
per configuration) against facts that do not come from the function itself.
CPU only."""

import math

import numpy as np
import pytest
import scipy.linalg

from oracle import DenseTrace
from oracle.fock import occupations, operator
from oracle.hamiltonian import hamiltonian_dense
from oracle.observables import density_matrix, label_histogram, label_projectors
from tests.tracecmp import rel_err
from workloads import make_impurity
from workloads.configs import random_string


@pytest.fixture(scope="module")
def k2():
    imp = make_impurity("kanamori2")
    return imp, DenseTrace(imp)


def test_D1_trace_is_one(k2):
    for name in ("kanamori2", "pshell_cf"):
        imp = make_impurity(name)
        dt = DenseTrace(imp)
        rng = np.random.Generator(np.random.PCG64(401))
        seen = 0
        for _ in range(10):
            s = random_string(rng, imp.n_flavors, imp.beta, 2 * int(rng.integers(1, 5)), "alternating")
            R, w = density_matrix(dt, s.tau, s.op)
            if w[0] == 0:
                assert np.all(R == 0)
                continue
            seen += 1
            assert abs(np.trace(R) - 1.0) < 1e-11
            assert rel_err(w, dt.trace(s.tau, s.op)) < 1e-11
        assert seen >= 5


def test_D2_order_zero_is_the_boltzmann_distribution(k2):
    """Empty configuration: R = exp(-beta H) / Z, diagonal in the eigenbasis,
    with the Kanamori atom's spectrum relative to E0 = -7: 0 x3, 1 x2, 2,
    2.25 x8, 7 x2 (U = 4, J = 0.5, mu = 4.75)."""
    imp, dt = k2
    R, _ = density_matrix(dt, [], [])
    assert np.max(np.abs(R - np.diag(np.diag(R)))) == 0
    levels = sorted([0.0] * 3 + [1.0] * 2 + [2.0] + [2.25] * 8 + [7.0] * 2)
    b = imp.beta
    want = np.exp(-b * np.array(levels))
    want /= want.sum()
    assert np.max(np.abs(np.sort(np.diag(R).real)[::-1] - np.sort(want)[::-1])) < 1e-15


def test_D3_label_sums_are_the_histogram(k2):
    """Tr[P_l R] for the projector on the states of electron number l equals
    the label histogram h_l, which inserts P_l at the start of every interval."""
    for name in ("kanamori2", "pshell"):
        imp = make_impurity(name)
        dt = DenseTrace(imp)
        lab = occupations(imp.n_flavors).sum(axis=1).astype(np.int64)
        P = label_projectors(dt, lab, imp.n_flavors + 1)
        rng = np.random.Generator(np.random.PCG64(402))
        seen = 0
        for _ in range(6):
            s = random_string(rng, imp.n_flavors, imp.beta, 2 * int(rng.integers(1, 4)), "alternating")
            R, w = density_matrix(dt, s.tau, s.op)
            if w[0] == 0:
                continue
            h, _ = label_histogram(dt, s.tau, s.op, P)
            got = np.array([np.trace(Pl @ R) for Pl in P])
            assert np.max(np.abs(got - h)) < 1e-11
            seen += 1
        assert seen >= 3


def _quadrature_density_matrix(imp, tau, op, nodes=8, piece=0.25):
    """Independent route in the occupation basis: propagators from scipy's
    expm (no eigendecomposition), the time-ordered product cut at tau and
    closed the other way round, integrated over tau by composite Gauss-Legendre
    quadrature on pieces of at most `piece` per interval."""
    H = hamiltonian_dense(imp.h1, imp.U)
    D = H.shape[0]
    ops = [operator(imp.n_flavors, int(o)).toarray() for o in op]
    edges = np.concatenate([[0.0], tau, [imp.beta]])
    n = len(tau)

    def P(x):
        return scipy.linalg.expm(-x * H)

    pre = [np.eye(D, dtype=complex)]
    for g in range(1, n + 1):
        pre.append(ops[g - 1] @ P(edges[g] - edges[g - 1]) @ pre[-1])
    suf = [None] * (n + 1)
    suf[n] = np.eye(D, dtype=complex)
    for g in range(n - 1, -1, -1):
        suf[g] = suf[g + 1] @ P(edges[g + 2] - edges[g + 1]) @ ops[g]
    w = np.trace(suf[0] @ P(edges[1]))
    x, wt = np.polynomial.legendre.leggauss(nodes)
    R = np.zeros((D, D), dtype=complex)
    for g in range(n + 1):
        a, b = edges[g], edges[g + 1]
        m = max(1, int(math.ceil((b - a) / piece)))
        for k in range(m):
            lo, hi = a + (b - a) * k / m, a + (b - a) * (k + 1) / m
            for xi, wi in zip(x, wt):
                t = 0.5 * (hi - lo) * xi + 0.5 * (hi + lo)
                R += 0.5 * (hi - lo) * wi * (P(t - a) @ pre[g] @ suf[g] @ P(b - t))
    return R / (imp.beta * w)


@pytest.mark.parametrize("name", ["kanamori2", "pshell_cf"])
def test_D4_quadrature_in_the_occupation_basis(name):
    """The closed-form interval integrals in the eigenbasis against numerical
    quadrature of the cut products in the occupation basis (expm propagators):
    a swapped pair (u, v) in the interval integral, a wrong interval or a
    misplaced cut moves the result far beyond the bar."""
    from threadpoolctl import threadpool_limits

    imp = make_impurity(name)
    dt = DenseTrace(imp)
    rng = np.random.Generator(np.random.PCG64(403))
    # many small (64 x 64) matrix exponentials: BLAS threads only add synchronisation
    with threadpool_limits(limits=1):
        _check_quadrature(imp, dt, rng)


def _check_quadrature(imp, dt, rng):
    seen = 0
    for _ in range(4):
        s = random_string(rng, imp.n_flavors, imp.beta, 2 * int(rng.integers(1, 3)), "alternating")
        R, w = density_matrix(dt, s.tau, s.op)
        if w[0] == 0:
            continue
        ref = _quadrature_density_matrix(imp, s.tau, s.op)
        got = dt.V @ R @ dt.V.conj().T
        assert np.max(np.abs(got - ref)) < 1e-9 * max(1.0, np.max(np.abs(ref)))
        seen += 1
    assert seen >= 2
