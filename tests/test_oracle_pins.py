"""Pins of the CPU oracle against facts fixed by the paper and by the
mathematics (not by the oracle itself).  CPU only."""

import math

import numpy as np
import pytest

from oracle import DenseTrace, densdens_trace, expm_trace
from oracle.densdens import densdens_partition_function
from oracle.labels import label_table, label_walk
from tests.tracecmp import add, close_enough, insert_ops, rel_err
from workloads import make_configs, make_impurity
from workloads.configs import random_string


@pytest.fixture(scope="module")
def k2():
    imp = make_impurity("kanamori2")
    return imp, DenseTrace(imp)


def _Z_closed(beta):
    # spectrum of the half-filled 2-orbital Kanamori atom (U=4, J=0.5, mu=4.75):
    # 0 x2 (N=0,4), -4.75 x8 (N=1,3), N=2: U-3J, U-J, U+J minus 2mu = -7 x3, -6 x2, -5
    # Z e^{-7 beta} expressed relative to E0 = -7
    return (2 * math.exp(-7 * beta) + 8 * math.exp(-2.25 * beta) + 3 + 2 * math.exp(-beta)
            + math.exp(-2 * beta)), 7 * beta


def test_P1_partition_function_closed_form(k2):
    imp, dt = k2
    got = dt.trace([], [])
    assert rel_err(got, _Z_closed(imp.beta)) < 1e-13
    assert rel_err(dt.partition_function(), _Z_closed(imp.beta)) < 1e-13


def test_P1_kanamori_two_electron_multiplets(k2):
    imp, dt = k2
    # N=0,4: 0 ; N=1,3: -4.75 ; N=2: U-3J, U-J, U+J minus 2 mu
    want = sorted([0.0, 0.0] + [-4.75] * 8 + [-7.0] * 3 + [-6.0] * 2 + [-5.0])
    assert np.allclose(np.sort(dt.E), want, atol=1e-12)


@pytest.mark.parametrize("tau", [0.3, 1.7, 5.0, 9.2])
def test_P2_hubbard_atom_greens_function(tau):
    """Sec. 4.1 atom (U=4, eps_f=-U/2, beta=10):
    Tr[e^{-(beta-tau)H} c e^{-tau H} c+] / Z = (e^{-tau U/2} + e^{-(beta-tau)U/2}) / (2(1+e^{-beta U/2}))."""
    imp = make_impurity("hubbard_atom")
    dt = DenseTrace(imp)
    U, beta = 4.0, imp.beta
    for flavor in (0, 1):
        w = dt.trace([0.0, tau], [2 * flavor + 1, 2 * flavor])
        z = dt.trace([], [])
        m, l = w
        mz, lz = z
        g = m / mz * math.exp(l - lz)
        want = (math.exp(-tau * U / 2) + math.exp(-(beta - tau) * U / 2)) / (2 * (1 + math.exp(-beta * U / 2)))
        assert abs(g - want) < 1e-13 * want


def test_P3_anticommutator_inserts_identity(k2):
    imp, dt = k2
    rng = np.random.Generator(np.random.PCG64(7))
    for i in range(40):
        s = random_string(rng, 4, imp.beta, 2 * int(rng.integers(0, 5)), "alternating")
        base = dt.trace(s.tau, s.op)
        t_new = float(rng.uniform(0, imp.beta))
        f = int(rng.integers(4))
        a = dt.trace(*insert_ops(s.tau, s.op, t_new, [2 * f + 1, 2 * f]))  # c_f c+_f
        b = dt.trace(*insert_ops(s.tau, s.op, t_new, [2 * f, 2 * f + 1]))  # c+_f c_f
        if base[0] == 0:
            assert abs(add(a, b)[0]) == pytest.approx(0, abs=1e-12 * max(abs(a[0]), abs(b[0]), 1e-300))
        else:
            assert rel_err(add(a, b), base) < 1e-11


def test_P3_particle_number_half_filling(k2):
    """sum_f Tr[e^{-beta H} n_f] = <N> Z = 2 Z at the particle-hole symmetric point."""
    imp, dt = k2
    tot = (0.0, 0.0)
    for f in range(4):
        tot = add(tot, dt.trace([3.3, 3.3], [2 * f, 2 * f + 1]))
    zm, zl = _Z_closed(imp.beta)
    assert rel_err(tot, (2 * zm, zl)) < 1e-13


def _shift(s_tau, s_op, delta, beta):
    t = (np.asarray(s_tau) + delta) % beta
    order = np.argsort(t, kind="stable")
    return t[order], np.asarray(s_op)[order]


@pytest.mark.parametrize("name", ["kanamori2", "pshell"])
def test_P4_cyclicity(name):
    imp = make_impurity(name)
    dt = DenseTrace(imp)
    rng = np.random.Generator(np.random.PCG64(11))
    for i in range(25):
        s = random_string(rng, imp.n_flavors, imp.beta, 2 * int(rng.integers(1, 6)), "alternating")
        w = dt.trace(s.tau, s.op)
        w2 = dt.trace(*_shift(s.tau, s.op, float(rng.uniform(0, imp.beta)), imp.beta))
        if w[0] != 0:
            assert rel_err(w2, w) < 1e-10


@pytest.mark.parametrize("name", ["kanamori2", "pshell", "pshell_cf"])
def test_P5_conjugation(name):
    """w(C)^* equals the trace of the reversed string with c <-> c+ and tau -> beta - tau."""
    imp = make_impurity(name)
    dt = DenseTrace(imp)
    rng = np.random.Generator(np.random.PCG64(13))
    for i in range(20):
        s = random_string(rng, imp.n_flavors, imp.beta, 2 * int(rng.integers(1, 6)), "alternating")
        w = dt.trace(s.tau, s.op)
        tau_r = imp.beta - s.tau[::-1]
        op_r = s.op[::-1] ^ 1
        wr = dt.trace(tau_r, op_r)
        if w[0] != 0:
            assert rel_err((np.conj(wr[0]), wr[1]), w) < 1e-10


def test_P6_gauge_invariance():
    a = make_impurity("pshell")
    b = make_impurity("pshell_real")
    assert a.is_complex and not b.is_complex
    da, db = DenseTrace(a), DenseTrace(b)
    assert np.allclose(da.E, db.E, atol=1e-10)
    rng = np.random.Generator(np.random.PCG64(17))
    for i in range(20):
        s = random_string(rng, 6, a.beta, 2 * int(rng.integers(1, 8)), "alternating")
        wa, wb = da.trace(s.tau, s.op), db.trace(s.tau, s.op)
        if wb[0] != 0:
            assert close_enough(wa, wb, db.abs_scale(s.tau, s.op))


def test_P7_density_density_brute_force_matches_dense():
    """Two independent constructions: bit enumeration vs dense eigenbasis chain."""
    imp = make_impurity("dd_dshell")
    dt = DenseTrace(imp)
    assert rel_err(densdens_partition_function(imp), dt.partition_function()) < 1e-12
    rng = np.random.Generator(np.random.PCG64(19))
    nz = 0
    for i in range(12):
        s = random_string(rng, 10, imp.beta, 2 * int(rng.integers(1, 16)), "alternating")
        a, b = densdens_trace(imp, s.tau, s.op), dt.trace(s.tau, s.op)
        if b[0] == 0:
            assert a[0] == 0
        else:
            nz += 1
            assert rel_err(a, b) < 1e-10
    assert nz >= 8


def test_P8_expm_route_matches_eigen_route_all_config0(k2):
    imp, dt = k2
    cfgs = make_configs(0)
    assert len(cfgs) == 1000
    nonzero = 0
    for c in cfgs:
        a, b = dt.trace(c.tau, c.op), expm_trace(imp, c.tau, c.op)
        if a[0] == 0 and b[0] == 0:
            continue
        nonzero += 1
        assert rel_err(a, b) < 1e-10
    assert nonzero > 300


def test_label_table_closed_form():
    """Every operator shifts each abelian charge by -+q_f; the table entry is
    dead exactly when no state with that label has the needed occupation."""
    for name in ("kanamori2", "pshell"):
        imp = make_impurity(name)
        keys, nxt = label_table(imp)
        qn = np.asarray(imp.qn)
        nf = imp.n_flavors
        occ = ((np.arange(1 << nf)[:, None] >> np.arange(nf)[None, :]) & 1)
        labs = occ @ qn.T
        for k in keys:
            in_k = np.all(labs == np.array(k), axis=1)
            for code in range(2 * nf):
                f, dag = code // 2, code % 2
                possible = np.any(in_k & (occ[:, f] == (0 if dag else 1)))
                want = tuple(int(v) for v in (np.array(k) + (qn[:, f] if dag else -qn[:, f]))) if possible else None
                assert nxt[(k, code)] == want


def test_label_walk_zero_strings_have_zero_trace(k2):
    imp, dt = k2
    table = label_table(imp)
    for c in make_configs(0, 300):
        surv = label_walk(imp, c.op, table)
        if not surv:
            assert dt.trace(c.tau, c.op)[0] == 0.0
