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


# ---------------------------------------------------------------------------
# cancellation scales, the component-wise eigensolve at beta = 50, both
# directions of the label walk, and the memory-bounded route
# ---------------------------------------------------------------------------

def _dd_pshell():
    from workloads.impurity import _density_density
    return _density_density("dd_pshell", 3, 8.0, 311, "NS", False)


@pytest.mark.parametrize("which", ["dd_dshell", "dd_pshell"])
def test_abs_scale_is_the_modulus_sum_of_the_enumeration(which):
    """For an occupation-diagonal H every Lehmann term of w_loc is one signed
    path of the bit enumeration, so A = sum of |terms| is the enumeration with
    the signs dropped.  (All paths of one string share their sign there, so
    A = |w|: negative traces catch a dropped modulus.)  Log scales reach
    ~2.5e3 at beta = 50, where every exp(l - M) carries ~2.5e3 ulp of
    rounding: bar 5e-12."""
    imp = make_impurity(which) if which == "dd_dshell" else _dd_pshell()
    dt = DenseTrace(imp)
    rng = np.random.Generator(np.random.PCG64(23))
    checked = negative = 0
    for _ in range(14):
        s = random_string(rng, imp.n_flavors, imp.beta, 2 * int(rng.integers(1, 12)), "alternating")
        a = dt.abs_scale(s.tau, s.op)
        m = densdens_trace(imp, s.tau, s.op, moduli=True)
        t = densdens_trace(imp, s.tau, s.op)
        if m[0] == 0:
            assert a[0] == 0
            continue
        checked += 1
        assert a[0] > 0
        assert rel_err(a, m) < 5e-12
        negative += t[0] < 0
    assert checked >= 8 and negative >= 2


def _lehmann_modulus_sum(dt, tau, op):
    """sum over all eigenstate paths a_0 -> a_1 -> ... -> a_n = a_0 of
    prod_j |<a_j+1| O_j |a_j>| exp(-dtau_j (E_a_j - E0)), enumerated path by
    path (16^n paths), as (value, log_scale) with log_scale = -beta E0."""
    n = len(op)
    D = dt.E.shape[0]
    E = dt.E - dt.E0
    gaps = np.diff(np.concatenate([[0.0], tau]))
    gaps[0] += dt.beta - tau[-1]               # P(tau_1) and P(beta - tau_n) both act on a_0
    paths = np.indices((D,) * n).reshape(n, -1)  # paths[j] = a_j
    w = np.ones(paths.shape[1])
    for j in range(n):
        M = np.abs(dt.op_matrix(int(op[j])))
        w *= M[paths[(j + 1) % n], paths[j]] * np.exp(-gaps[j] * E[paths[j]])
    return float(np.sum(w)), -dt.beta * dt.E0


def test_abs_scale_is_the_lehmann_modulus_sum_with_cancellation(k2):
    """Kanamori atom (spin flips and pair hopping: eigenstates are
    superpositions, so terms of one string carry different signs): A from the
    modulus chain against the path-by-path sum of |terms| at orders 2 and 4."""
    imp, dt = k2
    rng = np.random.Generator(np.random.PCG64(31))
    checked = cancelling = 0
    for i in range(24):
        s = random_string(rng, 4, imp.beta, 2 if i % 3 == 0 else 4, "random")
        a = dt.abs_scale(s.tau, s.op)
        w = dt.trace(s.tau, s.op)
        ref = _lehmann_modulus_sum(dt, s.tau, s.op)
        if ref[0] == 0:
            assert a[0] == 0
            continue
        checked += 1
        assert rel_err(a, ref) < 1e-12
        cancelling += abs(complex(w[0])) * math.exp(w[1] - a[1]) < 0.9 * a[0]
    assert checked >= 12 and cancelling >= 3


def _brute_histogram_moduli(imp, tau, op, n_labels):
    """The path enumeration of the density-density histogram with every path
    weight replaced by its modulus (the interval sums of moduli)."""
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
        wgt = math.exp(-expo)
        den += sign * wgt
        for dtau, st in segs:
            num[bin(st).count("1")] += wgt * dtau
    return num / (imp.beta * abs(den))


def test_label_histogram_abs_is_the_modulus_enumeration():
    from oracle.fock import occupations
    from oracle.observables import label_histogram_abs, label_projectors

    imp = _dd_pshell()
    dt = DenseTrace(imp)
    lab = occupations(imp.n_flavors).sum(axis=1).astype(np.int64)
    P = label_projectors(dt, lab, imp.n_flavors + 1)
    rng = np.random.Generator(np.random.PCG64(304))
    checked = 0
    for _ in range(10):
        s = random_string(rng, imp.n_flavors, imp.beta, 2 * int(rng.integers(1, 4)), "alternating")
        if dt.trace(s.tau, s.op)[0] == 0:
            continue
        got = label_histogram_abs(dt, s.tau, s.op, P)
        ref = _brute_histogram_moduli(imp, s.tau, s.op, imp.n_flavors + 1)
        assert np.all(got >= 0)
        assert np.max(np.abs(got - ref)) <= 1e-11 * max(1.0, float(np.max(ref)))
        checked += 1
    assert checked >= 4


def test_expm_route_matches_eigen_route_dshell_beta50():
    """The component-wise eigensolve (each connected component of H's nonzero
    pattern diagonalised alone, which the d-shell at beta = 50 needs) against
    scipy's matrix exponential in the occupation basis, which uses no
    eigendecomposition: the 20 lowest-order workload strings of the d-shell
    benchmark (orders 20-22, 1024 states)."""
    imp = make_impurity("dshell")
    dt = DenseTrace(imp)
    cfgs = make_configs(1, 400)
    low = sorted(range(len(cfgs)), key=lambda i: (cfgs[i].n, i))[:20]
    nonzero = 0
    for i in low:
        c = cfgs[i]
        a, b = dt.trace(c.tau, c.op), expm_trace(imp, c.tau, c.op)
        if a[0] == 0 and b[0] == 0:
            continue
        nonzero += 1
        assert rel_err(a, b) < 1e-10, (i, c.n)
    assert nonzero >= 15


def _reachable_start_labels(imp, op):
    """Start labels whose walk survives, by brute force over occupation states
    (bits, not the label table): from the states of label k, the labels of the
    states an operator leaves nonzero; the walk dies when that set is empty and
    survives if label k is among the labels reached at the end."""
    nf = imp.n_flavors
    qn = np.asarray(imp.qn)
    lab = [tuple(int(v) for v in ((np.array([(s >> (nf - 1 - f)) & 1 for f in range(nf)]) @ qn.T)))
           for s in range(1 << nf)]
    groups = {}
    for s, k in enumerate(lab):
        groups.setdefault(k, []).append(s)
    out = []
    for k0 in sorted(groups):
        cur = {k0}
        for o in op:
            f, dag = int(o) // 2, int(o) % 2
            bit = 1 << (nf - 1 - f)      # flavor 0 is the most significant bit (Jordan-Wigner order)
            nxt = set()
            for k in cur:
                for s in groups[k]:
                    if bool(s & bit) != bool(dag):
                        nxt.add(lab[s ^ bit])
            cur = nxt
            if not cur:
                break
        if k0 in cur:
            out.append(k0)
    return out


@pytest.mark.parametrize("name,rule", [("kanamori2", "random"), ("pshell", "alternating"), ("pshell_cf", "random")])
def test_label_walk_equals_state_reachability(name, rule):
    """Both directions of the label walk against brute force over occupation
    states (no label table): a label survives exactly when some chain of
    states with nonzero operator action leads from it back to it."""
    imp = make_impurity(name)
    table = label_table(imp)
    rng = np.random.Generator(np.random.PCG64(37))
    kept = 0
    for _ in range(40):
        s = random_string(rng, imp.n_flavors, imp.beta, 2 * int(rng.integers(1, 6)), rule)
        got = label_walk(imp, s.op, table)
        assert got == _reachable_start_labels(imp, s.op)
        kept += len(got)
    assert kept >= 20


@pytest.mark.parametrize("rule", ["random", "alternating"])
def test_label_walk_survivors_carry_weight(rule):
    """Survivor direction on the trace itself: in the crystal-field p-shell,
    every label group (N) is one connected component of H_loc, so propagators
    at generic times mix all states of a label and no surviving label can
    cancel.  With the projector P_k inserted at time 0 (it commutes with
    H_loc) the trace sums the start states of label k: exactly zero for every
    label the walk kills, nonzero for every label it keeps."""
    from scipy.sparse.csgraph import connected_components

    from oracle.hamiltonian import hamiltonian_sparse
    from oracle.labels import state_labels
    from oracle.observables import _inserted, label_projectors

    imp = make_impurity("pshell_cf")
    n_comp, _ = connected_components((abs(hamiltonian_sparse(imp.h1, imp.U)) > 0).astype(np.int8), directed=False)
    table = label_table(imp)
    keys = table[0]
    assert n_comp == len(keys)
    dt = DenseTrace(imp)
    ids = np.array([keys.index(tuple(int(v) for v in row)) for row in state_labels(imp)])
    P = label_projectors(dt, ids, len(keys))
    rng = np.random.Generator(np.random.PCG64(29))
    kept = killed = 0
    for _ in range(12):
        s = random_string(rng, imp.n_flavors, imp.beta, 2 * int(rng.integers(1, 5)), rule)
        surv = set(label_walk(imp, s.op, table))
        for k, key in enumerate(keys):
            m, _ = _inserted(dt, s.tau, s.op, 0, 0.0, P[k])
            if key in surv:
                assert m != 0, (s.op, key)
                kept += 1
            else:
                assert m == 0, (s.op, key)
                killed += 1
    assert kept >= 10 and killed >= 10


@pytest.mark.parametrize("name", ["pshell", "pshell_cf", "kanamori2"])
def test_memory_bounded_route_matches_the_plain_route(name, tmp_path):
    """trace_and_scale (operators on disk, creators as adjoints, zero columns
    dropped) against trace() and abs_scale(); random types make many columns
    die along the way."""
    imp = make_impurity(name)
    d0 = DenseTrace(imp)
    d1 = DenseTrace(imp, op_store=str(tmp_path))
    rng = np.random.Generator(np.random.PCG64(5))
    nz = 0
    for i in range(24):
        s = random_string(rng, imp.n_flavors, imp.beta, 2 * int(rng.integers(1, 8)),
                          "random" if i % 2 else "alternating")
        a, b = d0.trace(s.tau, s.op), d0.abs_scale(s.tau, s.op)
        x, y = d1.trace_and_scale(s.tau, s.op)
        if a[0] == 0:
            assert x[0] == 0
            continue
        nz += 1
        assert rel_err(x, a) < 1e-12 and rel_err(y, b) < 1e-12
    assert nz >= 12
