"""Seeded synthetic impurities: coefficients of the local Hamiltonian.

The local Hamiltonian of Sec. 2.1 (the local-Hamiltonian equation) is

    H_loc = sum_ij c+_i h1_ij c_j + 1/2 sum_ijkl U_ijkl c+_i c+_j c_k c_l ,

with h1 = t - mu*1.  This module draws h1 and U for the impurities the tests
and the benchmark use, plus the abelian charges of every flavor (the quantum
numbers that label sectors, Sec. 3.3.1).  Flavor enumeration follows App. A:
the generic basis lists all spin-down orbitals then all spin-up ones; the
coupled basis lists the j = l - 1/2 multiplet (m_j ascending) and then the
j = l + 1/2 multiplet.

The Kanamori and Slater-Condon forms are named in App. A but not written out;
the forms used here are the standard rotationally invariant ones (Kanamori:
U' = U - 2J with spin-flip and pair-hopping terms; Slater-Condon: Gaunt
coefficients times Slater integrals F^k, rotated to the coupled basis with
Clebsch-Gordan coefficients).
"""

from __future__ import annotations

import dataclasses
import math
from fractions import Fraction

import numpy as np


@dataclasses.dataclass
class Impurity:
    name: str
    n_flavors: int
    beta: float
    h1: np.ndarray          # (n_f, n_f): t - mu*1, Hermitian
    U: np.ndarray           # (n_f,)*4: H_int = 1/2 sum U_ijkl c+_i c+_j c_k c_l
    qn: np.ndarray          # (n_qn, n_f) integer charge of each flavor per quantum number
    qn_names: tuple
    params: dict

    @property
    def is_complex(self) -> bool:
        return bool(np.iscomplexobj(self.h1) or np.iscomplexobj(self.U))

    def u_terms(self, tol: float = 1e-14):
        """Nonzero entries of U as (i, j, k, l, value) arrays."""
        idx = np.nonzero(np.abs(self.U) > tol)
        return idx[0], idx[1], idx[2], idx[3], self.U[idx]


# ----------------------------------------------------------------------------
# angular-momentum algebra (exact rationals; no library dependence)
# ----------------------------------------------------------------------------

def _fact(n: int) -> int:
    return math.factorial(n)


def wigner_3j(j1, j2, j3, m1, m2, m3) -> float:
    """Wigner 3j symbol by the Racah formula.  Arguments may be half-integers
    given as Fractions or floats with .5 parts."""
    j1, j2, j3, m1, m2, m3 = (Fraction(x).limit_denominator(2) for x in (j1, j2, j3, m1, m2, m3))
    if m1 + m2 + m3 != 0:
        return 0.0
    if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return 0.0
    if j3 < abs(j1 - j2) or j3 > j1 + j2:
        return 0.0
    for a in (j1 + j2 - j3, j1 - j2 + j3, -j1 + j2 + j3, j1 + m1, j1 - m1, j2 + m2, j2 - m2, j3 + m3, j3 - m3):
        if a.denominator != 1:
            return 0.0
    t_min = max(0, int(j2 - j3 - m1), int(j1 - j3 + m2))
    t_max = min(int(j1 + j2 - j3), int(j1 - m1), int(j2 + m2))
    tri = Fraction(_fact(int(j1 + j2 - j3)) * _fact(int(j1 - j2 + j3)) * _fact(int(-j1 + j2 + j3)),
                   _fact(int(j1 + j2 + j3 + 1)))
    pre = tri * _fact(int(j1 + m1)) * _fact(int(j1 - m1)) * _fact(int(j2 + m2)) * _fact(int(j2 - m2)) \
        * _fact(int(j3 + m3)) * _fact(int(j3 - m3))
    s = Fraction(0)
    for t in range(t_min, t_max + 1):
        den = (_fact(t) * _fact(int(j3 - j2 + t + m1)) * _fact(int(j3 - j1 + t - m2))
               * _fact(int(j1 + j2 - j3 - t)) * _fact(int(j1 - t - m1)) * _fact(int(j2 - t + m2)))
        s += Fraction((-1) ** t, den)
    phase = (-1) ** int(j1 - j2 - m3)
    return float(phase * s) * math.sqrt(float(pre))


def gaunt_ck(l: int, k: int, m1: int, m2: int) -> float:
    """c^k(l m1; l m2) = sqrt(4 pi / (2k+1)) <l m1| Y_{k, m1-m2} |l m2> (Condon-Shortley)."""
    return ((-1) ** m1) * (2 * l + 1) * wigner_3j(l, k, l, 0, 0, 0) * wigner_3j(l, k, l, -m1, m1 - m2, m2)


def clebsch_gordan(j1, m1, j2, m2, j, m) -> float:
    """<j1 m1; j2 m2 | j m> via the 3j symbol."""
    j1, m1, j2, m2, j, m = (Fraction(x).limit_denominator(2) for x in (j1, m1, j2, m2, j, m))
    phase = (-1) ** int(j1 - j2 + m)
    return phase * math.sqrt(float(2 * j + 1)) * wigner_3j(j1, j2, j, m1, m2, -m)


# ----------------------------------------------------------------------------
# interaction tensors
# ----------------------------------------------------------------------------

def kanamori_U(n_orb: int, U: float, J: float) -> np.ndarray:
    """Rotationally invariant Kanamori tensor in the generic basis
    (flavor f = spin*n_orb + orbital, spin 0 = down, 1 = up), U' = U - 2J:

      U sum_a n_a,up n_a,dn + U' sum_{a!=b} n_a,up n_b,dn + (U'-J) sum_{a<b,s} n_a,s n_b,s
      - J sum_{a!=b} c+_{a,up} c_{a,dn} c+_{b,dn} c_{b,up}
      + J sum_{a!=b} c+_{a,up} c+_{a,dn} c_{b,dn} c_{b,up}
    written as 1/2 sum U_ijkl c+_i c+_j c_k c_l."""
    nf = 2 * n_orb
    T = np.zeros((nf,) * 4)
    Up = U - 2.0 * J

    def f(a, s):
        return s * n_orb + a

    for a in range(n_orb):
        for b in range(n_orb):
            for s in range(2):
                for sp in range(2):
                    i, j = f(a, s), f(b, sp)
                    if i == j:
                        continue
                    # density-density: U_{i j j i} n_i n_j (i != j)
                    if a == b:
                        T[i, j, j, i] += U
                    elif s != sp:
                        T[i, j, j, i] += Up
                    else:
                        T[i, j, j, i] += Up - J
            if a != b:
                up, dn = 1, 0
                # spin flip: -J c+_{a up} c_{a dn} c+_{b dn} c_{b up}
                #          = +J c+_{a up} c+_{b dn} c_{a dn} c_{b up}
                T[f(a, up), f(b, dn), f(a, dn), f(b, up)] += J
                T[f(b, dn), f(a, up), f(b, up), f(a, dn)] += J
                # pair hopping: J c+_{a up} c+_{a dn} c_{b dn} c_{b up}
                T[f(a, up), f(a, dn), f(b, dn), f(b, up)] += J
                T[f(a, dn), f(a, up), f(b, up), f(b, dn)] += J
    return T


def slater_U_product(l: int, F: dict) -> np.ndarray:
    """Slater-Condon tensor in the complex-harmonic product basis |l m s>
    (flavor = s*(2l+1) + m + l, spin down first).  F maps k -> F^k."""
    nm = 2 * l + 1
    ms = list(range(-l, l + 1))
    V = np.zeros((nm,) * 4)  # <m1 m2|V|m3 m4>
    ck = {k: np.array([[gaunt_ck(l, k, a, b) for b in ms] for a in ms]) for k in F}
    for i1, m1 in enumerate(ms):
        for i2, m2 in enumerate(ms):
            for i3, m3 in enumerate(ms):
                for i4, m4 in enumerate(ms):
                    if m1 + m2 != m3 + m4:
                        continue
                    V[i1, i2, i3, i4] = sum(Fk * ck[k][i1, i3] * ck[k][i4, i2] for k, Fk in F.items())
    nf = 2 * nm
    T = np.zeros((nf,) * 4)
    # H = 1/2 sum <m1 m2|V|m3 m4> c+_{m1 s} c+_{m2 s'} c_{m4 s'} c_{m3 s}
    for s in range(2):
        for sp in range(2):
            o, op = s * nm, sp * nm
            # T[i=(m1 s), j=(m2 s'), k=(m4 s'), l=(m3 s)] = V[m1 m2 m3 m4]
            T[o:o + nm, op:op + nm, op:op + nm, o:o + nm] += V.transpose(0, 1, 3, 2)
    return T


def coupled_basis_matrix(l: int) -> tuple[np.ndarray, np.ndarray]:
    """Real orthogonal T with c_{j m_j} = sum_{m s} T[(j m_j), (m s)] c_{m s}.
    Rows enumerate j = l-1/2 (m_j ascending) then j = l+1/2; columns follow
    the product basis.  Also returns 2*m_j of every coupled flavor."""
    nm = 2 * l + 1
    rows, twomj = [], []
    for j2 in (2 * l - 1, 2 * l + 1):
        j = Fraction(j2, 2)
        for mj2 in range(-j2, j2 + 1, 2):
            mj = Fraction(mj2, 2)
            row = np.zeros(2 * nm)
            for s, sz in ((0, Fraction(-1, 2)), (1, Fraction(1, 2))):
                m = mj - sz
                if m.denominator == 1 and abs(m) <= l:
                    row[s * nm + int(m) + l] = clebsch_gordan(l, m, Fraction(1, 2), sz, j, mj)
            rows.append(row)
            twomj.append(mj2)
    return np.array(rows), np.array(twomj, dtype=np.int64)


def rotate_U(U: np.ndarray, T: np.ndarray) -> np.ndarray:
    """U'_{abcd} = sum T_ai T_bj U_ijkl T_ck T_dl for real orthogonal T (c_a = sum_i T_ai c_i)."""
    return np.einsum("ai,bj,ijkl,ck,dl->abcd", T, T, U, T, T, optimize=True)


# ----------------------------------------------------------------------------
# fixed-particle-number spectrum (used only to place mu, R12-style reading)
# ----------------------------------------------------------------------------

def _lowest_energy_at_N(h1: np.ndarray, U: np.ndarray, N: int) -> float:
    """Lowest eigenvalue of H restricted to N particles, built directly on the
    occupation-number basis with the bit-string sign rule.  Used only to place
    the chemical potential of the f-shell impurities."""
    nf = h1.shape[0]
    states = np.array([s for s in range(1 << nf) if bin(s).count("1") == N], dtype=np.int64)
    index = -np.ones(1 << nf, dtype=np.int64)
    index[states] = np.arange(len(states))
    H = np.zeros((len(states), len(states)), dtype=np.result_type(h1, U, float))

    popcount = np.array([bin(x).count("1") for x in range(1 << nf)], dtype=np.int64)

    def popc(x):
        return popcount[x]

    def apply(ops, vals):
        # ops applied right-to-left: list of (flavor, dagger) in left-to-right order
        s = states.copy()
        sign = np.ones(len(s), dtype=np.int64)
        alive = np.ones(len(s), dtype=bool)
        for f, dag in reversed(ops):
            bit = np.int64(1) << f
            occ = (s & bit) != 0
            alive &= (~occ) if dag else occ
            sign *= np.where(popc(s & (bit - 1)) % 2 == 1, -1, 1)
            s = s ^ bit
        rows = index[s[alive]]
        cols = np.nonzero(alive)[0]
        np.add.at(H, (rows, cols), vals * sign[alive])

    for i in range(nf):
        for j in range(nf):
            if h1[i, j] != 0:
                apply([(i, 1), (j, 0)], h1[i, j])
    ii, jj, kk, ll = np.nonzero(np.abs(U) > 1e-14)
    for i, j, k, l_ in zip(ii, jj, kk, ll):
        if len({i, j}) < 2 or len({k, l_}) < 2:
            continue
        apply([(i, 1), (j, 1), (k, 0), (l_, 0)], 0.5 * U[i, j, k, l_])
    return float(np.linalg.eigvalsh(H)[0])


# ----------------------------------------------------------------------------
# the impurities
# ----------------------------------------------------------------------------

def _spin_charges(n_orb: int) -> np.ndarray:
    """(N, 2Sz) charges in the generic basis (down first)."""
    return np.array([[1] * (2 * n_orb), [-1] * n_orb + [1] * n_orb], dtype=np.int64)


def _gauge(h1: np.ndarray, U: np.ndarray, phi: np.ndarray):
    """Express H in the operators d_f = exp(i phi_f) c_f.  Spectrum and the
    trace of any string with as many c_f as c+_f per flavor are unchanged."""
    e = np.exp(1j * phi)
    h1g = h1 * e[:, None] * np.conj(e)[None, :]
    Ug = U * e[:, None, None, None] * e[None, :, None, None] \
        * np.conj(e)[None, None, :, None] * np.conj(e)[None, None, None, :]
    return h1g, Ug


def _kanamori2() -> Impurity:
    U, J = 4.0, 0.5
    mu = 4.75  # (3U - 5J)/2: particle-hole symmetric point of the two-orbital shell
    return Impurity("kanamori2", 4, 10.0, -mu * np.eye(4), kanamori_U(2, U, J), _spin_charges(2),
                    ("N", "2Sz"), dict(U=U, J=J, mu=mu))


def _hubbard_atom() -> Impurity:
    # Sec. 4.1 impurity: U = 4, eps_f = -U/2, beta = 10 (no bath needed for the trace)
    U = 4.0
    T = np.zeros((2,) * 4)
    T[0, 1, 1, 0] = T[1, 0, 0, 1] = U
    return Impurity("hubbard_atom", 2, 10.0, -U / 2 * np.eye(2), T, _spin_charges(1), ("N", "2Sz"),
                    dict(U=U, eps_f=-U / 2))


def _dshell(seed: int = 1001) -> Impurity:
    rng = np.random.Generator(np.random.PCG64(seed))
    U = float(rng.uniform(3.0, 6.0))
    J = float(rng.uniform(0.5, 1.0))
    cf = rng.normal(0.0, 0.2, size=5)
    mu = 4.5 * U - 10.0 * J
    h1 = np.diag(np.concatenate([cf, cf]) - mu)
    return Impurity("dshell", 10, 50.0, h1, kanamori_U(5, U, J), _spin_charges(5), ("N", "2Sz"),
                    dict(U=U, J=J, cf=cf.tolist(), mu=mu))


_F_RATIOS = (0.668, 0.494)  # F4/F2, F6/F2 "atomic ratios"


def _slater_F(F0: float, Jh: float, l: int = 3) -> dict:
    if l == 3:
        r4, r6 = _F_RATIOS
        F2 = 6435.0 * Jh / (286.0 + 195.0 * r4 + 250.0 * r6)
        return {0: F0, 2: F2, 4: r4 * F2, 6: r6 * F2}
    if l == 2:
        F2 = 14.0 * Jh / (1.0 + 0.625)
        return {0: F0, 2: F2, 4: 0.625 * F2}
    if l == 1:
        return {0: F0, 2: 5.0 * Jh}
    raise ValueError(l)


def shell_coupled(l: int, F: dict, xi: float) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(h1 without mu, U, 2m_j) for an l-shell in the coupled basis with
    spin-orbit coupling xi l.s (diagonal there) and Slater-Condon U."""
    T, twomj = coupled_basis_matrix(l)
    U = rotate_U(slater_U_product(l, F), T)
    nj_lo = 2 * l  # size of the j = l - 1/2 multiplet
    ls = np.array([-(l + 1) / 2.0] * nj_lo + [l / 2.0] * (2 * l + 2))
    return np.diag(xi * ls), U, twomj


def _shell(seed: int, l: int, beta: float, name: str, n0: int, cf_sigma: float = 0.0,
           cf_seed: int | None = None, gauge: bool = True, jz: bool = True) -> Impurity:
    rng = np.random.Generator(np.random.PCG64(seed))
    F0 = float(rng.uniform(4.0, 6.0))
    xi = float(rng.uniform(0.2, 0.4))
    Jh = 0.512
    F = _slater_F(F0, Jh, l)
    h1, U, twomj = shell_coupled(l, F, xi)
    nf = h1.shape[0]
    # mu: midpoint of the (n0-1 -> n0) and (n0 -> n0+1) addition energies
    e = {N: _lowest_energy_at_N(h1, U, N) for N in (n0 - 1, n0, n0 + 1)}
    mu = 0.5 * ((e[n0] - e[n0 - 1]) + (e[n0 + 1] - e[n0]))
    h1 = h1 - mu * np.eye(nf)
    phi = rng.uniform(0.0, 2 * np.pi, size=nf)
    if gauge:
        h1, U = _gauge(h1.astype(complex), U.astype(complex), phi)
    params = dict(F=F, xi=xi, mu=mu, Jh=Jh, phi=phi.tolist() if gauge else None)
    if cf_sigma > 0:
        crng = np.random.Generator(np.random.PCG64(cf_seed))
        A = crng.normal(0, cf_sigma, (nf, nf)) + 1j * crng.normal(0, cf_sigma, (nf, nf))
        h1 = h1 + 0.5 * (A + A.conj().T)
        params["cf_sigma"] = cf_sigma
    if jz and cf_sigma == 0:
        qn = np.array([[1] * nf, twomj], dtype=np.int64)
        names = ("N", "2Jz")
    else:
        qn = np.array([[1] * nf], dtype=np.int64)
        names = ("N",)
    return Impurity(name, nf, beta, h1, U, qn, names, params)


def _density_density(name: str, n_orb_shell: int, beta: float, seed: int, sectors: str,
                     spin_coupled: bool) -> Impurity:
    """Impurity whose H is diagonal in the occupation-number basis:
    H = sum_f eps_f n_f + 1/2 sum_{i!=j} V_ij n_i n_j.  Charges: N plus 2Sz
    (generic basis) or 2Jz (coupled basis), or N only."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nf = 2 * n_orb_shell
    V = rng.uniform(3.0, 5.0) + rng.normal(0, 0.3, (nf, nf))
    V = 0.5 * (V + V.T)
    np.fill_diagonal(V, 0.0)
    n0 = nf // 2 - (1 if nf == 14 else 0)
    eps = rng.normal(0, 0.3, nf) - V.sum() / nf * (n0 - 0.5) / (nf - 1)
    U = np.zeros((nf,) * 4)
    for i in range(nf):
        for j in range(nf):
            if i != j:
                U[i, j, j, i] = V[i, j]
    if spin_coupled:
        l = (nf // 2 - 1) // 2
        _, twomj = coupled_basis_matrix(l)
        second, second_name = twomj, "2Jz"
    else:
        second, second_name = np.array([-1] * (nf // 2) + [1] * (nf // 2)), "2Sz"
    if sectors == "N":
        qn, names = np.array([[1] * nf], dtype=np.int64), ("N",)
    else:
        qn, names = np.array([[1] * nf, second], dtype=np.int64), ("N", second_name)
    return Impurity(name, nf, beta, np.diag(eps), U, qn, names, dict(V=V.tolist(), eps=eps.tolist()))


_CACHE: dict = {}

# (number of flavors, beta) of every impurity, available without building it
IMPURITY_SHAPE = {
    "kanamori2": (4, 10.0), "dshell": (10, 50.0), "fshell": (14, 40.0), "fshell_cf": (14, 40.0),
    "fshell_real": (14, 40.0), "hubbard_atom": (2, 10.0), "pshell": (6, 20.0), "pshell_cf": (6, 20.0), "pshell_real": (6, 20.0),
    "dshell_so": (10, 30.0), "dd_dshell": (10, 50.0), "dd_fshell": (14, 40.0), "dd_fshell_n": (14, 40.0),
}

IMPURITY_NAMES = (
    "kanamori2",      # 2-orbital Kanamori atom, 16 states, (N, Sz) sectors, beta 10
    "dshell",         # 5-orbital Kanamori + spin-flip + pair hopping, 1024 states, (N, Sz), beta 50
    "fshell",         # 7-orbital Slater-Condon + SOC, gauge-complex, 16384 states, (N, Jz), beta 40
    "fshell_cf",      # fshell + random Hermitian crystal field, N-only sectors
    "fshell_real",    # fshell without the gauge phases (same spectrum, real H)
    "hubbard_atom",   # single-band atom of Sec. 4.1
    "pshell",         # 3-orbital Slater-Condon + SOC, gauge-complex, 64 states, (N, Jz)
    "pshell_cf",      # pshell + crystal field, N-only sectors
    "pshell_real",    # pshell without the gauge phases
    "dshell_so",      # 5-orbital Slater-Condon + SOC, gauge-complex, 1024 states, (N, Jz)
    "dd_dshell",      # density-density, 10 flavors, (N, Sz)
    "dd_fshell",      # density-density, 14 flavors, (N, Jz)
    "dd_fshell_n",    # same H, N-only sectors
)


def make_impurity(name: str) -> Impurity:
    """Deterministic (seeded) impurity by name; cached per process."""
    if name in _CACHE:
        return _CACHE[name]
    if name == "kanamori2":
        imp = _kanamori2()
    elif name == "hubbard_atom":
        imp = _hubbard_atom()
    elif name == "dshell":
        imp = _dshell()
    elif name == "fshell":
        imp = _shell(1002, 3, 40.0, "fshell", 5)
    elif name == "fshell_real":
        imp = _shell(1002, 3, 40.0, "fshell_real", 5, gauge=False)
    elif name == "fshell_cf":
        imp = _shell(1002, 3, 40.0, "fshell_cf", 5, cf_sigma=0.05, cf_seed=1003)
    elif name == "pshell":
        imp = _shell(1010, 1, 20.0, "pshell", 3)
    elif name == "pshell_real":
        imp = _shell(1010, 1, 20.0, "pshell_real", 3, gauge=False)
    elif name == "pshell_cf":
        imp = _shell(1010, 1, 20.0, "pshell_cf", 3, cf_sigma=0.05, cf_seed=1011)
    elif name == "dshell_so":
        imp = _shell(1012, 2, 30.0, "dshell_so", 5)
    elif name == "dd_dshell":
        imp = _density_density("dd_dshell", 5, 50.0, 1020, "NS", False)
    elif name == "dd_fshell":
        imp = _density_density("dd_fshell", 7, 40.0, 1021, "NJ", True)
    elif name == "dd_fshell_n":
        imp = _density_density("dd_fshell_n", 7, 40.0, 1021, "N", True)
        imp.name = "dd_fshell_n"
    else:
        raise KeyError(f"unknown impurity {name!r}; known: {IMPURITY_NAMES}")
    _CACHE[name] = imp
    return imp


# Discrete bath per flavor for the Markov step (Sec. 2.2 w_hyb): n_bath levels
# spread over [-2, 2] with a seeded jitter, amplitudes around 0.4; every flavor
# of an impurity gets its own draw.  Coefficients only; the hybridisation
# function built from them lives with its users.
BATH_LEVELS = {"kanamori2": 2, "pshell": 2, "pshell_cf": 2, "dshell": 3, "dshell_so": 3, "fshell": 3,
               "fshell_cf": 3}


def synthetic_bath(name: str, seed: int = 2024):
    """(eps, v), each [n_flavors, n_bath] float64."""
    nf, _ = IMPURITY_SHAPE[name]
    nb = BATH_LEVELS.get(name, 2)
    rng = np.random.Generator(np.random.PCG64([seed, sum(map(ord, name))]))
    base = np.linspace(-2.0, 2.0, nb) if nb > 1 else np.zeros(1)
    eps = base[None, :] + rng.normal(0.0, 0.15, (nf, nb))
    v = 0.4 + rng.normal(0.0, 0.05, (nf, nb))
    return eps, v
