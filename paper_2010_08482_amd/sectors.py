"""Host setup of the sector decomposition (Sec. 3.3.1) that the trace
library consumes.

The Hilbert space splits into sectors of fixed abelian charges (N, 2Sz or
2Jz, ...).  Per sector q this module builds H_loc restricted to q on the
occupation-number basis, diagonalises it (LAPACK), and expresses every
annihilator c_f as a dense block F_f(q) : H(q) -> H(s_f(q)) in the
eigenbases of the two sectors, element [m][n] = <m(s_f(q))| c_f |n(q)>.
The sector map s_alpha(q) becomes the integer table next[q][op] with op =
2*flavor + dagger and -1 for the zero sector.

This is input preparation, run once per impurity (the paper's
initialisation phase, Sec. 3.1); the trace itself runs on the GPU.
Occupation states are integers with bit f = occupation of flavor f; the sign
of c_f on |s> is (-1)^popcount(s & (2^f - 1)).
"""

from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


@dataclasses.dataclass
class SectorTable:
    n_flavors: int
    beta: float
    is_complex: bool
    qn_names: tuple
    labels: np.ndarray            # [n_sec, n_qn] int64, sorted lexicographically
    dims: np.ndarray              # [n_sec] int32
    energies: list                # per sector: eigenvalues (float64), grouped by invariant part of H
    next: np.ndarray              # [n_sec, 2*n_f] int32, -1 = zero sector
    blocks: list                  # [n_sec][n_f]: annihilator block d(next[q][2f]) x d(q) or None
    states: list                  # per sector: occupation states (int64) in basis order
    vectors: list | None = None   # per sector: eigenvectors (columns) on `states`, if kept

    @property
    def n_sectors(self) -> int:
        return int(self.dims.shape[0])

    @property
    def max_dim(self) -> int:
        return int(self.dims.max())

    def sector_of_label(self) -> dict:
        return {tuple(int(v) for v in row): q for q, row in enumerate(self.labels)}

    def e0(self) -> float:
        return float(min(float(np.min(e)) for e in self.energies))


def _popcount_table(nf: int) -> np.ndarray:
    t = np.zeros(1 << nf, dtype=np.int64)
    for b in range(nf):
        t += (np.arange(1 << nf) >> b) & 1
    return t


def _apply(states, ops, pc):
    """Apply a product of operators (given left to right as (flavor, dagger))
    to every state; returns (target states, signs, alive mask)."""
    s = states.copy()
    sign = np.ones(s.shape[0], dtype=np.int64)
    alive = np.ones(s.shape[0], dtype=bool)
    for f, dag in reversed(ops):
        bit = np.int64(1) << np.int64(f)
        occ = (s & bit) != 0
        alive &= ~occ if dag else occ
        sign = np.where(pc[s & (bit - 1)] & 1, -sign, sign)
        s = s ^ bit
    return s, sign, alive


def _hamiltonian_coo(h1, U, nf, pc):
    D = 1 << nf
    states = np.arange(D, dtype=np.int64)
    rows, cols, vals = [], [], []
    dtype = np.result_type(h1, U, np.float64)

    def add(ops, v):
        t, sg, al = _apply(states, ops, pc)
        rows.append(t[al])
        cols.append(states[al])
        vals.append((v * sg[al]).astype(dtype))

    for i in range(nf):
        for j in range(nf):
            if h1[i, j] != 0:
                add([(i, 1), (j, 0)], h1[i, j])
    nz = np.argwhere(np.abs(U) > 1e-14)
    for i, j, k, l in nz:
        if i == j or k == l:
            continue
        add([(i, 1), (j, 1), (k, 0), (l, 0)], 0.5 * U[i, j, k, l])
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def _eigh_invariant_parts(Hq: np.ndarray):
    """Eigenpairs of one sector block, computed separately on every connected
    component of the block's nonzero pattern and assembled part after part
    (parts in the order of their lowest occupation state, energies ascending
    inside each part).

    H_loc often conserves more than the charges that label sectors (the
    Kanamori form, for instance, keeps the set of singly occupied orbitals).
    A dense eigensolver run on the whole block leaves rounding-level weight
    of every eigenvector in the other invariant parts; operator blocks then
    carry ~1e-16 entries where the exact ones vanish, and at low temperature
    the propagators can amplify such a forbidden path by far more than
    1e16.  Solving each invariant part on its own keeps those entries exactly
    zero.  Keeping the eigenvectors of one part together keeps those zeros in
    contiguous ranges of the operator blocks, so whole 16 x 4 tiles of the
    MFMA products vanish and the kernels skip them (on the Kanamori d-shell
    70% of the tiles of the large blocks)."""
    d = Hq.shape[0]
    n_comp, comp = connected_components(sp.csr_matrix(Hq != 0), directed=False)
    if n_comp == 1:
        return np.linalg.eigh(Hq)
    E = np.zeros(d)
    V = np.zeros((d, d), dtype=Hq.dtype)
    pos = 0
    for k in range(n_comp):
        idx = np.nonzero(comp == k)[0]
        e, v = np.linalg.eigh(Hq[np.ix_(idx, idx)])
        E[pos:pos + idx.size] = e
        V[idx, pos:pos + idx.size] = v
        pos += idx.size
    return E, V


def build_sectors(imp, phase_seed: int | None = None, force_complex: bool = False,
                  keep_vectors: bool = False) -> SectorTable:
    """Sector table of an impurity (anything with n_flavors, beta, h1, U, qn).

    phase_seed: multiply every eigenvector by a random phase.  Eigenvectors
    are only defined up to such phases (and up to rotations inside
    degenerate levels); traces do not depend on the choice, but the blocks
    become genuinely complex, which exercises the complex kernels even when
    H_loc is real.  keep_vectors: keep every sector's eigenvectors in the
    table (to express sector-basis results on occupation states)."""
    nf = int(imp.n_flavors)
    D = 1 << nf
    h1 = np.asarray(imp.h1)
    U = np.asarray(imp.U)
    qn = np.asarray(imp.qn, dtype=np.int64)
    pc = _popcount_table(nf)
    states = np.arange(D, dtype=np.int64)
    occ = (states[:, None] >> np.arange(nf)[None, :]) & 1
    lab = occ @ qn.T                                           # [D, n_qn]
    keys, inv = np.unique(lab, axis=0, return_inverse=True)    # lexicographic
    inv = inv.reshape(-1)
    n_sec = keys.shape[0]
    sec_states = [np.nonzero(inv == q)[0].astype(np.int64) for q in range(n_sec)]
    local = np.zeros(D, dtype=np.int64)
    for q, st in enumerate(sec_states):
        local[st] = np.arange(st.shape[0])

    r, c, v = _hamiltonian_coo(h1, U, nf, pc)
    if np.any(inv[r] != inv[c]):
        raise ValueError("H_loc mixes sectors: the chosen charges are not conserved")
    cplx = bool(np.iscomplexobj(v) and np.any(np.imag(v) != 0)) or force_complex or phase_seed is not None
    dtype = np.complex128 if cplx else np.float64
    order = np.argsort(inv[c], kind="stable")
    r, c, v = r[order], c[order], v[order]
    bounds = np.searchsorted(inv[c], np.arange(n_sec + 1))

    rng = np.random.Generator(np.random.PCG64(phase_seed)) if phase_seed is not None else None
    energies, vecs = [], []
    for q in range(n_sec):
        d = sec_states[q].shape[0]
        Hq = np.zeros((d, d), dtype=dtype)
        a, b = bounds[q], bounds[q + 1]
        np.add.at(Hq, (local[r[a:b]], local[c[a:b]]), v[a:b].astype(dtype) if cplx else np.real(v[a:b]))
        if not np.allclose(Hq, Hq.conj().T, atol=1e-12):
            raise ValueError(f"sector {q}: H_loc block is not Hermitian")
        E, V = _eigh_invariant_parts(Hq)
        if rng is not None:
            V = V * np.exp(1j * rng.uniform(0, 2 * np.pi, d))[None, :]
        energies.append(E.astype(np.float64))
        vecs.append(V.astype(dtype))

    nxt = -np.ones((n_sec, 2 * nf), dtype=np.int32)
    blocks = [[None] * nf for _ in range(n_sec)]
    for q in range(n_sec):
        st = sec_states[q]
        for f in range(nf):
            bit = np.int64(1) << np.int64(f)
            has = (st & bit) != 0
            if np.any(~has):
                nxt[q, 2 * f + 1] = inv[st[~has][0] | bit]
            if not np.any(has):
                continue
            tgt = inv[st[has][0] ^ bit]
            nxt[q, 2 * f] = tgt
            src = st[has]
            sign = np.where(pc[src & (bit - 1)] & 1, -1.0, 1.0)
            CV = np.zeros((sec_states[tgt].shape[0], st.shape[0]), dtype=dtype)
            CV[local[src ^ bit]] = sign[:, None] * vecs[q][local[src]]
            blocks[q][f] = np.ascontiguousarray(vecs[tgt].conj().T @ CV)
    return SectorTable(nf, float(imp.beta), cplx, tuple(getattr(imp, "qn_names", ())), keys,
                       np.array([s.shape[0] for s in sec_states], dtype=np.int32), energies, nxt, blocks,
                       sec_states, vecs if keep_vectors else None)
