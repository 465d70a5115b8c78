"""Seeded operator strings: the configurations C of the hybridisation
expansion (Sec. 2.2), already time ordered.

A string is (tau, op): times 0 <= tau_0 <= ... < beta and operator codes
op = 2*flavor + dagger (dagger = 1 for a creator).  op[0] at tau[0] acts
first (rightmost in the product).  Every flavor carries as many creators as
annihilators, as in the configurations the Markov chain visits.

Two type rules:
  * "random":      per flavor, the k creators and k annihilators are placed
                   on that flavor's 2k time slots in random order;
  * "alternating": per flavor, creators and annihilators alternate in time
                   with a random first type.  Markov states reached by the
                   Pauli-aware pair moves of App. D have this form (a flavor
                   cannot be created twice in a row).
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .impurity import IMPURITY_SHAPE


@dataclasses.dataclass
class OperatorString:
    tau: np.ndarray  # float64 [n]
    op: np.ndarray   # int32 [n]

    @property
    def n(self) -> int:
        return int(self.op.shape[0])


def random_string(rng: np.random.Generator, n_flavors: int, beta: float, n_ops: int,
                  rule: str = "alternating") -> OperatorString:
    if n_ops % 2:
        raise ValueError("n_ops must be even")
    pairs = rng.multinomial(n_ops // 2, [1.0 / n_flavors] * n_flavors)
    taus, ops = [], []
    for f, k in enumerate(pairs):
        if k == 0:
            continue
        t = np.sort(rng.uniform(0.0, beta, 2 * k))
        if rule == "alternating":
            first = int(rng.integers(2))
            dag = (np.arange(2 * k) + first) % 2
        elif rule == "random":
            dag = rng.permutation(np.array([0] * k + [1] * k))
        else:
            raise ValueError(rule)
        taus.append(t)
        ops.append(2 * f + dag)
    if not taus:
        return OperatorString(np.zeros(0), np.zeros(0, dtype=np.int32))
    tau = np.concatenate(taus)
    op = np.concatenate(ops).astype(np.int32)
    order = np.argsort(tau, kind="stable")
    return OperatorString(tau[order].astype(np.float64), op[order])


@dataclasses.dataclass(frozen=True)
class WorkloadSpec:
    config_id: int
    impurity: str
    n_configs: int
    order_lo: int
    order_hi: int
    rule: str


SPECS = {
    0: WorkloadSpec(0, "kanamori2", 1000, 0, 20, "random"),
    1: WorkloadSpec(1, "dshell", 10_000, 20, 80, "alternating"),
    2: WorkloadSpec(2, "fshell", 10_000, 40, 160, "alternating"),
    3: WorkloadSpec(3, "fshell_cf", 2000, 60, 200, "alternating"),
}


def config_string(config_id: int, i: int, spec: WorkloadSpec | None = None,
                  n_flavors: int | None = None, beta: float | None = None) -> OperatorString:
    """Configuration i of a workload, seeded by PCG64(10^6 * config_id + i)."""
    spec = spec or SPECS[config_id]
    if n_flavors is None or beta is None:
        n_flavors, beta = IMPURITY_SHAPE[spec.impurity]
    rng = np.random.Generator(np.random.PCG64(1_000_000 * config_id + i))
    n = 2 * int(rng.integers(spec.order_lo // 2, spec.order_hi // 2 + 1))
    return random_string(rng, n_flavors, beta, n, spec.rule)


def make_configs(config_id: int, count: int | None = None, start: int = 0,
                 spec: WorkloadSpec | None = None) -> list[OperatorString]:
    spec = spec or SPECS[config_id]
    count = spec.n_configs - start if count is None else count
    n_flavors, beta = IMPURITY_SHAPE[spec.impurity]
    return [config_string(config_id, start + i, spec, n_flavors, beta) for i in range(count)]


def pack(strings: list[OperatorString]):
    """Concatenate strings into CSR form: (offsets int64[n+1], tau f64, op i32)."""
    offs = np.zeros(len(strings) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([s.n for s in strings])
    tau = np.concatenate([s.tau for s in strings]) if strings else np.zeros(0)
    op = np.concatenate([s.op for s in strings]).astype(np.int32) if strings else np.zeros(0, np.int32)
    return offs, np.ascontiguousarray(tau, dtype=np.float64), np.ascontiguousarray(op, dtype=np.int32)


def insert_pair(rng: np.random.Generator, s: OperatorString, n_flavors: int, beta: float) -> OperatorString:
    """Proposal of the Markov chain's pair insertion (App. D): a flavor f and a
    time ta are drawn uniformly, tb uniformly in the stretch from ta to the next
    operator of flavor f (cyclically, wrapping at beta), and the pair goes in
    with the types that keep flavor f alternating: a creator first where f is
    empty at ta, an annihilator first where it is occupied (either, at random,
    where f has no operator yet)."""
    f = int(rng.integers(n_flavors))
    ta = float(rng.uniform(0.0, beta))
    mine = s.tau[(s.op >> 1) == f]
    kinds = s.op[(s.op >> 1) == f] & 1
    if mine.size == 0:
        gap = beta
        occupied = bool(rng.integers(2))
    else:
        after = np.nonzero(mine > ta)[0]
        j = int(after[0]) if after.size else 0
        gap = (mine[j] - ta) if after.size else (mine[0] + beta - ta)
        occupied = kinds[j] == 0  # the next operator of f removes an electron
    tb = ta + float(rng.uniform(0.0, gap))
    if tb >= beta:
        tb -= beta
    first = 2 * f + (0 if occupied else 1)
    second = 2 * f + (1 if occupied else 0)
    tau = np.concatenate([s.tau, [ta, tb]])
    op = np.concatenate([s.op, np.array([first, second], dtype=np.int32)])
    order = np.argsort(tau, kind="stable")
    return OperatorString(tau[order].astype(np.float64), op[order].astype(np.int32))


def remove_pair(rng: np.random.Generator, s: OperatorString, n_flavors: int) -> OperatorString:
    """Proposal of the pair removal (App. D): a flavor with operators is drawn
    uniformly and two of its operators that are neighbours in time (cyclically)
    are removed, which keeps the flavor alternating."""
    flavors = [f for f in range(n_flavors) if np.any((s.op >> 1) == f)]
    if not flavors:
        return s
    f = flavors[int(rng.integers(len(flavors)))]
    idx = np.nonzero((s.op >> 1) == f)[0]
    i = int(rng.integers(idx.size))
    drop = {int(idx[i]), int(idx[(i + 1) % idx.size])}
    keep = np.array([j for j in range(s.n) if j not in drop], dtype=np.int64)
    return OperatorString(s.tau[keep].copy(), s.op[keep].astype(np.int32))
