"""Writes the stored expected values of the GPU parity tests.

Calls only the CPU oracle (oracle/) and the seeded input generators
(workloads/).  Each record: configuration index (or seed), operator count,
oracle trace as (mantissa re, im, log_scale) and the cancellation scale A
(sum of moduli of the Lehmann terms, same log units).

    python tests/golden/make_golden.py [name ...]
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import DenseTrace  # noqa: E402
from workloads import make_configs, make_impurity  # noqa: E402
from workloads.configs import random_string  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def record(dt, idx, s):
    m, l = dt.trace(s.tau, s.op)
    a, la = dt.abs_scale(s.tau, s.op)
    m = complex(m)
    return {"i": int(idx), "n": int(s.n), "re": m.real, "im": m.imag, "log_scale": l, "abs": a, "abs_log": la}


def config_set(name, impurity, config_id, count):
    imp = make_impurity(impurity)
    dt = DenseTrace(imp)
    out = []
    t0 = time.time()
    for i, s in enumerate(make_configs(config_id, count)):
        out.append(record(dt, i, s))
        if (i + 1) % 25 == 0:
            print(f"{name}: {i + 1}/{count} ({time.time() - t0:.0f}s)", flush=True)
    return {"impurity": impurity, "config_id": config_id, "records": out}


def random_set(name, impurity, seed, count, lo, hi):
    imp = make_impurity(impurity)
    dt = DenseTrace(imp)
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n = 2 * int(rng.integers(lo // 2, hi // 2 + 1))
        s = random_string(rng, imp.n_flavors, imp.beta, n, "alternating")
        r = record(dt, i, s)
        r["tau"] = s.tau.tolist()
        r["op"] = s.op.tolist()
        out.append(r)
    print(f"{name}: {count} done", flush=True)
    return {"impurity": impurity, "seed": seed, "records": out}


def low_order_set(name, impurity, seed, orders):
    """Full-size impurities (16384 states): a few strings of low order, the
    most the dense oracle affords (each operator costs a 16384^3 product).
    The operator matrices are dropped after each string to bound memory."""
    imp = make_impurity(impurity)
    t0 = time.time()
    dt = DenseTrace(imp)
    print(f"{name}: eigenbasis in {time.time() - t0:.0f}s", flush=True)
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i, n in enumerate(orders):
        s = random_string(rng, imp.n_flavors, imp.beta, n, "alternating")
        r = record(dt, i, s)
        r["tau"] = s.tau.tolist()
        r["op"] = s.op.tolist()
        out.append(r)
        dt._ops.clear()
        print(f"{name}: string {i + 1}/{len(orders)} (order {n}) {time.time() - t0:.0f}s", flush=True)
    return {"impurity": impurity, "seed": seed, "records": out}


def workload_set(name, impurity, config_id, indices, store):
    """Workload strings of a full-size impurity at production order, through
    the oracle's memory-bounded route (operator matrices on disk under
    `store`, zero columns dropped).  The file is rewritten after every string."""
    imp = make_impurity(impurity)
    t0 = time.time()
    # strings already in the file (from an earlier run of this set) are kept, not recomputed
    path = os.path.join(HERE, name + ".json")
    done = {}
    if os.path.exists(path):
        with open(path) as fh:
            old = json.load(fh)
        if old.get("impurity") == impurity and old.get("config_id") == config_id:
            done = {int(r["i"]): r for r in old["records"]}
    os.makedirs(store, exist_ok=True)
    dt = DenseTrace(imp, op_store=store)
    print(f"{name}: eigenbasis in {time.time() - t0:.0f}s", flush=True)
    cfgs = make_configs(config_id, max(indices) + 1)
    out = []
    for i in indices:
        if i in done:
            out.append(done[i])
            continue
        s = cfgs[i]
        (m, l), (a, la) = dt.trace_and_scale(s.tau, s.op)
        m = complex(m)
        out.append({"i": int(i), "n": int(s.n), "re": m.real, "im": m.imag, "log_scale": l, "abs": a,
                    "abs_log": la, "tau": s.tau.tolist(), "op": s.op.tolist()})
        with open(os.path.join(HERE, name + ".json"), "w") as fh:
            json.dump({"impurity": impurity, "config_id": config_id, "records": out}, fh, indent=0)
        print(f"{name}: configuration {i} (order {s.n}) {time.time() - t0:.0f}s", flush=True)
    return {"impurity": impurity, "config_id": config_id, "records": out}


SETS = {
    # d-shell workload strings (the benchmark's configurations), first 256
    "dshell_config1": lambda: config_set("dshell_config1", "dshell", 1, 256),
    # complex impurities small enough for the dense oracle
    "pshell_random": lambda: random_set("pshell_random", "pshell", 77, 120, 2, 60),
    "pshell_cf_random": lambda: random_set("pshell_cf_random", "pshell_cf", 78, 120, 2, 60),
    "dshell_so_random": lambda: random_set("dshell_so_random", "dshell_so", 79, 80, 2, 80),
    # the generic f-shell impurities of the (N, Jz) and crystal-field workloads at full size
    "fshell_low": lambda: low_order_set("fshell_low", "fshell", 81, [2, 2, 2, 4]),
    "fshell_cf_low": lambda: low_order_set("fshell_cf_low", "fshell_cf", 82, [2, 2, 4]),
    # production-order workload strings of the f-shell (N, Jz) benchmark (orders 44, 40 and 42; the three
    # cheapest for the dense oracle among its first 400 configurations of order <= 44)
    "fshell_workload": lambda: workload_set("fshell_workload", "fshell", 2, [93, 391, 16],
                                            os.environ.get("ORACLE_OP_STORE", "/tmp/oracle_ops_fshell")),
    # production-order strings of the crystal-field f-shell benchmark (order 60, its lowest; the two
    # cheapest for the dense oracle among the 26 of order 60 in its 2000 configurations)
    "fshell_cf_workload": lambda: workload_set("fshell_cf_workload", "fshell_cf", 3, [480, 1667],
                                               os.environ.get("ORACLE_OP_STORE", "/tmp/oracle_ops_fshell_cf")),
}

if __name__ == "__main__":
    names = sys.argv[1:] or list(SETS)
    for name in names:
        data = SETS[name]()
        with open(os.path.join(HERE, name + ".json"), "w") as fh:
            json.dump(data, fh, indent=0)
        print("wrote", name, flush=True)
