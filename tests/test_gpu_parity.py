"""GPU parity of the trace library against the CPU oracle, through the C ABI.

Every comparison uses the parity bar of tests/tracecmp.close_enough:
|gpu - oracle| <= 1e-10 |oracle|, or, for cancellation-dominated traces,
<= 1e-12 A with A the sum of moduli of the Lehmann terms.
"""

import json
import math
import os

import numpy as np
import pytest

from tests.tracecmp import close_enough, rel_err
from workloads import make_configs, make_impurity
from workloads.configs import OperatorString, pack, random_string

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_08482_amd import ctrace

    return ctrace


@pytest.fixture(scope="module")
def ctx(lib):
    from paper_2010_08482_amd.sectors import build_sectors

    cache = {}

    def get(name, phase_seed=None, arena_bytes=None):
        key = (name, phase_seed, arena_bytes)
        if key not in cache:
            say(f"[setup] sectors + ctr_set_impurity: {name} phase_seed={phase_seed} arena={arena_bytes}")
            tab = build_sectors(make_impurity(name), phase_seed=phase_seed)
            cache[key] = (tab, lib.TraceContext(tab, arena_bytes=arena_bytes))
        return cache[key]

    yield get
    for _, c in cache.values():
        c.close()


HIST_KERNELS = {"wave": 1, "block": 2, "stream": 3, "grouped": 4, "grouped_rows": 5}


def pair(v):
    m = complex(v["re"], v["im"])
    return (m if m.imag != 0 else m.real), float(v["log_scale"])


def load_golden(name):
    with open(os.path.join(HERE, "golden", name + ".json")) as fh:
        return json.load(fh)


def golden_pair(r):
    return complex(r["re"], r["im"]), r["log_scale"]


def check_against(out, refs, scales, label):
    bad = []
    worst = 0.0
    for i, (v, ref, sc) in enumerate(zip(out, refs, scales)):
        got = pair(v)
        if ref[0] == 0:
            assert got[0] == 0 or (v["flags"] & 1), f"{label} #{i}: oracle zero, gpu {got}"
            continue
        if not close_enough(got, ref, sc):
            bad.append((i, rel_err(got, ref)))
        worst = max(worst, rel_err(got, ref))
    say(f"{label}: {len(out)} traces, worst rel err {worst:.2e}, failures {bad[:5]}")
    assert not bad


def agree(a, b, label, rtol=1e-10, atol_scale=1e-12):
    """Two GPU evaluations of the same batch against each other at the R14 bar:
    |a - b| <= rtol |b|, or <= atol_scale exp(log_abs) for cancellation-
    dominated traces (log_abs: the sum of moduli of the evaluated
    contributions, never above the oracle's Lehmann modulus sum)."""
    assert np.array_equal(a["flags"], b["flags"]) and np.array_equal(a["n_strings"], b["n_strings"]), label
    worst = 0.0
    cancel = 0
    for x, y in zip(a, b):
        if y["re"] == 0 and y["im"] == 0:
            assert x["re"] == 0 and x["im"] == 0, label
            continue
        scale = (1.0, max(float(x["log_abs"]), float(y["log_abs"])))
        assert close_enough(pair(x), pair(y), scale, rtol, atol_scale), (label, rel_err(pair(x), pair(y)))
        r = rel_err(pair(x), pair(y))
        worst = max(worst, r)
        cancel += r > rtol
    say(f"{label}: worst rel {worst:.2e}, {cancel} cancellation-dominated")
    return worst


# ---------------------------------------------------------------------------
# order zero and the 16-state atom
# ---------------------------------------------------------------------------

def test_partition_function_closed_form(ctx):
    tab, c = ctx("kanamori2")
    say("[gpu] ctr_trace n=0 kanamori2")
    v = c.trace([], [])
    b = 10.0
    z = (2 * math.exp(-7 * b) + 8 * math.exp(-2.25 * b) + 3 + 2 * math.exp(-b) + math.exp(-2 * b)), 7 * b
    assert rel_err(pair(v), z) < 1e-13
    assert v["n_strings"] == tab.n_sectors


def test_config0_all_1000_vs_oracle(ctx):
    from oracle import DenseTrace

    tab, c = ctx("kanamori2")
    imp = make_impurity("kanamori2")
    dt = DenseTrace(imp)
    cfgs = make_configs(0)
    say("[gpu] ctr_trace_batch config0 x1000")
    out = c.trace_batch(cfgs)
    refs = [dt.trace(s.tau, s.op) for s in cfgs]
    scales = [dt.abs_scale(s.tau, s.op) for s in cfgs]
    check_against(out, refs, scales, "config0")
    # the zero-string set: no survivor <=> CTR_FLAG_ZERO
    for v, s in zip(out, cfgs):
        assert bool(v["flags"] & 1) == (v["n_strings"] == 0)


def _label_walk_check(ctx, name, cfgs):
    from oracle.labels import label_table, label_walk

    tab, c = ctx(name)
    imp = make_impurity(name)
    table = label_table(imp)
    labels = [tuple(int(x) for x in row) for row in tab.labels]
    for i, s in enumerate(cfgs):
        got = sorted(labels[q] for q in c.strings(s.op))
        want = sorted(label_walk(imp, s.op, table))
        assert got == want, f"{name} #{i}"


def test_strings_match_oracle_label_walk_config0(ctx):
    say("[gpu] ctr_strings config0 x1000")
    _label_walk_check(ctx, "kanamori2", make_configs(0))


def test_strings_match_oracle_label_walk_config1(ctx):
    say("[gpu] ctr_strings config1 x150")
    _label_walk_check(ctx, "dshell", make_configs(1, 150))


# ---------------------------------------------------------------------------
# d-shell workload at full size (the benchmark's batch and launch path)
# ---------------------------------------------------------------------------

def _device_batch(lib, c, strings):
    import torch

    offs, tau, op = pack(strings)
    dev = f"cuda:{c.device}"
    d_offs = torch.from_numpy(offs).to(dev)
    d_tau = torch.from_numpy(tau).to(dev)
    d_op = torch.from_numpy(op).to(dev)
    d_out = torch.zeros(len(strings) * lib.VALUE_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    lib.ctr_trace_batch_device(c.ctx, len(strings), d_offs.data_ptr(), d_tau.data_ptr(), d_op.data_ptr(),
                               d_out.data_ptr())
    c.synchronize()
    return np.frombuffer(d_out.cpu().numpy().tobytes(), dtype=lib.VALUE_DTYPE)


def test_config1_full_batch_device_path_vs_golden(lib, ctx):
    tab, c = ctx("dshell")
    g = load_golden("dshell_config1")
    cfgs = make_configs(1)
    assert len(cfgs) == 10_000
    say("[gpu] ctr_trace_batch_device config1 x10000")
    out = _device_batch(lib, c, cfgs)
    k = len(g["records"])
    check_against(out[:k], [golden_pair(r) for r in g["records"]],
                  [(r["abs"], r["abs_log"]) for r in g["records"]], "config1 golden (full-size batch)")
    assert np.all(np.isfinite(out["re"])) and np.all(np.isfinite(out["log_scale"]))
    assert not np.any(out["flags"] & 4)
    # every value is below its own lazy bound
    la = np.array([math.log(math.hypot(v["re"], v["im"])) + v["log_scale"] if (v["re"] or v["im"]) else -np.inf
                   for v in out])
    assert np.all(la <= out["log_bound"] + 1e-9)
    # the host-pointer path agrees bit for bit
    say("[gpu] ctr_trace_batch config1 x300 host path")
    host = c.trace_batch(cfgs[:300])
    assert np.array_equal(host["re"], out["re"][:300]) and np.array_equal(host["log_scale"], out["log_scale"][:300])


def test_cancellation_scale_between_trace_and_lehmann_sum(lib, ctx):
    """log_abs (sum of the moduli of the evaluated contributions) lies between
    log|trace| and the oracle's sum of moduli of all Lehmann terms."""
    g = load_golden("dshell_config1")
    tab, c = ctx("dshell")
    recs = g["records"]
    cfgs = make_configs(1, len(recs))
    say("[gpu] cancellation scale dshell x256")
    for kernel in (lib.CTR_KERNEL_WAVE, lib.CTR_KERNEL_GROUPED):
        out = c.trace_batch(cfgs, kernel=kernel)
        n_checked = 0
        for v, r in zip(out, recs):
            if v["re"] == 0 and v["im"] == 0:
                assert v["log_abs"] == -np.inf
                continue
            la = lib.log_abs(v)
            assert la <= v["log_abs"] + 1e-9
            A = math.log(r["abs"]) + r["abs_log"] if r["abs"] > 0 else -np.inf
            assert v["log_abs"] <= A + 1e-9
            n_checked += 1
        assert n_checked > 100


@pytest.mark.parametrize("name", ["pshell_random", "pshell_cf_random", "dshell_so_random"])
def test_complex_impurities_vs_golden(ctx, name):
    g = load_golden(name)
    tab, c = ctx(g["impurity"])
    assert tab.is_complex
    strings = [(np.array(r["tau"]), np.array(r["op"], dtype=np.int32)) for r in g["records"]]
    say(f"[gpu] ctr_trace_batch {name} x{len(strings)}")
    out = c.trace_batch(strings)
    check_against(out, [golden_pair(r) for r in g["records"]], [(r["abs"], r["abs_log"]) for r in g["records"]],
                  name)


@pytest.mark.parametrize("name,kernels", [("fshell_low", ("block", "stream", "grouped", "grouped_rows")),
                                          ("fshell_cf_low", ("stream", "grouped"))])
def test_generic_fshell_low_orders_vs_golden(lib, ctx, name, kernels):
    """The generic 16384-state f-shell impurities against the dense oracle at
    the few low orders it affords (stored values), every kernel that runs them."""
    path = os.path.join(HERE, "golden", name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"{name}.json not generated")
    g = load_golden(name)
    tab, c = ctx(g["impurity"])
    strings = [(np.array(r["tau"]), np.array(r["op"], dtype=np.int32)) for r in g["records"]]
    for k in kernels:
        say(f"[gpu] ctr_trace_batch {name} x{len(strings)} kernel={k}")
        out = c.trace_batch(strings, kernel=HIST_KERNELS[k])
        check_against(out, [golden_pair(r) for r in g["records"]],
                      [(r["abs"], r["abs_log"]) for r in g["records"]], f"{name}/{k}")


@pytest.mark.parametrize("name,config_id,kernels",
                         [("fshell_workload", 2, ("block", "stream", "grouped", "grouped_rows")),
                          ("fshell_cf_workload", 3, ("stream", "grouped_rows"))])
def test_fshell_workload_strings_vs_golden(lib, ctx, name, config_id, kernels):
    """Workload strings of the generic f-shell benchmarks at production order
    (orders 40-44 of the (N, Jz) impurity, 60 of the crystal-field one)
    against the dense oracle (memory-bounded route, stored values): every
    FP64 kernel that runs the impurity, and FP32-split."""
    path = os.path.join(HERE, "golden", name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"{name}.json not generated")
    g = load_golden(name)
    assert g["config_id"] == config_id
    tab, c = ctx(g["impurity"])
    cfgs = make_configs(config_id, max(r["i"] for r in g["records"]) + 1)
    strings = [cfgs[r["i"]] for r in g["records"]]
    for s_, r in zip(strings, g["records"]):
        assert s_.n == r["n"] and np.allclose(s_.tau, r["tau"]) and np.array_equal(s_.op, r["op"])
    refs = [golden_pair(r) for r in g["records"]]
    scales = [(r["abs"], r["abs_log"]) for r in g["records"]]
    assert all(r[0] != 0 for r in refs)
    # at these orders the Lehmann modulus sum is 10^13-10^15 times |w|, which makes its
    # 1e-12 A bar looser than |w| itself: hold every value to 1e-10 of |w| as well
    outs = {}
    for k in kernels:
        say(f"[gpu] {name} strings x{len(strings)} kernel={k}")
        outs[k] = c.trace_batch(strings, kernel=HIST_KERNELS[k])
    say(f"[gpu] {name} strings FP32-split")
    outs["fp32-split"] = c.trace_batch(strings, precision=lib.CTR_FP32_SPLIT, kernel=lib.CTR_KERNEL_GROUPED,
                                       slices=7)
    for k, out in outs.items():
        check_against(out, refs, scales, f"{name} {k}")
        for v, ref in zip(out, refs):
            assert rel_err(pair(v), ref) <= 1e-10, (k, rel_err(pair(v), ref))


# ---------------------------------------------------------------------------
# full f-shell size: density-density impurity, exact by state enumeration
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("phase_seed", [None, 5])
def test_fshell_size_density_density_vs_enumeration(ctx, phase_seed):
    from oracle import densdens_trace

    tab, c = ctx("dd_fshell", phase_seed)
    assert tab.max_dim == 327 and tab.is_complex == (phase_seed is not None)
    imp = make_impurity("dd_fshell")
    cfgs = make_configs(2, 48)  # 14 flavors, beta 40, orders 40..160
    say(f"[gpu] ctr_trace_batch dd_fshell phase={phase_seed} x{len(cfgs)}")
    out = c.trace_batch(cfgs)
    refs = [densdens_trace(imp, s.tau, s.op) for s in cfgs]
    scales = [densdens_trace(imp, s.tau, s.op, moduli=True) for s in cfgs]
    check_against(out, refs, scales, f"dd_fshell phase={phase_seed}")
    assert sum(1 for r in refs if r[0] != 0) >= 10


def test_fshell_gauge_invariance(ctx):
    _, cg = ctx("fshell")
    _, cr = ctx("fshell_real")
    cfgs = make_configs(2, 40)
    say("[gpu] ctr_trace_batch fshell (complex) vs fshell_real x40")
    a, b = cg.trace_batch(cfgs), cr.trace_batch(cfgs)
    agree(a, b, "fshell complex vs real (gauge)")
    assert sum(1 for y in b if y["re"] != 0) >= 10


# ---------------------------------------------------------------------------
# identities at d-shell size
# ---------------------------------------------------------------------------

def test_cyclicity_and_anticommutation_dshell(ctx):
    from tests.tracecmp import add, insert_ops

    tab, c = ctx("dshell")
    rng = np.random.Generator(np.random.PCG64(3))
    beta = tab.beta
    say("[gpu] cyclicity / anticommutation dshell")
    # bar R14 with the cancellation scale of the evaluations themselves (log_abs)
    def scale(*vs):
        return 1.0, max(float(v["log_abs"]) for v in vs)

    for i in range(20):
        s = random_string(rng, 10, beta, 2 * int(rng.integers(5, 30)), "alternating")
        vw = c.trace(s.tau, s.op)
        w = pair(vw)
        d = float(rng.uniform(0, beta))
        t2 = (s.tau + d) % beta
        o = np.argsort(t2, kind="stable")
        v2 = c.trace(t2[o], s.op[o])
        if w[0] != 0:
            assert close_enough(pair(v2), w, scale(vw, v2)), (i, rel_err(pair(v2), w))
        t_new = float(rng.uniform(0, beta))
        f = int(rng.integers(10))
        va = c.trace(*insert_ops(s.tau, s.op, t_new, [2 * f + 1, 2 * f]))
        vb = c.trace(*insert_ops(s.tau, s.op, t_new, [2 * f, 2 * f + 1]))
        if w[0] != 0:
            assert close_enough(add(pair(va), pair(vb)), w, scale(vw, va, vb)), (i, rel_err(add(pair(va), pair(vb)), w))


# ---------------------------------------------------------------------------
# edge cases, errors, arena, determinism, lazy bounds
# ---------------------------------------------------------------------------

def test_error_paths(lib, ctx):
    tab, c = ctx("dshell")
    say("[gpu] error paths")
    with pytest.raises(lib.CtraceError) as e:
        c.trace([1.0, 0.5], [0, 1])
    assert e.value.status == -4
    with pytest.raises(lib.CtraceError) as e:
        c.trace([0.5, 1.0], [0, 99])
    assert e.value.status == -5
    with pytest.raises(lib.CtraceError) as e:
        c.trace([0.5, tab.beta], [0, 1])
    assert e.value.status == -5
    v = c.trace([0.5], [1])                       # odd: no string survives
    assert v["flags"] & 1 and v["re"] == 0 and v["n_strings"] == 0
    v = c.trace([0.5, 0.6], [1, 1])              # c+ c+ of one flavor: zero
    assert v["flags"] & 1
    assert c.trace_batch([]).shape == (0,)
    v = c.trace([0.7, 0.7], [2 * 3 + 1, 2 * 3])  # equal times, c c+: allowed
    assert v["n_strings"] > 0


def test_device_path_flags_invalid_configuration(lib, ctx):
    tab, c = ctx("dshell")
    good = make_configs(1, 3)
    bad = (np.array([2.0, 1.0]), np.array([0, 1], dtype=np.int32))
    from workloads.configs import OperatorString

    strings = [good[0], OperatorString(*bad), good[1], good[2]]
    say("[gpu] device path with one unsorted configuration")
    out = _device_batch(lib, c, strings)
    ref = c.trace_batch([good[0], good[1], good[2]])
    assert out[1]["flags"] & 4 and out[1]["re"] == 0
    assert np.array_equal(out[[0, 2, 3]]["re"], ref["re"])


def test_arena_oom_then_chunked_batches_identical(lib, ctx):
    tab, big = ctx("dshell")
    cfgs = make_configs(1, 300)
    say("[gpu] small-arena chunking dshell x300")
    ref = big.trace_batch(cfgs)
    resident = lib.ctr_arena_resident_bytes(big.ctx)
    with pytest.raises(lib.CtraceError) as e:
        lib.TraceContext(tab, arena_bytes=max(1 << 20, resident // 2))
    assert e.value.status == -2
    small = lib.TraceContext(tab, arena_bytes=resident + (1 << 20))
    try:
        # ~5 KiB of scratch per configuration: several chunks of the wavefront kernel
        ref_w = big.trace_batch(cfgs, kernel=lib.CTR_KERNEL_WAVE)
        out = small.trace_batch(cfgs, kernel=lib.CTR_KERNEL_WAVE)
        assert np.array_equal(out["re"], ref_w["re"]) and np.array_equal(out["log_scale"], ref_w["log_scale"])
        # grouped rounds: the carried matrices do not fit, the batch is halved until they do;
        # every column's arithmetic is independent of how the batch is grouped
        assert np.array_equal(ref["re"], ref_w["re"])  # the automatic choice here is the wavefront kernel
        mid = lib.TraceContext(tab, arena_bytes=resident + (8 << 20))
        try:
            out = mid.trace_batch(cfgs, kernel=lib.CTR_KERNEL_GROUPED)
            ref_g = big.trace_batch(cfgs, kernel=lib.CTR_KERNEL_GROUPED)
            assert np.array_equal(out["re"], ref_g["re"]) and np.array_equal(out["log_scale"], ref_g["log_scale"])
        finally:
            mid.close()
        # forced grouped rounds that cannot fit one configuration: out of memory
        with pytest.raises(lib.CtraceError) as e:
            small.trace_batch(cfgs, kernel=lib.CTR_KERNEL_GROUPED)
        assert e.value.status == -2
    finally:
        small.close()


def test_auto_falls_back_when_grouped_rounds_do_not_fit(lib, ctx):
    """f-shell (327-state sectors): AUTO takes the grouped rounds for 300 traces,
    and the LDS workgroup kernel when the arena cannot hold their scratch."""
    tab, big = ctx("fshell")
    cfgs = make_configs(2, 300)
    say("[gpu] AUTO fallback fshell x300")
    auto = big.trace_batch(cfgs)
    grouped = big.trace_batch(cfgs, kernel=lib.CTR_KERNEL_GROUPED)
    block = big.trace_batch(cfgs, kernel=lib.CTR_KERNEL_BLOCK)
    assert np.array_equal(auto["re"], grouped["re"]) and np.array_equal(auto["im"], grouped["im"])
    small = lib.TraceContext(tab, arena_bytes=lib.ctr_arena_resident_bytes(big.ctx) + (1 << 20))
    try:
        out = small.trace_batch(cfgs)
        assert np.array_equal(out["re"], block["re"]) and np.array_equal(out["im"], block["im"])
    finally:
        small.close()


def test_grouped_rounds_agree_with_per_string_kernels(lib, ctx):
    """Block-grouped rounds against the wavefront kernel on 2000 d-shell traces
    (different MFMA shapes: rounding-level agreement) and against the LDS
    workgroup kernel on the complex 327-state f-shell."""
    tab, c = ctx("dshell")
    cfgs = make_configs(1, 2000)
    say("[gpu] grouped vs wavefront dshell x2000")
    b = c.trace_batch(cfgs, kernel=lib.CTR_KERNEL_WAVE)
    for k in (lib.CTR_KERNEL_GROUPED, lib.CTR_KERNEL_GROUPED_ROWS):
        a = c.trace_batch(cfgs, kernel=k)
        assert agree(a, b, f"grouped {k} vs wavefront dshell") < 1e-11
    tab, c = ctx("fshell")
    cfgs = make_configs(2, 300)
    say("[gpu] grouped vs block fshell x300")
    b = c.trace_batch(cfgs, kernel=lib.CTR_KERNEL_BLOCK)
    for k in (lib.CTR_KERNEL_GROUPED, lib.CTR_KERNEL_GROUPED_ROWS):
        a = c.trace_batch(cfgs, kernel=k)
        agree(a, b, f"grouped {k} vs block fshell")


def test_determinism_and_batch_order(ctx):
    tab, c = ctx("dshell")
    cfgs = make_configs(1, 400)
    say("[gpu] determinism dshell x400")
    a = c.trace_batch(cfgs)
    b = c.trace_batch(cfgs)
    r = c.trace_batch(cfgs[::-1])[::-1]
    for x in (b, r):
        assert np.array_equal(a["re"], x["re"]) and np.array_equal(a["im"], x["im"])
        assert np.array_equal(a["log_scale"], x["log_scale"])


def test_lazy_bound_and_rejection(lib, ctx):
    tab, c = ctx("dshell")
    cfgs = make_configs(1, 300)
    offs, tau, op = pack(cfgs)
    say("[gpu] lazy bounds dshell x300")
    # reference through the same kernel the lazy call runs (nothing rejected at -inf)
    exact = c.lazy_batch(offs, tau, op, np.full(len(cfgs), -np.inf))
    assert not np.any(exact["flags"] & 2)
    la = np.array([lib.log_abs(v) for v in exact])
    lb = exact["log_bound"]
    assert np.all(la <= lb + 1e-9)
    # single-configuration bound call agrees with the batch field
    assert abs(c.bound(cfgs[7].tau, cfgs[7].op) - lb[7]) < 1e-9
    rng = np.random.Generator(np.random.PCG64(9))
    thr = lb + rng.uniform(-3.0, 3.0, size=lb.size)
    out = c.lazy_batch(offs, tau, op, thr)
    rej = (out["flags"] & 2) != 0
    # everything below the plan bound is rejected; refined bounds reject more
    assert np.all(rej[(lb < thr) & (exact["n_strings"] > 0)])
    say(f"lazy: {int(np.sum(lb < thr))} rejected by the plan bound, {int(np.sum(rej))} in total")
    keep = ~rej
    assert np.array_equal(out["re"][keep], exact["re"][keep])
    assert np.array_equal(out["log_scale"][keep], exact["log_scale"][keep])
    # no false rejection: a rejected trace is truly below its threshold
    assert np.all(la[rej] < thr[rej])
    assert np.all(out["re"][rej] == 0)
    # the single-configuration call gives the batch's decision and value
    for i in range(0, 300, 37):
        one = c.lazy(cfgs[i].tau, cfgs[i].op, thr[i])
        assert (one["flags"] & 2) == (out["flags"][i] & 2), i
        if not rej[i]:
            assert close_enough(pair(one), pair(out[i]), (1.0, float(out["log_abs"][i]))), i


@pytest.mark.parametrize("name,cid,count,kernel,split", [
    ("dshell", 1, 300, "auto", False), ("dshell", 1, 200, "block", False), ("dshell", 1, 200, "block", True),
    ("dshell", 1, 300, "grouped", False), ("pshell", 2, 200, "auto", False), ("dd_fshell_n", 3, 12, "auto", False)])
def test_lazy_refinement_rejects_only_below_threshold(lib, ctx, name, cid, count, kernel, split):
    """Thresholds between |trace| and the plan bound: only the refined bounds
    (Frobenius norm of the running product, exact panel values) can reject."""
    k = {"auto": lib.CTR_KERNEL_AUTO, "block": lib.CTR_KERNEL_BLOCK, "grouped": lib.CTR_KERNEL_GROUPED}[kernel]
    prec = lib.CTR_FP32_SPLIT if split else lib.CTR_FP64
    tab, c = ctx(name)
    imp = make_impurity(name)
    strings = make_configs(cid, count) if name != "pshell" else \
        [random_string(np.random.Generator(np.random.PCG64(100 + i)), imp.n_flavors, imp.beta, 40, "alternating")
         for i in range(count)]
    offs, tau, op = pack(strings)
    say(f"[gpu] lazy refinement {name} x{count} kernel={kernel} split={split}")
    exact = c.lazy_batch(offs, tau, op, np.full(len(strings), -np.inf), prec, k)
    assert not np.any(exact["flags"] & 2)
    la = np.array([lib.log_abs(v) for v in exact])
    lb = exact["log_bound"]
    live = np.isfinite(la)
    rng = np.random.Generator(np.random.PCG64(21))
    thr = np.where(live, la + rng.uniform(0.0, 1.0, size=la.size) * (lb - la), -np.inf)
    thr = np.where(rng.uniform(size=la.size) < 0.5, thr, la - 1.0)   # half of them must be kept
    out = c.lazy_batch(offs, tau, op, thr, prec, k)
    rej = (out["flags"] & 2) != 0
    assert np.all(la[rej] < thr[rej])            # no false rejection
    keep = ~rej
    assert np.array_equal(out["re"][keep], exact["re"][keep])
    assert not np.any(rej & (thr < la))
    say(f"lazy refinement {name}: {int(np.sum(rej))} of {int(np.sum(thr > la))} rejectable configurations rejected")


@pytest.mark.parametrize("kernel", ["wave", "block", "stream", "grouped", "grouped_rows"])
def test_every_chain_kernel_matches_the_oracle(lib, ctx, kernel):
    """The chain kernels (wavefront, LDS workgroup, streaming, block-grouped
    rounds, row-chunked grouped rounds) forced on impurities the oracle covers."""
    k = HIST_KERNELS[kernel]
    g = load_golden("dshell_config1")
    tab, c = ctx("dshell")
    recs = g["records"][:96]
    say(f"[gpu] kernel={kernel} dshell x{len(recs)}")
    out = c.trace_batch(make_configs(1, len(recs)), kernel=k)
    check_against(out, [golden_pair(r) for r in recs], [(r["abs"], r["abs_log"]) for r in recs], f"dshell {kernel}")
    for name in ("pshell_random", "dshell_so_random"):
        g = load_golden(name)
        tab, c = ctx(g["impurity"])
        strings = [(np.array(r["tau"]), np.array(r["op"], dtype=np.int32)) for r in g["records"]]
        say(f"[gpu] kernel={kernel} {name}")
        out = c.trace_batch(strings, kernel=k)
        check_against(out, [golden_pair(r) for r in g["records"]], [(r["abs"], r["abs_log"]) for r in g["records"]],
                      f"{name} {kernel}")


def test_kernel_option_errors(lib, ctx):
    tab, c = ctx("dshell")
    with pytest.raises(lib.CtraceError) as e:
        c.trace([0.5, 1.0], [1, 0], precision=lib.CTR_FP32_SPLIT, kernel=lib.CTR_KERNEL_WAVE)
    assert e.value.status == -7
    with pytest.raises(lib.CtraceError) as e:
        c.trace([0.5, 1.0], [1, 0], precision=lib.CTR_FP32_SPLIT, kernel=lib.CTR_KERNEL_STREAM)
    assert e.value.status == -7
    with pytest.raises(lib.CtraceError) as e:
        c.trace([0.5, 1.0], [1, 0], kernel=7)
    assert e.value.status == -1


@pytest.mark.parametrize("phase_seed", [None, 11])
def test_sectors_of_3432_states_density_density_vs_enumeration(lib, ctx, phase_seed):
    """N-only sectors of the 14-flavor shell (largest 3432 states): the
    streaming kernel and the (row-chunked) grouped rounds, checked against
    exact state enumeration."""
    from oracle import densdens_trace

    tab, c = ctx("dd_fshell_n", phase_seed)
    assert tab.max_dim == 3432
    imp = make_impurity("dd_fshell_n")
    cfgs = make_configs(3, 10)  # 14 flavors, beta 40, orders 60..200
    refs = [densdens_trace(imp, s.tau, s.op) for s in cfgs]
    scales = [densdens_trace(imp, s.tau, s.op, moduli=True) for s in cfgs]
    for k in ("stream", "grouped"):
        say(f"[gpu] ctr_trace_batch dd_fshell_n phase={phase_seed} x{len(cfgs)} kernel={k}")
        out = c.trace_batch(cfgs, kernel=HIST_KERNELS[k])
        check_against(out, refs, scales, f"dd_fshell_n phase={phase_seed} {k}")
    assert sum(1 for r in refs if r[0] != 0) >= 5
    with pytest.raises(lib.CtraceError) as e:
        c.trace(cfgs[0].tau, cfgs[0].op, kernel=lib.CTR_KERNEL_BLOCK)
    assert e.value.status == -7


# ---------------------------------------------------------------------------
# FP32-split precision (FP32 MFMA on exact integer slices, FP64 elsewhere)
# ---------------------------------------------------------------------------

def test_fp32_split_d_shell_vs_golden_and_fp64(lib, ctx):
    tab, c = ctx("dshell")
    g = load_golden("dshell_config1")
    cfgs = make_configs(1, len(g["records"]))
    say("[gpu] ctr_trace_batch FP32_SPLIT config1 x256")
    out = c.trace_batch(cfgs, precision=lib.CTR_FP32_SPLIT)
    check_against(out, [golden_pair(r) for r in g["records"]], [(r["abs"], r["abs_log"]) for r in g["records"]],
                  "config1 fp32-split vs oracle")
    f64 = c.trace_batch(cfgs)
    # six slices against the FP64 path at the R14 bar (cancellation scale log_abs)
    agree(out, f64, "config1 fp32-split (6 slices) vs fp64")


def test_fp32_split_seven_slices_d_shell_vs_golden_and_fp64(lib, ctx):
    """Seven 8-bit slices: stored oracle values, and agreement with the FP64
    path within 1e-11 relative on every nonzero trace."""
    tab, c = ctx("dshell")
    g = load_golden("dshell_config1")
    cfgs = make_configs(1, len(g["records"]))
    say("[gpu] ctr_trace_batch FP32_SPLIT 7 slices config1 x256")
    out = c.trace_batch(cfgs, precision=lib.CTR_FP32_SPLIT, slices=7)
    check_against(out, [golden_pair(r) for r in g["records"]], [(r["abs"], r["abs_log"]) for r in g["records"]],
                  "config1 fp32-split 7 slices vs oracle")
    f64 = c.trace_batch(cfgs, kernel=lib.CTR_KERNEL_BLOCK)
    worst = max(rel_err(pair(a), pair(b)) for a, b in zip(out, f64) if b["re"] != 0)
    say(f"config1 fp32-split (7 slices) vs fp64 worst rel {worst:.2e}")
    assert worst < 1e-11


@pytest.mark.parametrize("name", ["pshell_random", "dshell_so_random"])
@pytest.mark.parametrize("kernel,slices", [("block", 6), ("grouped", 6), ("grouped", 7)])
def test_fp32_split_complex_vs_golden(lib, ctx, name, kernel, slices):
    """FP32-split on the per-string LDS kernel and on the row-chunked grouped
    rounds against stored oracle values."""
    g = load_golden(name)
    tab, c = ctx(g["impurity"])
    strings = [(np.array(r["tau"]), np.array(r["op"], dtype=np.int32)) for r in g["records"]]
    say(f"[gpu] ctr_trace_batch FP32_SPLIT {name} kernel={kernel} slices={slices}")
    out = c.trace_batch(strings, precision=lib.CTR_FP32_SPLIT, kernel=HIST_KERNELS[kernel], slices=slices)
    check_against(out, [golden_pair(r) for r in g["records"]], [(r["abs"], r["abs_log"]) for r in g["records"]],
                  f"{name} fp32-split {kernel} {slices}")


@pytest.mark.parametrize("name", ["fshell_low", "fshell_cf_low"])
def test_fp32_split_generic_fshell_vs_golden(lib, ctx, name):
    """FP32-split (seven slices, grouped rounds) on the generic 16384-state
    f-shell impurities, (N, Jz) and crystal-field, against the dense oracle."""
    g = load_golden(name)
    tab, c = ctx(g["impurity"])
    strings = [(np.array(r["tau"]), np.array(r["op"], dtype=np.int32)) for r in g["records"]]
    say(f"[gpu] ctr_trace_batch FP32_SPLIT {name} x{len(strings)}")
    out = c.trace_batch(strings, precision=lib.CTR_FP32_SPLIT, kernel=lib.CTR_KERNEL_GROUPED, slices=7)
    check_against(out, [golden_pair(r) for r in g["records"]], [(r["abs"], r["abs_log"]) for r in g["records"]],
                  f"{name} fp32-split")


@pytest.mark.parametrize("name,cid,count", [("dd_fshell", 2, 48), ("dd_fshell_n", 3, 10)])
def test_fp32_split_fshell_size_density_density_vs_enumeration(lib, ctx, name, cid, count):
    """FP32-split at full f-shell size and workload orders (40-160, 60-200),
    phase-randomised complex blocks, against exact state enumeration."""
    from oracle import densdens_trace

    tab, c = ctx(name, 7)
    imp = make_impurity(name)
    cfgs = make_configs(cid, count)
    say(f"[gpu] FP32_SPLIT {name} x{len(cfgs)}")
    out = c.trace_batch(cfgs, precision=lib.CTR_FP32_SPLIT, kernel=lib.CTR_KERNEL_GROUPED, slices=7)
    refs = [densdens_trace(imp, s.tau, s.op) for s in cfgs]
    scales = [densdens_trace(imp, s.tau, s.op, moduli=True) for s in cfgs]
    check_against(out, refs, scales, f"{name} fp32-split")


def test_fp32_split_fshell_workload_vs_fp64(lib, ctx):
    """FP32-split (seven slices) against the FP64 path on 300 workload
    configurations of the generic f-shell (N, Jz) at orders 40-160, R14 bar."""
    tab, c = ctx("fshell")
    cfgs = make_configs(2, 300)
    say("[gpu] FP32_SPLIT vs FP64 fshell x300")
    a = c.trace_batch(cfgs, precision=lib.CTR_FP32_SPLIT, kernel=lib.CTR_KERNEL_GROUPED, slices=7)
    b = c.trace_batch(cfgs, kernel=lib.CTR_KERNEL_GROUPED)
    agree(a, b, "fshell fp32-split (7) vs fp64")


def test_fp32_split_rejects_unsupported_slices(lib, ctx):
    tab, c = ctx("kanamori2")
    o = lib.ctr_opts()
    o.precision = lib.CTR_FP32_SPLIT
    o.slices = 3
    v = lib.ctr_value()
    tau = np.array([1.0, 2.0])
    op = np.array([1, 0], dtype=np.int32)
    st = lib._lib.ctr_trace(c.ctx, 2, lib._ptr(tau, lib.ctypes.c_double), lib._ptr(op, lib.ctypes.c_int32),
                            lib.ctypes.byref(o), lib.ctypes.byref(v))
    assert st == -7


# ---------------------------------------------------------------------------
# serving: continuous batching over several impurities
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("own_streams,grid_share,cf", [(False, None, False), (True, None, False),
                                                      (True, (0.25, 0.75), False), (True, (0.5, 0.5, 0.5), True)])
def test_server_results_match_alone(lib, ctx, own_streams, grid_share, cf):
    """Requests for two impurities (real d-shell, complex p-shell), plain and
    lazy, submitted from four threads while earlier ones are on the GPU: every
    result equals the same request evaluated alone, within the parity bar;
    also with each impurity on a stream of its own (the passes overlap on the
    device), with each impurity's kernels launched on a share of their grids,
    and with the crystal-field f-shell (3432-state sectors) as a third lane."""
    import threading

    import torch

    tab_d, cd = ctx("dshell")
    tab_p, cp = ctx("pshell")
    imp_p = make_impurity("pshell")
    lanes = [cd, cp]
    tabs = [tab_d, tab_p]
    if cf:
        tab_c, cc = ctx("fshell_cf")
        lanes.append(cc)
        tabs.append(tab_c)
    rng = np.random.Generator(np.random.PCG64(31))
    reqs = []  # (impurity, string, log threshold)
    for s in make_configs(1, 400):
        reqs.append((0, s, -math.inf))
    for i in range(200):
        reqs.append((1, random_string(rng, imp_p.n_flavors, imp_p.beta, 2 * int(rng.integers(1, 30)), "alternating"),
                     -math.inf))
    if cf:
        for s in make_configs(3, 10):
            reqs.append((2, s, -math.inf))
    say("[gpu] server: reference values alone")
    alone = []
    for k, s, _ in reqs:
        alone.append(lanes[k].trace(s.tau, s.op))
    # every fourth d-shell request becomes lazy with a threshold around its value
    lazy_idx = list(range(0, 400, 4))
    for i in lazy_idx:
        k, s, _ = reqs[i]
        la = lib.log_abs(alone[i])
        thr = la + float(rng.uniform(-2.0, 2.0)) if np.isfinite(la) else -1.0
        reqs[i] = (k, s, thr)
        alone[i] = cd.lazy_batch(np.array([0, s.n]), s.tau, s.op, np.array([thr]))[0]
    order = rng.permutation(len(reqs))
    served = list(lanes)
    if own_streams:
        served = [lib.TraceContext(t, stream=torch.cuda.Stream()) for t in tabs]
    srv = lib.TraceServer(served, max_batch=96, grid_share=grid_share)
    try:
        def submit(part):
            for j in part:
                k, s, thr = reqs[j]
                while srv.submit(k, int(j), s.tau, s.op, thr) == lib.CTR_ERR_BUSY:
                    pass
        say("[gpu] server: 4 submitting threads")
        th = [threading.Thread(target=submit, args=(order[t::4],)) for t in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        srv.drain()
        res = srv.poll(max_results=len(reqs) + 10)
        passes, evaluated = srv.stats()
    finally:
        srv.close()
        if own_streams:
            for c in served:
                c.close()
    assert len(res) == len(reqs) and evaluated == len(reqs)
    assert np.all(res["status"] == 0)
    assert passes < len(reqs) and res["batch"].max() > 1   # requests were batched
    say(f"server: {len(reqs)} requests in {passes} device passes, largest batch {res['batch'].max()}")
    for r in res:
        j = int(r["tag"])
        k = int(r["impurity"])
        assert k == reqs[j][0]
        got, ref = r["value"], alone[j]
        assert (got["flags"] & 2) == (ref["flags"] & 2), j
        if ref["re"] == 0 and ref["im"] == 0:
            assert got["re"] == 0 and got["im"] == 0
            continue
        assert close_enough(pair(got), pair(ref), (1.0, max(float(got["log_abs"]), float(ref["log_abs"])))), j
    # contexts are usable again after the server is gone
    v = cd.trace(reqs[1][1].tau, reqs[1][1].op)
    assert np.array_equal(v["re"], alone[1]["re"])


def test_server_pass_cap_admits_one_request_per_pass(lib, ctx):
    """A cap on a pass's estimated work below any single request's: every pass
    still admits one request (never none), and the values are unchanged."""
    tab, c = ctx("dshell")
    configs = make_configs(1, 40)
    alone = [c.trace(s.tau, s.op) for s in configs]
    srv = lib.TraceServer([c], max_batch=64, max_pass_flop=1.0)
    try:
        for j, s in enumerate(configs):
            while srv.submit(0, j, s.tau, s.op) == lib.CTR_ERR_BUSY:
                pass
        srv.drain()
        res = srv.poll(max_results=100)
        passes, evaluated = srv.stats()
    finally:
        srv.close()
    assert len(res) == len(configs) and evaluated == len(configs) and passes == len(configs)
    assert np.all(res["batch"] == 1) and np.all(res["status"] == 0)
    for r in res:
        j = int(r["tag"])
        got, ref = r["value"], alone[j]
        if ref["re"] == 0 and ref["im"] == 0:
            assert got["re"] == 0 and got["im"] == 0
            continue
        assert close_enough(pair(got), pair(ref), (1.0, max(float(got["log_abs"]), float(ref["log_abs"])))), j


def test_server_rejects_invalid_and_reports_busy(lib, ctx):
    tab, c = ctx("dshell")
    srv = lib.TraceServer([c], max_batch=8, max_pending=1)
    try:
        with pytest.raises(lib.CtraceError) as e:
            srv.submit(0, 1, [1.0, 0.5], [0, 1])
        assert e.value.status == -4
        with pytest.raises(lib.CtraceError) as e:
            srv.submit(0, 2, [0.5, 1.0], [0, 99])
        assert e.value.status == -5
        with pytest.raises(lib.CtraceError) as e:
            srv.submit(3, 3, [0.5, 1.0], [0, 1])
        assert e.value.status == -1
        s = make_configs(1, 1)[0]
        st = [srv.submit(0, 10 + i, s.tau, s.op) for i in range(64)]
        assert st[0] == 0 and lib.CTR_ERR_BUSY in st   # one pending slot: some submissions bounce
        srv.drain()
        res = srv.poll(max_results=100)
        assert len(res) == sum(1 for x in st if x == 0)
    finally:
        srv.close()


# ---------------------------------------------------------------------------
# maximum sizes and degenerate batches
# ---------------------------------------------------------------------------

def test_maximum_operator_count_vs_oracle(lib, ctx):
    """512 operators (the most a configuration may hold) on the 2-orbital atom
    and 200-300 on the d-shell, every kernel that runs them, against the
    oracle; 513 operators are refused."""
    from oracle import DenseTrace

    rng = np.random.Generator(np.random.PCG64(55))
    for name, orders in (("kanamori2", (512, 510, 256)), ("dshell", (300, 200))):
        tab, c = ctx(name)
        imp = make_impurity(name)
        dt = DenseTrace(imp)
        strings = [random_string(rng, imp.n_flavors, imp.beta, n, "alternating") for n in orders]
        refs = [dt.trace(s.tau, s.op) for s in strings]
        scales = [dt.abs_scale(s.tau, s.op) for s in strings]
        kernels = [lib.CTR_KERNEL_WAVE, lib.CTR_KERNEL_BLOCK, lib.CTR_KERNEL_STREAM, lib.CTR_KERNEL_GROUPED,
                   lib.CTR_KERNEL_GROUPED_ROWS]
        for k in kernels:
            say(f"[gpu] maximum orders {name} {orders} kernel={k}")
            out = c.trace_batch(strings, kernel=k)
            check_against(out, refs, scales, f"{name} max orders kernel {k}")
        assert sum(1 for r in refs if r[0] != 0) >= 1
    tab, c = ctx("kanamori2")
    s = random_string(rng, 4, tab.beta, 514, "alternating")
    with pytest.raises(lib.CtraceError) as e:
        c.trace(s.tau[:513], s.op[:513])
    assert e.value.status == -1


def test_grouped_rounds_on_degenerate_batches(lib, ctx):
    """Grouped rounds on batches whose configurations have no product step:
    order 0 (the partition function), odd or dead strings (exact zero), and a
    mix with ordinary ones; same values as the wavefront kernel."""
    from workloads.configs import OperatorString

    tab, c = ctx("dshell")
    z = (np.zeros(0), np.zeros(0, dtype=np.int32))
    odd = (np.array([1.0]), np.array([1], dtype=np.int32))
    dead = (np.array([1.0, 2.0]), np.array([1, 1], dtype=np.int32))
    two = (np.array([1.0, 2.0]), np.array([1, 0], dtype=np.int32))
    for batch in ([z] * 300, [odd, dead] * 150, [z, odd, dead, two] * 75 + list(
            (s.tau, s.op) for s in make_configs(1, 60))):
        say(f"[gpu] grouped degenerate batch of {len(batch)}")
        w = c.trace_batch(batch, kernel=lib.CTR_KERNEL_WAVE)
        for k in (lib.CTR_KERNEL_GROUPED, lib.CTR_KERNEL_GROUPED_ROWS):
            g = c.trace_batch(batch, kernel=k)
            assert np.array_equal(g["flags"], w["flags"]) and np.array_equal(g["n_strings"], w["n_strings"])
            for a, b in zip(g, w):
                if b["re"] == 0 and b["im"] == 0:
                    assert a["re"] == 0 and a["im"] == 0
                else:
                    assert rel_err(pair(a), pair(b)) < 1e-12
    with pytest.raises(lib.CtraceError) as e:
        c.trace_batch([OperatorString(np.array([2.0, 1.0]), np.array([1, 0], dtype=np.int32))],
                      kernel=lib.CTR_KERNEL_GROUPED)
    assert e.value.status == -4


def test_autotuner_picks_a_kernel_that_then_runs_under_auto(lib, ctx):
    """ctr_tune times every FP64 chain kernel on a sample; AUTO then runs the
    chosen one (bit-identical to forcing it) for batches of a quarter of the
    sample or more, and the built-in choice below."""
    tab, shared = ctx("dshell")
    c = lib.TraceContext(tab)
    try:
        cfgs = make_configs(1, 600)
        offs, tau, op = pack(cfgs)
        say("[gpu] autotune dshell x600")
        chosen, ms = c.tune(offs, tau, op)
        say(f"autotune: chose {chosen}, ms {ms}")
        assert chosen in ms and set(ms) == {1, 2, 3, 4}   # every kernel runs the d-shell
        assert ms[chosen] == min(ms.values())
        auto = c.trace_packed(offs, tau, op)
        forced = c.trace_packed(offs, tau, op, kernel=chosen)
        assert np.array_equal(auto["re"], forced["re"]) and np.array_equal(auto["log_scale"], forced["log_scale"])
        small = make_configs(1, 40)   # below a quarter of the sample: built-in choice (wavefront)
        a = c.trace_batch(small)
        w = c.trace_batch(small, kernel=lib.CTR_KERNEL_WAVE)
        assert np.array_equal(a["re"], w["re"])
        # the grouped rounds in the tile shape the tuner kept agree with the per-string kernel
        g = c.trace_packed(offs, tau, op, kernel=lib.CTR_KERNEL_GROUPED)
        wv = c.trace_packed(offs, tau, op, kernel=lib.CTR_KERNEL_WAVE)
        for x, y in zip(g, wv):
            if y["re"] != 0:
                assert rel_err(pair(x), pair(y)) < 1e-10 * max(1.0, math.exp(y["log_abs"] - y["log_scale"]
                                                                            - math.log(abs(y["re"]))))
    finally:
        c.close()


def test_autotuner_times_both_grouped_tile_shapes_fshell(lib, ctx):
    """On the f-shell the grouped rounds have two tile shapes (12 x 2 and 8 x 3
    wavefronts x row tiles); after tuning, whichever was kept gives the same
    traces as the per-string kernel."""
    tab, shared = ctx("fshell")
    c = lib.TraceContext(tab)
    try:
        cfgs = make_configs(2, 300)
        offs, tau, op = pack(cfgs)
        say("[gpu] autotune fshell x300")
        chosen, ms = c.tune(offs, tau, op)
        say(f"autotune fshell: chose {chosen}, ms {ms}")
        assert 4 in ms
        g = c.trace_packed(offs, tau, op, kernel=lib.CTR_KERNEL_GROUPED)
        b = c.trace_packed(offs, tau, op, kernel=lib.CTR_KERNEL_BLOCK)
        n = 0
        for x, y in zip(g, b):
            if y["re"] == 0 and y["im"] == 0:
                continue
            n += 1
            ratio = max(1.0, math.exp(y["log_abs"] - y["log_scale"] - math.log(abs(complex(y["re"], y["im"])))))
            assert rel_err(pair(x), pair(y)) < 1e-10 * ratio
        assert n > 100
    finally:
        c.close()


# ---------------------------------------------------------------------------
# label histogram (density-matrix estimator summed over a conserved label)
# ---------------------------------------------------------------------------

def _sector_n(tab):
    return np.array([bin(int(st[0])).count("1") for st in tab.states], dtype=np.int32)


def _hist_strings(imp, seed, count, max_order):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = [random_string(rng, imp.n_flavors, imp.beta, 0, "alternating")]
    for _ in range(count - 1):
        out.append(random_string(rng, imp.n_flavors, imp.beta, 2 * int(rng.integers(1, max_order // 2 + 1)),
                                 "alternating"))
    return out


def _check_hist(out, hist, refs, label):
    """refs: (h_ref, scale_ref, A/|w| of the trace) per configuration.  Bar:
    |h - h_ref| <= 1e-10 |h_ref| + 1e-12 (scale + A/|w|).  The entries are
    fractions of one (they sum to one), so the absolute part is measured
    against that normalisation, times the trace's own cancellation ratio:
    an entry whose exact value is zero moves by rounding-level couplings in
    H_loc (the dense Hamiltonian carries ~2e-16 between states the sector
    builder keeps apart), by far less than 1e-12 of the total."""
    worst, bad, nz = 0.0, [], 0
    for i, (v, h, (href, sc, ratio)) in enumerate(zip(out, hist, refs)):
        if not np.any(href):
            assert not np.any(h), f"{label} #{i}: oracle zero trace, gpu histogram {h}"
            continue
        nz += 1
        d = np.abs(h - href)
        tol = 1e-10 * np.abs(href) + 1e-12 * (sc + ratio)
        worst = max(worst, float(np.max(d / np.maximum(np.abs(href), 1e-300))))
        if np.any(d > tol):
            bad.append((i, float(np.max(d - tol))))
    say(f"{label}: {len(out)} configurations ({nz} nonzero), worst rel err {worst:.2e}, failures {bad[:5]}")
    assert not bad
    return nz


def _oracle_hist_refs(imp, strings, state_label, n_labels):
    from oracle import DenseTrace
    from oracle.observables import label_histogram, label_histogram_abs, label_projectors

    dt = DenseTrace(imp)
    P = label_projectors(dt, state_label, n_labels)
    refs = []
    for s in strings:
        h, w = label_histogram(dt, s.tau, s.op, P)
        if w[0] == 0:
            refs.append((h, np.zeros(n_labels), 0.0))
            continue
        a = dt.abs_scale(s.tau, s.op)
        refs.append((h, label_histogram_abs(dt, s.tau, s.op, P), abs(a[0]) * math.exp(a[1] - w[1]) / abs(w[0])))
    return refs


_HIST_REFS = {}


@pytest.mark.parametrize("name,kernel,slices", [
    ("kanamori2", "wave", 0), ("kanamori2", "grouped", 0), ("pshell", "wave", 0), ("pshell", "block", 0),
    ("pshell", "stream", 0), ("pshell", "grouped", 0), ("pshell", "block", 7)])
def test_valence_histogram_vs_oracle(lib, ctx, name, kernel, slices):
    """h_N of random configurations (order 0 included) against the oracle's
    projector insertion in every interval; bar as in _check_hist."""
    from oracle.fock import occupations

    tab, c = ctx(name)
    imp = make_impurity(name)
    strings = _hist_strings(imp, 401, 40, 12)
    n_labels = imp.n_flavors + 1
    if name not in _HIST_REFS:
        _HIST_REFS[name] = _oracle_hist_refs(imp, strings, occupations(imp.n_flavors).sum(axis=1), n_labels)
    refs = _HIST_REFS[name]
    offs, tau, op = pack(strings)
    say(f"[gpu] ctr_trace_histogram {name} kernel={kernel} slices={slices} x{len(strings)}")
    out, hist = c.histogram(offs, tau, op, _sector_n(tab), n_labels,
                            precision=lib.CTR_FP32_SPLIT if slices else lib.CTR_FP64,
                            kernel=HIST_KERNELS[kernel], slices=slices)
    assert _check_hist(out, hist, refs, f"{name}/{kernel}/{slices}") >= 20
    # order zero: the Boltzmann weights of the N sectors
    E0 = tab.e0()
    z = np.zeros(n_labels)
    for q, e in enumerate(tab.energies):
        z[_sector_n(tab)[q]] += np.sum(np.exp(-imp.beta * (np.asarray(e) - E0)))
    assert np.max(np.abs(hist[0] - z / z.sum())) < 1e-13


def test_histogram_over_sector_index_labels(lib, ctx):
    """Label = sector index (more labels than one register pass holds), so
    the histogram is the weight of every sector; compared with the oracle's
    projectors built from the states' abelian charges."""
    from oracle.fock import occupations

    tab, c = ctx("pshell")
    imp = make_impurity("pshell")
    labs = occupations(imp.n_flavors) @ np.asarray(imp.qn).T
    of = tab.sector_of_label()
    state_sector = np.array([of[tuple(int(x) for x in row)] for row in labs])
    strings = _hist_strings(imp, 402, 24, 8)
    refs = _oracle_hist_refs(imp, strings, state_sector, tab.n_sectors)
    offs, tau, op = pack(strings)
    say(f"[gpu] ctr_trace_histogram pshell sector labels ({tab.n_sectors}) x{len(strings)}")
    out, hist = c.histogram(offs, tau, op, np.arange(tab.n_sectors), tab.n_sectors)
    assert tab.n_sectors > 16
    assert _check_hist(out, hist, refs, "pshell/sector-labels") >= 12


@pytest.mark.parametrize("name,cid,count,kernels", [("dshell", 1, 256, ("wave", "grouped")),
                                                    ("fshell", 2, 48, ("block", "grouped")),
                                                    ("fshell_cf", 3, 8, ("stream", "grouped_rows"))])
def test_histogram_full_size_sum_rule_and_kernels_agree(lib, ctx, name, cid, count, kernels):
    """Full-size impurities: the labels of every nonzero configuration sum to
    one, and two chain kernels agree, both within 1e-10 times the
    configuration's cancellation ratio (sum of string moduli over |w|)."""
    tab, c = ctx(name)
    imp = make_impurity(name)
    n_labels = imp.n_flavors + 1
    offs, tau, op = pack(make_configs(cid, count))
    res = []
    for k in kernels:
        say(f"[gpu] ctr_trace_histogram {name} workload {cid} x{count} kernel={k}")
        res.append(c.histogram(offs, tau, op, _sector_n(tab), n_labels, kernel=HIST_KERNELS[k]))
    (out, h0), (_, h1) = res
    nz = 0
    for i, v in enumerate(out):
        if v["re"] == 0 and v["im"] == 0:
            assert not np.any(h0[i]) and not np.any(h1[i])
            continue
        nz += 1
        ratio = max(1.0, math.exp(v["log_abs"] - v["log_scale"] - math.log(abs(complex(v["re"], v["im"])))))
        assert abs(h0[i].sum() - 1.0) <= 1e-10 * ratio, (i, h0[i].sum())
        assert np.max(np.abs(h0[i] - h1[i])) <= 1e-10 * ratio, i
    assert nz >= count // 2


def test_histogram_argument_errors(lib, ctx):
    tab, c = ctx("kanamori2")
    offs, tau, op = pack(_hist_strings(make_impurity("kanamori2"), 403, 4, 4))
    with pytest.raises(lib.CtraceError) as e:
        c.histogram(offs, tau, op, np.full(tab.n_sectors, 5), 5)
    assert e.value.status == -5  # CTR_ERR_RANGE: label >= n_labels
    with pytest.raises(lib.CtraceError):
        c.histogram(offs, tau, op, np.zeros(tab.n_sectors), 0)


# ---------------------------------------------------------------------------
# Markov chains around the trace (pair moves, w_hyb fast updates, lazy batch)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,n_chains,steps", [("kanamori2", 32, 300), ("pshell", 16, 150)])
def test_markov_chains_follow_the_oracle(lib, ctx, name, n_chains, steps):
    """Same uniforms, same decisions and configurations as the oracle's chains
    (determinants from scratch, dense traces); a chain whose decision lies
    within 1e-9 of its threshold is dropped from the comparison from then on."""
    from oracle import DenseTrace
    from oracle.markov import OracleChain
    from workloads.impurity import synthetic_bath

    tab, c = ctx(name)
    imp = make_impurity(name)
    eps, v = synthetic_bath(name)
    baths = [(eps[f], v[f]) for f in range(imp.n_flavors)]
    mc = lib.MarkovChains(c, n_chains, eps, v)
    dt = DenseTrace(imp)
    ref = [OracleChain(dt, baths) for _ in range(n_chains)]
    rng = np.random.Generator(np.random.PCG64(601))
    live = [True] * n_chains
    ties = accepted = 0
    say(f"[gpu] ctr_mc_step {name} {n_chains} chains x {steps} steps")
    for step in range(steps):
        u = rng.uniform(size=(n_chains, 6))
        dec = mc.step(u)
        for i in range(n_chains):
            if not live[i]:
                continue
            d, margin = ref[i].step(u[i])
            if abs(margin) < 1e-9:
                live[i] = False
                ties += 1
                continue
            assert dec[i] == d, (step, i, dec[i], d, margin)
            accepted += d == 1
        if step % 10 == 9 or step == steps - 1:
            for i in range(n_chains):
                if not live[i]:
                    continue
                tau, op, la_loc, la_hyb = mc.config(i)
                assert tau.tolist() == ref[i].tau and op.tolist() == ref[i].op, (step, i)
                assert abs(la_loc - ref[i].la_loc) <= 1e-10 * max(1.0, abs(ref[i].la_loc)), (step, i)
                assert abs(la_hyb - ref[i].la_hyb) <= 1e-8 * max(1.0, abs(ref[i].la_hyb)), (step, i)
    st = mc.stats()
    say(f"{name}: accepted {accepted}, ties {ties}, stats {st}, mean order "
        f"{np.mean([len(r.op) for r in ref]):.1f}")
    assert ties <= 2 and accepted >= n_chains * steps // 20
    mc.close()


def test_markov_chains_sample_the_anderson_impurity(lib):
    """The library's chains sample |w_loc w_hyb| of a two-flavor Anderson
    impurity; the N histogram averaged over them equals the occupation from
    exact diagonalisation of impurity plus bath (4 sigma over chains)."""
    from oracle.markov import anderson_occupation
    from paper_2010_08482_amd.sectors import build_sectors
    from tests.test_oracle_markov import anderson_two_flavor

    imp, baths = anderson_two_flavor()
    exact = anderson_occupation(imp, baths)
    tab = build_sectors(imp)
    c = lib.TraceContext(tab)
    n_chains = 512
    eps = np.array([b[0] for b in baths])
    v = np.array([b[1] for b in baths])
    mc = lib.MarkovChains(c, n_chains, eps, v)
    n_of_sector = np.array([bin(int(st[0])).count("1") for st in tab.states], dtype=np.int32)
    rng = np.random.Generator(np.random.PCG64(602))
    say(f"[gpu] ctr_mc_step anderson {n_chains} chains")
    for _ in range(300):
        mc.step(rng.uniform(size=(n_chains, 6)))
    sums = np.zeros(n_chains)
    n_meas = 0
    for step in range(600):
        mc.step(rng.uniform(size=(n_chains, 6)))
        if step % 5 == 0:
            cfgs = [mc.config(i)[:2] for i in range(n_chains)]
            offs, tau, op = pack([OperatorString(t, o) for t, o in cfgs])
            _, hist = c.histogram(offs, tau, op, n_of_sector, imp.n_flavors + 1)
            sums += np.real(hist @ np.arange(imp.n_flavors + 1))
            n_meas += 1
    per_chain = sums / n_meas
    est, err = per_chain.mean(), per_chain.std(ddof=1) / math.sqrt(n_chains)
    say(f"anderson: exact {exact:.5f}, chains {est:.5f} +- {err:.5f}, stats {mc.stats()}")
    assert abs(est - exact) < 4 * err + 1e-3
    mc.close()
    c.close()


def test_markov_chains_full_and_lazy_batches_decide_alike(lib, ctx):
    """Full trace batches with the decision on the host take the same
    decisions as lazy batches (a rejected bound implies a rejected value)."""
    from workloads.impurity import synthetic_bath

    tab, c = ctx("dshell")
    eps, v = synthetic_bath("dshell")
    strings = make_configs(1, 256)
    chains = [lib.MarkovChains(c, 256, eps, v, full_traces=f) for f in (False, True)]
    for mc in chains:
        for i, st in enumerate(strings):
            mc.set_config(i, st.tau, st.op)
    rng = np.random.Generator(np.random.PCG64(603))
    say("[gpu] ctr_mc_step dshell 256 chains x 30 steps, lazy and full batches")
    for _ in range(30):
        u = rng.uniform(size=(256, 6))
        d0, d1 = chains[0].step(u), chains[1].step(u)
        assert np.array_equal(d0, d1)
    for i in range(256):
        a, b = chains[0].config(i), chains[1].config(i)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        assert abs(a[2] - b[2]) <= 1e-12 * max(1.0, abs(b[2]))
    s0, s1 = chains[0].stats(), chains[1].stats()
    assert s0["accepted"] == s1["accepted"] > 0 and s1["lazy_rejected"] == 0 and s0["lazy_rejected"] > 0
    for mc in chains:
        mc.close()


def test_markov_chain_argument_errors(lib, ctx):
    from workloads.impurity import synthetic_bath

    tab, c = ctx("kanamori2")
    eps, v = synthetic_bath("kanamori2")
    mc = lib.MarkovChains(c, 4, eps, v)
    with pytest.raises(lib.CtraceError) as e:
        mc.step(np.full((4, 6), 1.0))
    assert e.value.status == -5  # uniforms must lie in [0, 1)
    with pytest.raises(lib.CtraceError):
        mc.set_config(0, [1.0, 2.0], [1, 3])  # unbalanced flavors
    with pytest.raises(lib.CtraceError):
        mc.set_config(0, [1.0, 2.0, 3.0, 4.0], [1, 1, 0, 0])  # flavor 0 not alternating
    mc.set_config(1, [1.0, 2.0], [1, 0])
    tau, op, la_loc, la_hyb = mc.config(1)
    assert tau.tolist() == [1.0, 2.0] and op.tolist() == [1, 0] and math.isfinite(la_loc) and math.isfinite(la_hyb)
    mc.close()


# ---------------------------------------------------------------------------
# density-matrix estimator (Sec. 2.3.2)
# ---------------------------------------------------------------------------

def _occupation_index_map(nf):
    """Builder state integer (bit f = flavor f) -> oracle index (flavor 0 most significant)."""
    return np.array([int(format(s, f"0{nf}b")[::-1], 2) for s in range(1 << nf)])


def _blocks_on_occupation_states(tab, blocks, rev):
    D = 1 << tab.n_flavors
    out = np.zeros((D, D), dtype=complex)
    for q, B in enumerate(blocks):
        st = rev[tab.states[q]]
        V = tab.vectors[q]
        out[np.ix_(st, st)] = V @ B @ V.conj().T
    return out


@pytest.mark.parametrize("name", ["kanamori2", "pshell", "pshell_cf"])
def test_density_matrix_vs_oracle(lib, name):
    """The estimator per configuration and summed over a weighted batch against
    the oracle's, compared as operators on the occupation states (both sides
    move their eigenbasis blocks there, so eigenvector phases and bases inside
    degenerate levels drop out).  Bar: 1e-10 of the largest entry plus 1e-12 of
    the configuration's cancellation ratio A / |w|."""
    from oracle import DenseTrace
    from oracle.observables import density_matrix
    from paper_2010_08482_amd.sectors import build_sectors

    imp = make_impurity(name)
    tab = build_sectors(imp, keep_vectors=True)
    dt = DenseTrace(imp)
    rev = _occupation_index_map(imp.n_flavors)
    rng = np.random.Generator(np.random.PCG64(707))
    strings = [OperatorString(np.zeros(0), np.zeros(0, dtype=np.int32))]
    strings += [random_string(rng, imp.n_flavors, imp.beta, 2 * int(rng.integers(1, 6)), "alternating")
                for _ in range(14)]
    c = lib.TraceContext(tab)
    try:
        refs = []
        for i, s in enumerate(strings):
            say(f"[gpu] ctr_density_matrix {name} configuration {i} (order {s.n})")
            out, blocks = c.density_matrix(np.array([0, s.n]), s.tau, s.op)
            R, w = density_matrix(dt, s.tau, s.op)
            got = _blocks_on_occupation_states(tab, blocks, rev)
            if w[0] == 0:
                assert np.all(got == 0)
                refs.append(None)
                continue
            ref = dt.V @ R @ dt.V.conj().T
            refs.append(ref)
            a, al = dt.abs_scale(s.tau, s.op)
            ratio = a / abs(complex(w[0])) * math.exp(al - w[1])
            err = np.max(np.abs(got - ref))
            assert err <= 1e-10 * np.max(np.abs(ref)) + 1e-12 * ratio, (i, err)
            assert abs(sum(np.trace(B) for B in blocks) - 1.0) <= 1e-10 + 1e-12 * ratio
        # a weighted batch: sum_C weight_C R(C)
        offs, tau, op = pack(strings)
        wts = rng.standard_normal(len(strings)) + 1j * rng.standard_normal(len(strings))
        say(f"[gpu] ctr_density_matrix {name} weighted batch of {len(strings)}")
        out, blocks = c.density_matrix(offs, tau, op, weight=wts)
        got = _blocks_on_occupation_states(tab, blocks, rev)
        ref = sum(wt * r for wt, r in zip(wts, refs) if r is not None)
        assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))
        assert sum(1 for r in refs if r is not None) >= 8
    finally:
        c.close()


def test_density_matrix_label_sums_match_histogram_dshell(lib, ctx):
    """Workload size (d-shell, 1024 states, beta = 50): the traces of every
    N-block of the estimator equal the valence histogram of the same
    configurations (a different kernel: interval times of the sector walk),
    and every estimator has trace 1."""
    tab, c = ctx("dshell")
    cfgs = make_configs(1, 24)
    n_of = np.array([bin(int(st[0])).count("1") for st in tab.states], dtype=np.int32)
    offs, tau, op = pack(cfgs)
    say("[gpu] valence histogram vs density-matrix blocks dshell x24")
    vals, hist = c.histogram(offs, tau, op, n_of, 11)
    for i, s in enumerate(cfgs):
        out, blocks = c.density_matrix(np.array([0, s.n]), s.tau, s.op)
        if vals[i]["re"] == 0:
            assert all(np.all(B == 0) for B in blocks)
            continue
        ratio = math.exp(float(vals[i]["log_abs"]) - float(vals[i]["log_scale"])) / abs(complex(vals[i]["re"], vals[i]["im"]))
        sums = np.zeros(11, dtype=complex)
        for q, B in enumerate(blocks):
            sums[n_of[q]] += np.trace(B)
        assert np.max(np.abs(sums - hist[i])) <= 1e-10 + 1e-12 * ratio, i
        assert abs(sums.sum() - 1.0) <= 1e-10 + 1e-12 * ratio


def test_grouped_rounds_as_one_graph(lib, ctx):
    """CTR_OPT_GRAPH: the rounds of every chunk launched as one HIP graph give
    the values of the round-by-round launches, bit for bit, call after call
    (eager calls in between), on the grouped wavefront, workgroup and
    row-chunked kernels and on the FP32-split items."""
    cases = [("dshell", make_configs(1, 300), lib.CTR_FP64, lib.CTR_KERNEL_GROUPED),
             ("fshell", make_configs(2, 60), lib.CTR_FP64, lib.CTR_KERNEL_GROUPED),
             ("fshell", make_configs(2, 60), lib.CTR_FP64, lib.CTR_KERNEL_GROUPED_ROWS),
             ("pshell", None, lib.CTR_FP32_SPLIT, lib.CTR_KERNEL_GROUPED)]
    rng = np.random.Generator(np.random.PCG64(808))
    for name, cfgs, prec, kern in cases:
        tab, c = ctx(name)
        if cfgs is None:
            cfgs = [random_string(rng, tab.n_flavors, tab.beta, 2 * int(rng.integers(0, 20)), "alternating")
                    for _ in range(120)]
        offs, tau, op = pack(cfgs)
        for rep in range(3):
            say(f"[gpu] graph vs eager rounds {name} kernel={kern} precision={prec} call {rep}")
            e = c.trace_packed(offs, tau, op, precision=prec, kernel=kern, slices=7 if prec else 0)
            g = c.trace_packed(offs, tau, op, precision=prec, kernel=kern, slices=7 if prec else 0,
                               flags=lib.CTR_OPT_GRAPH)
            for f in ("re", "im", "log_scale", "flags", "n_strings"):
                assert np.array_equal(e[f], g[f]), (name, f, rep)
