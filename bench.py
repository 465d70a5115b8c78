"""Throughput benchmark of the CT-HYB local trace on one MI355X.

One step = one pass of the whole trace path (sector-string walk, rotation,
lazy bounds, block-product chains, close, merge) over one batch of
configurations, inputs already resident in HBM.  The default workload is the
crystal-field f-shell: 14 flavors, 16384 states, Slater-Condon interaction,
spin-orbit coupling and a random Hermitian crystal field (sectors by N only,
largest block 3432), beta = 40, 2000 configurations at orders 60..200, complex
FP64; 200 configurations per step, so the 10 timed steps cover all 2000.
The d-shell (5-orbital Kanamori, 1024 states) and the f-shell (N, Jz)
workloads run as side legs in the same line.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--batch B] [--workload 1|2|3] [--no-cpu]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
# The paper's own acceleration figures (abstract and Sec. 4): whole CT-HYB runs of
# delta-Pu at 600 K, one NVIDIA Volta GPU with one CPU against one CPU, FP64.
# Reported beside the measurement as context only: another machine and another
# quantity (end-to-end solver time, not trace evaluations).
PAPER_CONTEXT = {
    "ctqmc_speedup_with_crystal_field": ">600x",
    "ctqmc_speedup_without_crystal_field": ">100x",
    "hardware": "Summit: 1 NVIDIA Volta GPU + 1 CPU vs 1 CPU",
    "precision": "FP64",
    "quantity": "whole CT-HYB solver, delta-Pu at 600 K (not trace evals/s)",
    "use": "context only",
}
PEAK_HBM_GBS = 8000.0

WORKLOADS = {
    1: dict(name="dshell-kanamori-10^4-orders20-80", impurity="dshell", config_id=1),
    2: dict(name="fshell-slater-soc-10^4-orders40-160", impurity="fshell", config_id=2),
    3: dict(name="fshell-slater-soc-cf-2000-orders60-200", impurity="fshell_cf", config_id=3),
}


def algorithmic_flops(tab, strings):
    """Flops the block method must do: for every surviving string rotated to its
    narrowest sector (width N), 2*N*d_out*d_in per block product (8x for
    complex); the first product (identity times a propagator: a copy) and the
    last operator (diagonal only) are not products."""
    dims = np.asarray(tab.dims, dtype=np.int64)
    nxt = np.asarray(tab.next)
    c = 8 if tab.is_complex else 2
    total = 0.0
    ns = tab.n_sectors
    for s in strings:
        n = s.n
        if n < 2:
            continue
        cur = np.arange(ns)
        alive = np.ones(ns, dtype=bool)
        seq = np.empty((n + 1, ns), dtype=np.int64)
        seq[0] = cur
        for p in range(n):
            nx = nxt[np.where(alive, cur, 0), s.op[p]]
            alive &= nx >= 0
            cur = np.where(alive, nx, 0)
            seq[p + 1] = cur
        alive &= cur == np.arange(ns)
        for q0 in np.nonzero(alive)[0]:
            path = seq[:n, q0]
            d = dims[path]
            j = int(np.argmin(d))
            width = int(d[j])
            dd = np.roll(d, -j)              # d at positions j, j+1, ..., j-1
            d_out = np.roll(dd, -1)
            # steps t = 1 .. n-2 are block products
            total += c * width * float(np.sum(dd[1:n - 1] * d_out[1:n - 1]))
    return total


def kernel_name(tab, kernel, slices):
    """Name of the chain kernel behind a CTR_KERNEL_* code the library reports
    for its last call (ctr_last_kernel): the grouped rounds keep every row of a
    block in one wavefront up to 32 (complex) / 128 (real) rows and in one
    workgroup up to 384, the row-chunked items cover any size."""
    xr = (tab.max_dim + 15) // 16 * 16
    if kernel == 4:
        return "k_gstep_wave" if xr <= (32 if tab.is_complex else 128) else "k_gstep"
    names = {1: "k_chain_wave", 2: "k_chain", 3: "k_chain_big", 5: "k_gbig"}
    name = names.get(kernel, f"kernel {kernel}")
    return name + ("_split" if slices and kernel == 5 else "")


# HBM-side bytes per launch of the dominant kernel (FETCH_SIZE + WRITE_SIZE from
# rocprofv3, scaled by the counters' reading for a plain 1 GiB device copy),
# per workload, valid only for the kernel source they were measured on: any
# change to that source makes the figure stale (reported as None).
TRAFFIC_MEASURED = {
    ("k_chain_wave", "dshell-kanamori-10^4-orders20-80, 10000 per step"): {
        "source": "ctrace_kernels.hip",
        "sha256": "3dc1033163cc10ec655db74d0593e1d526dcdbbb8b63403c0bc60f246ecfe420",
        "bytes": 1.4633e9},
    ("k_gbig", "fshell-slater-soc-cf-2000-orders60-200, 200 per step"): {
        "source": "ctrace_group.hip",
        "sha256": "d710a66bffc9cc6f77b33b6e8bee79d06a15acdf92fce1b463f65a884267d5ff",
        "bytes": 199.341e9},
    ("k_gstep", "fshell-slater-soc-10^4-orders40-160, 10000 per step"): {
        "source": "ctrace_group.hip",
        "sha256": "d710a66bffc9cc6f77b33b6e8bee79d06a15acdf92fce1b463f65a884267d5ff",
        "bytes": 26.513e9},
}


def measured_traffic(kernel, workload):
    import hashlib

    rec = TRAFFIC_MEASURED.get((kernel, workload))
    if not rec:
        return None
    src = os.path.join(ROOT, "paper_2010_08482_amd", "csrc", rec["source"])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    return rec["bytes"] if sha == rec["sha256"] else None


def lazy_leg(ctx, imp, strings, w_old):
    """Metropolis decisions on pair-insertion proposals (App. D moves, lazy
    trace of Sec. 3.3.1): each configuration is the old state, the proposal
    inserts one pair, and the threshold is r |w_old| with r ~ U(0,1) drawn
    first (every other acceptance factor taken as 1).  Times the lazy batch and
    the full batch on the same proposals, both through the host entry points."""
    from paper_2010_08482_amd import ctrace
    from workloads.configs import insert_pair, pack

    rng = np.random.Generator(np.random.PCG64(4242))
    props = [insert_pair(rng, s, imp.n_flavors, imp.beta) for s in strings]
    r = rng.uniform(0.0, 1.0, size=len(props))
    la_old = np.array([ctrace.log_abs(v) for v in w_old[: len(props)]])
    log_thr = np.where(np.isfinite(la_old), np.log(r) + la_old, -np.inf)
    offs, tau, op = pack(props)
    ctx.lazy_batch(offs, tau, op, log_thr)  # warm
    t0 = time.perf_counter()
    lz = ctx.lazy_batch(offs, tau, op, log_thr)
    t_lazy = time.perf_counter() - t0
    t0 = time.perf_counter()
    full = ctx.trace_packed(offs, tau, op)
    t_full = time.perf_counter() - t0
    la_new = np.array([ctrace.log_abs(v) for v in full])
    rej = (lz["flags"] & ctrace.CTR_FLAG_REJECTED) != 0
    should = la_new < log_thr
    return {"proposals": len(props), "rejected_frac": float(rej.mean()),
            "rejectable_frac": float(should.mean()),
            "false_rejections": int(np.sum(rej & ~should)),
            "decisions_per_s": len(props) / t_lazy, "full_traces_per_s": len(props) / t_full,
            "speedup": t_full / t_lazy, "entry": "ctr_trace_lazy_batch vs ctr_trace_batch (host arrays)"}


def histogram_leg(ctx, tab, imp, strings):
    """Valence histogram (Sec. 2.3.2 estimator summed over the sectors of each
    N, as in Sec. 4.2) of every configuration beside its trace, against the
    traces alone, both through the host entry points."""
    from workloads.configs import pack

    n_of_sector = np.array([bin(int(st[0])).count("1") for st in tab.states], dtype=np.int32)
    n_labels = imp.n_flavors + 1
    offs, tau, op = pack(strings)
    ctx.histogram(offs, tau, op, n_of_sector, n_labels)  # warm
    t0 = time.perf_counter()
    out, hist = ctx.histogram(offs, tau, op, n_of_sector, n_labels)
    t_hist = time.perf_counter() - t0
    t0 = time.perf_counter()
    ctx.trace_packed(offs, tau, op)
    t_tr = time.perf_counter() - t0
    dev = []
    for v, h in zip(out, hist):
        if v["re"] == 0 and v["im"] == 0:
            continue
        ratio = max(1.0, math.exp(v["log_abs"] - v["log_scale"] - math.log(abs(complex(v["re"], v["im"])))))
        dev.append(abs(h.sum() - 1.0) / ratio)
    return {"labels": "N", "n_labels": n_labels, "configurations": len(strings),
            "values_per_s": len(strings) / t_hist, "traces_only_per_s": len(strings) / t_tr,
            "overhead": t_hist / t_tr - 1.0,
            "max_sum_rule_dev_over_cancellation": float(max(dev)) if dev else None,
            "entry": "ctr_trace_histogram vs ctr_trace_batch (host arrays)"}


def markov_leg(ctx, wl_impurity, strings, n_chains, steps, full_traces=False):
    """Markov steps around the trace (App. D pair moves, w_hyb fast updates on
    the host, one trace batch per step on the GPU, lazy unless full_traces):
    n_chains chains start from the workload's configurations and make `steps`
    timed moves each."""
    from paper_2010_08482_amd import ctrace
    from workloads.impurity import synthetic_bath

    eps, v = synthetic_bath(wl_impurity)
    n_chains = min(n_chains, len(strings))
    mc = ctrace.MarkovChains(ctx, n_chains, eps, v, full_traces=full_traces)
    started = 0
    for i in range(n_chains):
        try:
            mc.set_config(i, strings[i].tau, strings[i].op)
            started += 1
        except ctrace.CtraceError:
            pass  # zero weight: the chain starts at order zero
    rng = np.random.Generator(np.random.PCG64(4343))
    for _ in range(3):
        mc.step(rng.uniform(size=(n_chains, 6)))
    s0 = mc.stats()
    h0, g0 = mc.timing()
    us = [rng.uniform(size=(n_chains, 6)) for _ in range(steps)]
    t0 = time.perf_counter()
    for u in us:
        mc.step(u)
    el = time.perf_counter() - t0
    s1 = mc.stats()
    h1, g1 = mc.timing()
    prop = s1["proposed"] - s0["proposed"]
    orders = [len(mc.config(i)[1]) for i in range(n_chains)]
    mc.close()
    return {"chains": n_chains, "started_from_workload": started, "steps": steps,
            "moves_per_s": n_chains * steps / el, "ms_per_step": el / steps * 1e3,
            "accepted_frac": (s1["accepted"] - s0["accepted"]) / max(prop, 1),
            "lazy_rejected_frac": (s1["lazy_rejected"] - s0["lazy_rejected"]) / max(prop, 1),
            "mean_order": float(np.mean(orders)),
            "host_ms_per_step": (h1 - h0) / steps, "trace_batch_ms_per_step": (g1 - g0) / steps,
            "entry": "ctr_mc_step (host hybridisation updates + one " +
                     ("ctr_trace_batch" if full_traces else "ctr_trace_lazy_batch") + " per step)"}


def cpu_baseline(imp, strings, seconds_budget=20.0):
    """The CPU oracle (dense full-space FP64 chain) on a bounded sample."""
    from threadpoolctl import threadpool_info

    from oracle import DenseTrace

    dt = DenseTrace(imp)
    done = []
    t0 = time.perf_counter()
    for s in strings:
        done.append(dt.trace(s.tau, s.op))
        if time.perf_counter() - t0 > seconds_budget:
            break
    el = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info() if p.get("internal_api") in
                   ("openblas", "mkl", "blis")] or [1])
    return len(done) / el, len(done), el, threads, done


def cpu_oracle_extrapolated(tab, strings, probe_dim=2048):
    """The dense CPU oracle's cost on a full-size impurity, extrapolated: it
    multiplies one 2^n x 2^n matrix per operator, so a trace costs the mean
    operator count times one such product, timed here at probe_dim and scaled
    by (2^n / probe_dim)^3.  Labelled as extrapolated."""
    from threadpoolctl import threadpool_info

    D = 1 << tab.n_flavors
    dtype = np.complex128 if tab.is_complex else np.float64
    rng = np.random.Generator(np.random.PCG64(5))
    a = rng.standard_normal((probe_dim, probe_dim)).astype(dtype)
    b = rng.standard_normal((probe_dim, probe_dim)).astype(dtype)
    a @ b  # warm
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        a @ b
    t_probe = (time.perf_counter() - t0) / reps
    t_product = t_probe * (D / probe_dim) ** 3
    mean_ops = float(np.mean([s.n for s in strings]))
    threads = max([p.get("num_threads", 1) for p in threadpool_info() if p.get("internal_api") in
                   ("openblas", "mkl", "blis")] or [1])
    return {"value": 1.0 / (t_product * mean_ops), "unit": "trace evals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"extrapolated: the dense oracle's step (one {D}x{D} {'complex' if tab.is_complex else 'real'} "
                      f"product per operator) timed at {probe_dim}^3 ({t_probe * 1e3:.1f} ms, 3 repeats) and scaled by "
                      f"({D}/{probe_dim})^3, x {mean_ops:.0f} operators per trace (mean of the workload); one "
                      f"2^14-state trace takes hours on the host"}


def cpu_block_sparse(tab, strings, seconds_budget=5.0):
    """The same sector-block algorithm (walk, block products, trace) in NumPy
    FP64 on the host (the tests' block reference), on a bounded sample: with
    every BLAS thread and with one, the paper's GPU-versus-one-core setting."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from tests.blockref import block_trace

    def run():
        n, t0 = 0, time.perf_counter()
        for s in strings:
            block_trace(tab, s.tau, s.op)
            n += 1
            if time.perf_counter() - t0 > seconds_budget:
                break
        return n, time.perf_counter() - t0

    n_all, el_all = run()
    threads = max([p.get("num_threads", 1) for p in threadpool_info() if p.get("internal_api") in
                   ("openblas", "mkl", "blis")] or [1])
    with threadpool_limits(limits=1):
        n_one, el_one = run()
    return {"value_all_cores": n_all / el_all, "cores": threads, "value_one_core": n_one / el_one,
            "unit": "trace evals/s", "kind": "block-sparse NumPy (tests/blockref.py)",
            "sample": f"first {n_all} / {n_one} configurations, {el_all:.1f} s / {el_one:.1f} s"}


def serve_main(args, emit: bool = True):
    """Serving mix: 256 Markov chains spread over the d-shell, f-shell (N, Jz)
    and crystal-field f-shell impurities (62.5 / 25 / 12.5%; without the
    crystal field 75 / 25%); trace requests arrive as a Poisson stream, each
    the chain's configuration after one pair insertion or removal (App. D
    moves), orders starting from N(100, 30) clipped to [2, 240].  A chain has
    at most one request in flight (its next move depends on the decision): an
    arrival that picks a chain whose proposal is still on the GPU makes no
    move (counted).  Admission per impurity by arena footprint (hbm_budget), a
    stream and a grid share per impurity.  Reports throughput and latency
    percentiles per impurity from submission to result.  Prints one JSON line."""
    import threading

    import torch

    from paper_2010_08482_amd import ctrace
    from paper_2010_08482_amd.sectors import build_sectors
    from workloads import make_impurity
    from workloads.configs import insert_pair, random_string, remove_pair

    names = ["dshell", "fshell"] + (["fshell_cf"] if args.serve_cf else [])
    chain_share = [0.75, 0.25] if not args.serve_cf else [0.625, 0.25, 0.125]
    imps = [make_impurity(n) for n in names]
    free, _ = torch.cuda.mem_get_info(0)
    budget = int(args.serve_budget_gib * (1 << 30))
    ctxs = []
    for imp in imps:
        tab = build_sectors(imp)
        print(f"[serve] {imp.name}: {tab.n_sectors} sectors, largest block {tab.max_dim}", file=sys.stderr, flush=True)
        # a stream per impurity, so that the lanes' passes overlap on the device
        ctxs.append(ctrace.TraceContext(tab, scratch_bytes=int(min(free // (4 * len(imps)), max(budget, 1 << 30) + (1 << 30))),
                                        stream=torch.cuda.Stream()))
    rng = np.random.Generator(np.random.PCG64(2024))
    n_chains = 256
    kind = rng.choice(len(names), size=n_chains, p=chain_share)
    chains = []
    for c in range(n_chains):
        imp = imps[kind[c]]
        n = int(np.clip(round(rng.normal(100.0, 30.0) / 2) * 2, 2, 240))
        chains.append(random_string(rng, imp.n_flavors, imp.beta, n, "alternating"))
    n_arr = int(args.serve_rate * args.serve_seconds)
    t_arr = np.cumsum(rng.exponential(1.0 / args.serve_rate, size=n_arr))
    c_arr = rng.integers(n_chains, size=n_arr)
    mrng = np.random.Generator(np.random.PCG64(2025))  # moves, in issue order
    reqs = []   # (chain, impurity, string), in issue order
    share = [float(x) for x in args.serve_grid_share.split(",")] if args.serve_grid_share else None
    if share is not None:
        share = (share + [1.0] * len(names))[: len(names)]
    srv = ctrace.TraceServer(ctxs, max_batch=args.serve_batch, hbm_budget=budget, grid_share=share,
                             max_pass_flop=args.serve_max_pass_gflop * 1e9)
    results = []
    lock = threading.Lock()
    busy_chain = np.zeros(n_chains, dtype=bool)
    dropped = 0
    done = threading.Event()

    def collect():
        while True:
            r = srv.poll(max_results=8192, wait=True)
            if len(r) == 0:
                if done.is_set():
                    break
                time.sleep(2e-4)  # nothing in flight
                continue
            rows = r.tolist()
            with lock:
                results.extend(rows)
                for row in rows:
                    busy_chain[reqs[int(row[0])][0]] = False

    poller = threading.Thread(target=collect)
    poller.start()
    t0 = time.perf_counter()
    for a in range(n_arr):
        while time.perf_counter() - t0 < t_arr[a]:
            pass
        c = int(c_arr[a])
        with lock:
            if busy_chain[c]:
                # the chain's previous proposal is still being decided: no new move from it
                dropped += 1
                continue
            busy_chain[c] = True
        imp = imps[kind[c]]
        s = chains[c]
        if s.n <= 2 or (s.n + 2 <= 240 and mrng.uniform() < 0.5):
            s = insert_pair(mrng, s, imp.n_flavors, imp.beta)
        else:
            s = remove_pair(mrng, s, imp.n_flavors)
        chains[c] = s
        i = len(reqs)
        reqs.append((c, int(kind[c]), s))
        while srv.submit(int(kind[c]), i, s.tau, s.op) == ctrace.CTR_ERR_BUSY:
            pass
    t_sub = time.perf_counter() - t0
    srv.drain()
    t_end = time.perf_counter() - t0
    done.set()
    poller.join()
    results.extend(srv.poll(max_results=8192).tolist())
    passes, evaluated = srv.stats()
    srv.close()
    n_req = len(reqs)
    lat = np.array([r[4] for r in results])
    imp_of = np.array([r[1] for r in results])
    bat = np.array([r[5] for r in results])
    per = {}
    for k, n in enumerate(names):
        m = imp_of == k
        if m.any():
            per[n] = {"requests": int(m.sum()), "p50_ms": float(np.percentile(lat[m], 50)),
                      "p99_ms": float(np.percentile(lat[m], 99)), "mean_batch": float(bat[m].mean()),
                      "chains": int(np.sum(kind == k))}
    line = {
        "metric": "serving: trace requests/s with p50/p99 latency (continuous batching)",
        "value": len(results) / t_end,
        "unit": "trace evals/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "offered_rate": args.serve_rate,
        "arrivals": n_arr,
        "arrivals_on_busy_chains": dropped,
        "submit_seconds": t_sub,
        "seconds": t_end,
        "requests": n_req,
        "completed": len(results),
        "statuses_ok": int(sum(1 for r in results if r[2] == 0)),
        "device_passes": passes,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "from": "ctr_server_submit to result"},
        "per_impurity": per,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "serving mix: 256 Markov chains, Poisson arrivals, pair insert/remove moves, "
                               "one request in flight per chain",
                   "impurities": names, "chain_share": chain_share, "max_batch": args.serve_batch,
                   "hbm_budget_bytes": budget, "grid_share": share, "streams": "one per impurity",
                   "max_pass_gflop": args.serve_max_pass_gflop or None},
    }
    for c in ctxs:
        c.close()
    if emit:
        print(json.dumps(line), flush=True)
    return line


def _rel_errors(a, b):
    """Relative differences |a - b| / |b| and against the cancellation scale
    exp(log_abs) of b, over the configurations where b is nonzero."""
    rel, rel_a = [], []
    for x, y in zip(a, b):
        if y["re"] == 0 and y["im"] == 0:
            continue
        M = max(x["log_scale"], y["log_scale"])
        u = complex(x["re"], x["im"]) * math.exp(x["log_scale"] - M)
        v = complex(y["re"], y["im"]) * math.exp(y["log_scale"] - M)
        rel.append(abs(u - v) / abs(v))
        rel_a.append(abs(u - v) / math.exp(y["log_abs"] - M))
    return np.array(rel), np.array(rel_a)


def _dist(x):
    return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99)), "max": float(x.max()),
            "n": int(x.size)} if x.size else None


def throughput_leg(wl_id, n_configs, batch, steps, warmup, kernel_opt, split_configs, split_slices, lazy_sample,
                   no_cpu, headline):
    """FP64 throughput of one workload through the device entry point (inputs
    resident in HBM): `steps` timed steps, step k evaluating batch k (cycling)
    of `batch` configurations; chain-kernel time from HIP events on the
    library's stream; the roofline of the dominant kernel; an FP32-split leg on
    the first `split_configs` configurations; a lazy leg; the CPU oracle."""
    import torch

    from paper_2010_08482_amd import ctrace
    from paper_2010_08482_amd.sectors import build_sectors
    from workloads import make_configs, make_impurity
    from workloads.configs import pack

    wl = WORKLOADS[wl_id]
    imp = make_impurity(wl["impurity"])
    tab = build_sectors(imp)
    strings = make_configs(wl["config_id"], n_configs or None)
    n_cfg = len(strings)
    B = min(batch or n_cfg, n_cfg)
    n_batches = (n_cfg + B - 1) // B
    name = wl["name"] if not n_configs else f"{wl['name']} (first {n_cfg})"
    covered = min(steps, n_batches) * B
    print(f"[bench] {name}: {n_cfg} configurations, {tab.n_sectors} sectors, largest block {tab.max_dim}, "
          f"{B} per step", file=sys.stderr, flush=True)
    free, _ = torch.cuda.mem_get_info(0)
    # per-call scratch: the grouped rounds keep every surviving string's carried matrix resident
    ctx = ctrace.TraceContext(tab, scratch_bytes=int(min(free * 0.55, 150 << 30)))
    peaks = ctrace.ctr_probe_peaks(ctx.ctx) if headline else None
    offs, tau, op = pack(strings)
    dev = "cuda:0"
    d_offs, d_tau, d_op = (torch.from_numpy(a).to(dev) for a in (offs, tau, op))
    vsz = ctrace.VALUE_DTYPE.itemsize
    d_out = torch.zeros(n_cfg * vsz, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def run(b, precision=ctrace.CTR_FP64, out=None, count=None, slices=0):
        c0 = (b % n_batches) * B
        m = min(B, n_cfg - c0) if count is None else count
        ctrace.ctr_trace_batch_device(ctx.ctx, m, d_offs.data_ptr() + 8 * c0, d_tau.data_ptr(), d_op.data_ptr(),
                                      (out if out is not None else d_out).data_ptr() + vsz * c0, precision,
                                      kernel_opt if precision == ctrace.CTR_FP64 else ctrace.CTR_KERNEL_AUTO, slices)
        return m

    for k in range(warmup):
        run(k)
        torch.cuda.synchronize()
        print(f"[bench] warmup step {k + 1}/{warmup} done", file=sys.stderr, flush=True)
    ctrace.ctr_kernel_timing(ctx.ctx, True)
    ctrace.ctr_kernel_timing_read(ctx.ctx)
    torch.cuda.synchronize()
    done = 0
    t0 = time.perf_counter()
    for k in range(steps):
        done += run(k)
        # progress (host side: the grouped rounds wait once per batch for their schedule)
        print(f"[bench] step {k + 1}/{steps} enqueued ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    chain_ms, launches = ctrace.ctr_kernel_timing_read(ctx.ctx)
    ctrace.ctr_kernel_timing(ctx.ctx, False)
    kcode, _ = ctrace.ctr_last_kernel(ctx.ctx)
    kname = kernel_name(tab, kcode, 0)
    flops = sum(algorithmic_flops(tab, strings[(k % n_batches) * B:(k % n_batches) * B + B]) for k in range(steps))
    out = np.frombuffer(d_out.cpu().numpy().tobytes(), dtype=ctrace.VALUE_DTYPE)
    print(f"[bench] {steps} steps in {elapsed:.3f}s; {kname} {chain_ms / max(launches, 1):.3f} ms per launch over "
          f"{launches} launches", file=sys.stderr, flush=True)
    per_launch = chain_ms / max(launches, 1)
    achieved = flops / (chain_ms * 1e-3) / 1e12 if chain_ms > 0 else None
    workload_key = f"{name}, {B} per step"
    rec = {
        "value": done / elapsed, "unit": "trace evals/s", "steps": steps, "warmup": warmup,
        "ms_per_step": elapsed / steps * 1e3, "dtype": "c128" if tab.is_complex else "f64",
        "config": {"workload": workload_key + (f", {steps} steps cover {covered} of {n_cfg}" if steps else ""),
                   "impurity": wl["impurity"], "n_configs": n_cfg, "configs_per_step": B,
                   "sectors": int(tab.n_sectors), "largest_block": int(tab.max_dim), "beta": tab.beta,
                   "complex": bool(tab.is_complex), "precision": "FP64"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS if achieved else None,
                     "traffic": measured_traffic(kname, workload_key), "kernel": kname,
                     "algorithmic_flop_per_launch": flops / max(launches, 1), "launch_ms": per_launch,
                     "launches": launches, "chain_ms": chain_ms},
        "measured_peaks": peaks,
    }

    if split_configs:
        # FP32-split leg: block products on FP32 MFMA over exact 8-bit slices, first configurations
        m = min(split_configs, n_cfg)
        print(f"[bench] FP32-split leg: {m} configurations", file=sys.stderr, flush=True)
        d_s = torch.zeros_like(d_out)
        d_f = torch.zeros_like(d_out)
        run(0, ctrace.CTR_FP64, d_f, m)
        run(0, ctrace.CTR_FP32_SPLIT, d_s, m, split_slices)
        torch.cuda.synchronize()
        ctrace.ctr_kernel_timing(ctx.ctx, True)
        ctrace.ctr_kernel_timing_read(ctx.ctx)
        ts = time.perf_counter()
        run(0, ctrace.CTR_FP32_SPLIT, d_s, m, split_slices)
        torch.cuda.synchronize()
        el_s = time.perf_counter() - ts
        ms_s, n_s = ctrace.ctr_kernel_timing_read(ctx.ctx)
        ctrace.ctr_kernel_timing(ctx.ctx, False)
        ks, sl = ctrace.ctr_last_kernel(ctx.ctx)
        outs = np.frombuffer(d_s.cpu().numpy().tobytes(), dtype=ctrace.VALUE_DTYPE)[:m]
        outf = np.frombuffer(d_f.cpu().numpy().tobytes(), dtype=ctrace.VALUE_DTYPE)[:m]
        rel_s, rel_a = _rel_errors(outs, outf)
        fl = algorithmic_flops(tab, strings[:m])
        per = fl / (ms_s * 1e-3) / 1e12 if ms_s > 0 else 0.0
        nprod = sl * (sl + 1) // 2
        rec["fp32_split"] = {
            "value": m / el_s, "unit": "trace evals/s", "configurations": m, "slice_bits": 8, "slices": sl,
            "kernel": kernel_name(tab, ks, sl), "fp32_products_per_fma": nprod, "chain_ms": ms_s,
            "achieved_fp64_equivalent_tflops": per,
            # the slice products the method needs (nprod FP32 products per FP64 multiply-add)
            "needed_fp32_tflops": nprod * per, "frac_fp32_peak": nprod * per / 157.3,
            "rel_err_vs_fp64": _dist(rel_s), "err_vs_fp64_over_abs_sum": _dist(rel_a),
            "meets_1e-10": bool(np.all((rel_s <= 1e-10) | (rel_a <= 1e-12))) if rel_s.size else None}

    if lazy_sample:
        lz = strings[:lazy_sample]
        print(f"[bench] lazy leg: {len(lz)} proposals", file=sys.stderr, flush=True)
        full = ctx.trace_batch(lz)
        rec["lazy"] = lazy_leg(ctx, imp, lz, full)

    if not no_cpu:
        print("[bench] CPU baselines", file=sys.stderr, flush=True)
        if wl_id == 1:
            sample = strings[:24]
            rate, got, el, threads, refs = cpu_baseline(imp, sample)
            rec["cpu_baseline"] = {"value": rate, "unit": "trace evals/s", "cores": threads, "kind": "oracle",
                                   "sample": f"first {got} of the {n_cfg} configurations, dense 2^10-dim FP64 "
                                             f"chain, {el:.1f} s"}
            errs = []
            for v, ref in zip(out[:got], refs):
                if ref[0] == 0:
                    continue
                M = max(v["log_scale"], ref[1])
                a = complex(v["re"], v["im"]) * math.exp(v["log_scale"] - M)
                b = complex(ref[0]) * math.exp(ref[1] - M)
                errs.append(abs(a - b) / abs(b))
            rec["rel_err_vs_oracle_sample"] = _dist(np.array(errs))
            rec["cpu_block_sparse"] = cpu_block_sparse(tab, strings)
        else:
            # a 2^14-state dense trace takes hours on the host: the oracle's cost per
            # operator is timed on a smaller product and scaled (labelled extrapolated)
            rec["cpu_baseline"] = cpu_oracle_extrapolated(tab, strings)
    ctx.close()
    return name, rec


def dshell_extras(args):
    """The d-shell workload's other legs: valence histogram, Markov chains
    (lazy and full trace batches), single-configuration latency."""
    from paper_2010_08482_amd import ctrace
    from paper_2010_08482_amd.sectors import build_sectors
    from workloads import make_configs, make_impurity

    imp = make_impurity("dshell")
    tab = build_sectors(imp)
    strings = make_configs(1)
    ctx = ctrace.TraceContext(tab, scratch_bytes=8 << 30)
    print("[bench] d-shell histogram, Markov and latency legs", file=sys.stderr, flush=True)
    rec = {"histogram": histogram_leg(ctx, tab, imp, strings)}
    if args.mc_chains > 0:
        mk = markov_leg(ctx, "dshell", strings, args.mc_chains, args.mc_steps)
        mk["full_traces"] = markov_leg(ctx, "dshell", strings, args.mc_chains, args.mc_steps, True)
        rec["markov"] = mk
    lat = []
    for s in strings[: args.latency_sample]:
        t = time.perf_counter()
        ctx.trace(s.tau, s.op)
        lat.append((time.perf_counter() - t) * 1e3)
    if lat:
        rec["latency_ms"] = {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                             "entry": "ctr_trace (one configuration, host pointers)"}
    ctx.close()
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=3, choices=sorted(WORKLOADS))
    ap.add_argument("--batch", type=int, default=-1,
                    help="configurations per step (-1: 200 for the crystal-field f-shell, all otherwise)")
    ap.add_argument("--n-configs", type=int, default=0, help="use only the first N configurations (0 = all)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--latency-sample", type=int, default=200)
    ap.add_argument("--split-configs", type=int, default=-1,
                    help="configurations of the FP32-split leg (-1: 16 crystal-field, 2000 f-shell, all d-shell; 0 = skip)")
    ap.add_argument("--split-slices", type=int, default=7, choices=[6, 7],
                    help="8-bit slices per operand of the FP32-split leg")
    ap.add_argument("--lazy-sample", type=int, default=-1,
                    help="pair-insertion proposals of the lazy leg (-1: 100 crystal-field, all otherwise; 0 = skip)")
    ap.add_argument("--mc-chains", type=int, default=4096, help="chains of the d-shell Markov leg (0 = skip)")
    ap.add_argument("--mc-steps", type=int, default=20, help="timed steps of the Markov leg")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="copy this many MiB once with a plain device copy (HBM counter calibration)")
    ap.add_argument("--kernel", default="auto", choices=["auto", "wave", "block", "stream", "grouped", "grouped_rows"],
                    help="chain kernel of the timed FP64 steps (default: the library's automatic choice)")
    ap.add_argument("--no-also", action="store_true", help="skip the side legs (d-shell, f-shell (N, Jz), serving)")
    ap.add_argument("--serve", action="store_true", help="run the serving mix instead of the throughput step")
    ap.add_argument("--serve-no-cf", dest="serve_cf", action="store_false",
                    help="serving mix: leave out the crystal-field f-shell")
    ap.add_argument("--serve-budget-gib", type=float, default=8.0,
                    help="serving mix: arena bytes (GiB) one impurity's device pass may occupy")
    ap.add_argument("--serve-rate", type=float, default=5e4, help="serving mix: Poisson arrival rate (1/s)")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="serving mix: seconds of arrivals")
    ap.add_argument("--serve-batch", type=int, default=4096, help="serving mix: most requests per device pass")
    ap.add_argument("--serve-grid-share", default="1,1,0.5",
                    help="serving mix: per-impurity fractions of the persistent grids ('' = full grids)")
    ap.add_argument("--serve-max-pass-gflop", type=float, default=0.0,
                    help="serving mix: cap on one pass's estimated block-product GFLOP (0 = no cap)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: every run here has a single MI355X and the trace path has no "
              "multi-GPU leg; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.serve:
        serve_main(args)
        return

    import torch

    from paper_2010_08482_amd import ctrace

    kernel = {"auto": ctrace.CTR_KERNEL_AUTO, "wave": ctrace.CTR_KERNEL_WAVE, "block": ctrace.CTR_KERNEL_BLOCK,
              "stream": ctrace.CTR_KERNEL_STREAM, "grouped": ctrace.CTR_KERNEL_GROUPED,
              "grouped_rows": ctrace.CTR_KERNEL_GROUPED_ROWS}[args.kernel]
    if args.calib_copy_mib:
        src = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def defaults(wl_id):
        batch = args.batch if args.batch >= 0 else (200 if wl_id == 3 else 0)
        split = args.split_configs if args.split_configs >= 0 else {1: 10_000, 2: 2000, 3: 16}[wl_id]
        lazy = args.lazy_sample if args.lazy_sample >= 0 else (100 if wl_id == 3 else 10_000)
        return batch, split, lazy

    batch, split_n, lazy_n = defaults(args.workload)
    name, rec = throughput_leg(args.workload, args.n_configs, batch, args.steps, args.warmup, kernel, split_n,
                                  args.split_slices, lazy_n, args.no_cpu, True)
    line = {
        "metric": "trace evals/sec + MFMA % peak (FP32-split vs FP64) at <=1e-10 rel err; p50/p99",
        "value": rec["value"],
        "unit": "trace evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": rec["dtype"],
        "data": "synthetic",
        "config": rec["config"],
        "roofline": rec["roofline"],
        "cpu_baseline": rec.get("cpu_baseline"),
        "measured_peaks": rec["measured_peaks"],
        "fp32_split": rec.get("fp32_split"),
        "lazy": rec.get("lazy"),
        "paper_context": PAPER_CONTEXT,
    }
    for k in ("cpu_block_sparse", "rel_err_vs_oracle_sample"):
        if k in rec:
            line[k] = rec[k]
    if not args.no_also:
        also = {}
        for wl_id in (1, 2):
            if wl_id == args.workload:
                continue
            b, sp, lz = defaults(wl_id)
            n, r = throughput_leg(wl_id, 0, b, 3, 1, ctrace.CTR_KERNEL_AUTO, sp, args.split_slices, lz,
                                     args.no_cpu, False)
            r.pop("measured_peaks", None)
            also[n] = r
        try:
            also["dshell extras"] = dshell_extras(args)
        except Exception as e:  # reported in the line; the measurements above stand
            also["dshell extras"] = {"error": f"{type(e).__name__}: {e}"}
        line["also"] = also
        # the serving mix (bench.py --serve for other settings)
        sargs = argparse.Namespace(**vars(args))
        print("[bench] serving mix", file=sys.stderr, flush=True)
        try:
            sv = serve_main(sargs, emit=False)
            line["serving"] = {k: sv[k] for k in ("value", "unit", "offered_rate", "completed", "statuses_ok",
                                                  "device_passes", "latency_ms", "per_impurity", "config")}
        except Exception as e:  # reported in the line; the trace measurement above stands
            line["serving"] = {"error": f"{type(e).__name__}: {e}"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
