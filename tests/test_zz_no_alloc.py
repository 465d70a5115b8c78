"""The allocation-free entry point (ctr_trace_batch_device_static) against
the arena entry point it shares its kernels with, through the C ABI: two
calls in a row, the second smaller, on a real (d-shell, wavefront kernel)
and a complex (p-shell, LDS workgroup kernel) impurity; stored oracle values
on the d-shell batch; an oversized batch is refused before any device work."""

import json
import os

import numpy as np
import pytest

from tests.tracecmp import close_enough, rel_err
from workloads import make_configs, make_impurity
from workloads.configs import pack

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)


def _on_device(lib, strings, dev):
    import torch

    offs, tau, op = pack(strings)
    d = [torch.from_numpy(a).to(dev) for a in (offs, tau, op)]
    out = torch.zeros(len(strings) * lib.VALUE_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    return d, out


def _read(lib, c, out):
    c.synchronize()
    return np.frombuffer(out.cpu().numpy().tobytes(), dtype=lib.VALUE_DTYPE).copy()


def _run(lib, c, strings, static):
    (o, t, p), out = _on_device(lib, strings, f"cuda:{c.device}")
    fn = lib.ctr_trace_batch_device_static if static else lib.ctr_trace_batch_device
    fn(c.ctx, len(strings), o.data_ptr(), t.data_ptr(), p.data_ptr(), out.data_ptr())
    return _read(lib, c, out)


def _same(a, b, label):
    assert np.array_equal(a["flags"], b["flags"]) and np.array_equal(a["n_strings"], b["n_strings"]), label
    worst = 0.0
    for x, y in zip(a, b):
        if y["re"] == 0 and y["im"] == 0:
            assert x["re"] == 0 and x["im"] == 0, label
            continue
        gx = (complex(x["re"], x["im"]), float(x["log_scale"]))
        gy = (complex(y["re"], y["im"]), float(y["log_scale"]))
        worst = max(worst, rel_err(gx, gy))
    say(f"{label}: {len(a)} traces, worst rel diff {worst:.2e}")
    assert worst <= 1e-10


@pytest.mark.parametrize("name,cid,n1,n2", [("dshell", 1, 3000, 700), ("pshell", None, 400, 90)])
def test_static_scratch_matches_arena_entry_point(name, cid, n1, n2):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_08482_amd import ctrace as lib
    from paper_2010_08482_amd.sectors import build_sectors

    tab = build_sectors(make_impurity(name))
    c = lib.TraceContext(tab)
    try:
        if cid is not None:
            cfgs = make_configs(cid, n1)
        else:
            from workloads.configs import random_string

            rng = np.random.Generator(np.random.PCG64(606))
            cfgs = [random_string(rng, tab.n_flavors, tab.beta, 2 * int(rng.integers(0, 20)), "alternating")
                    for _ in range(n1)]
        for label, strings in (("first call", cfgs), ("second call, smaller", cfgs[::-1][:n2])):
            say(f"[gpu] {name} {label}: static and arena entry points, {len(strings)} configurations")
            got = _run(lib, c, strings, True)
            ref = _run(lib, c, strings, False)
            _same(got, ref, f"{name} {label}")
        if name == "dshell":
            g = json.load(open(os.path.join(HERE, "golden", "dshell_config1.json")))
            recs = g["records"]
            say(f"[gpu] dshell static entry point vs stored oracle values ({len(recs)})")
            got = _run(lib, c, make_configs(1, len(recs)), True)
            for v, r in zip(got, recs):
                ref = (complex(r["re"], r["im"]), r["log_scale"])
                if ref[0] == 0:
                    assert v["re"] == 0 and v["im"] == 0
                    continue
                assert close_enough((complex(v["re"], v["im"]), float(v["log_scale"])), ref, (r["abs"], r["abs_log"]))
        # a batch beyond the static array is refused before any device work
        per = 1 + lib.CTR_STATIC_SCRATCH_BYTES // 1024
        big = (cfgs * (per // len(cfgs) + 1))[:per]
        say(f"[gpu] {name}: oversized batch of {len(big)} configurations")
        (o, t, p), out = _on_device(lib, big, f"cuda:{c.device}")
        with pytest.raises(lib.CtraceError) as e:
            lib.ctr_trace_batch_device_static(c.ctx, len(big), o.data_ptr(), t.data_ptr(), p.data_ptr(), out.data_ptr())
        assert e.value.status == -2 and "static array" in str(e.value)
    finally:
        c.close()
