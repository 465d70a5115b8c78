"""Comparison helpers for traces given as (mantissa, log_scale) pairs,
value = mantissa * exp(log_scale).  Shared by the tests only."""

import math

import numpy as np


def aligned(a, b):
    """Both values scaled by a common exp(-M) so they can be subtracted."""
    (ma, la), (mb, lb) = a, b
    if ma == 0 and mb == 0:
        return 0.0, 0.0
    if ma == 0:
        return 0.0, complex(mb)
    if mb == 0:
        return complex(ma), 0.0
    M = max(la, lb)
    return complex(ma) * math.exp(la - M), complex(mb) * math.exp(lb - M)


def rel_err(got, ref):
    """|got - ref| / |ref| (inf if ref is zero and got is not)."""
    g, r = aligned(got, ref)
    if r == 0:
        return 0.0 if g == 0 else math.inf
    return abs(g - r) / abs(r)


def add(a, b):
    (ma, la), (mb, lb) = a, b
    if ma == 0:
        return b
    if mb == 0:
        return a
    M = max(la, lb)
    return complex(ma) * math.exp(la - M) + complex(mb) * math.exp(lb - M), M


def to_float(a):
    m, l = a
    return complex(m) * math.exp(l)


def insert_ops(tau, op, t_new, codes):
    """Insert operators 'codes' (in array order) at time t_new."""
    tau = np.asarray(tau, dtype=np.float64)
    op = np.asarray(op, dtype=np.int64)
    pos = int(np.searchsorted(tau, t_new, side="right"))
    k = len(codes)
    return (np.concatenate([tau[:pos], [t_new] * k, tau[pos:]]),
            np.concatenate([op[:pos], codes, op[pos:]]))


def close_enough(got, ref, scale, rtol=1e-10, atol_scale=1e-12):
    """Parity bar: |got - ref| <= rtol |ref|, or, for cancellation-dominated
    traces, |got - ref| <= atol_scale * A where A (same log units) is the sum
    of moduli of the Lehmann terms (see DenseTrace.abs_scale)."""
    g, r = aligned(got, ref)
    diff = abs(g - r)
    if diff <= rtol * abs(r):
        return True
    (ma, la) = scale
    M = max(got[1] if got[0] != 0 else -math.inf, ref[1] if ref[0] != 0 else -math.inf)
    if ma == 0 or M == -math.inf:
        return diff == 0
    return diff <= atol_scale * ma * math.exp(la - M)
