"""Test-side helpers: rounding to the storage precisions (written from the IEEE definitions, not
taken from the library) and small seeded structures."""

import numpy as np

import wfq_inputs as wi
from wfq_inputs import geometry as geo


def round_bf16(x):
    """Round float64 values to bfloat16 (nearest, ties to even) and return them as float64."""
    x = np.asarray(x, dtype=np.float64)
    bits = x.view(np.uint64)
    sign = bits >> np.uint64(63)
    exp = (bits >> np.uint64(52)) & np.uint64(0x7FF)
    mant = bits & np.uint64((1 << 52) - 1)
    keep = mant >> np.uint64(45)
    rest = mant & np.uint64((1 << 45) - 1)
    half = np.uint64(1 << 44)
    up = (rest > half) | ((rest == half) & ((keep & np.uint64(1)) == np.uint64(1)))
    # value = 2^(e-1023) * (1 + keep/128), plus one unit of 2^-7 when rounding up
    e = exp.astype(np.int64) - 1023
    m = 1.0 + (keep.astype(np.float64) + up.astype(np.float64)) / 128.0
    out = np.ldexp(m, e)
    out = np.where(exp == 0, 0.0, out)
    return np.where(sign == 1, -out, out)


def round_to(prec, x):
    if prec == "fp64":
        return np.asarray(x, dtype=np.float64)
    if prec == "fp32":
        return np.asarray(x, dtype=np.float32).astype(np.float64)
    return round_bf16(x)


UNIT = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16": 2.0 ** -8}


def ragged_tube(periods=60, n=5, seed=21):
    """(n,n) tube with 4 n atoms per period: 1200 atoms for the defaults (several 256-tiles + a tail)."""
    return geo.jitter(geo.nanotube(n, n, periods), 0.01, seed)


GRAPHENE = wi.workloads.GRAPHENE
