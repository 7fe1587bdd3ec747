"""Pins for the integer natural log used by every decision (the oracle's
log-domain reading of Eq. 1 and 2): a 40-digit decimal logarithm, and the
from-scratch Python definition used by the replay pin."""
import decimal
import math

import numpy as np
import pytest

from _replay import spec_log

decimal.getcontext().prec = 40


def _ulp_err(x: int, got: float) -> float:
    ref = decimal.Decimal(x).ln()
    if x == 1:
        return 0.0 if got == 0.0 else float("inf")
    err = abs(decimal.Decimal(got) - ref)
    return float(err / decimal.Decimal(math.ulp(float(ref))))


def _inputs():
    rng = np.random.Generator(np.random.PCG64(7))
    xs = list(range(1, 20001))
    xs += [int(v) for v in rng.integers(1, 2**53, size=3000, dtype=np.int64)]
    xs += [int(v) for v in np.exp(rng.uniform(0, math.log(2**53 - 1), 3000)).astype(np.int64)]
    for e in range(1, 53):
        xs += [2**e - 1, 2**e, 2**e + 1]
    xs += [2**53 - 1]
    return sorted(set(x for x in xs if 1 <= x < 2**53))


def test_log_accuracy_vs_decimal(oracle_mod):
    xs = _inputs()
    got = oracle_mod.log(np.array(xs, dtype=np.uint64))
    worst = 0.0
    for x, y in zip(xs, got.tolist()):
        worst = max(worst, _ulp_err(x, y))
    assert worst <= 1.0, worst


def test_log_exact_points(oracle_mod):
    got = oracle_mod.log(np.array([1, 2, 4, 2**20, 2**52], dtype=np.uint64))
    assert got[0] == 0.0
    # powers of two reduce to e * ln 2 through the split constant
    for e, y in zip([1, 2, 20, 52], got[1:]):
        assert abs(y - e * math.log(2.0)) <= 2 * math.ulp(e * math.log(2.0))


def test_log_monotone(oracle_mod):
    xs = np.arange(1, 200001, dtype=np.uint64)
    y = oracle_mod.log(xs)
    assert np.all(np.diff(y) > 0)


def test_python_definition_bitwise(oracle_mod):
    xs = _inputs()[::7]
    got = oracle_mod.log(np.array(xs, dtype=np.uint64))
    for x, y in zip(xs, got.tolist()):
        assert spec_log(x) == y, x
