"""Audit the oracle's floating-point decisions against exact arithmetic.

* alpha = 1: f = K / V is rational, so "f(K', V') > f(K, V)" is the integer
  test K' V > K V'.  Every decision whose computed margin |t| exceeds 1e-9
  must agree with it.
* any alpha: re-decide sampled decisions (all near-ties plus a random
  sample) with a 40-digit decimal logarithm; a disagreement is allowed only
  for a true margin within 1e-11 of the 2^-40 threshold.
"""
import decimal
import math

import numpy as np
import pytest

from paper_1301_0955_amd import workloads as W

decimal.getcontext().prec = 40
EPS = 2.0 ** -40


def _traces(oracle_mod, scales, nodes):
    g, _, _, _ = W.workload_small()
    o = oracle_mod.Oracle.from_graph(g)
    out = []
    for u in nodes:
        *_, trace = o.run_set([u], scales, trace_cap=2_000_000)
        out += trace
    return out


def test_alpha_one_matches_integer_test(oracle_mod):
    tr = _traces(oracle_mod, [1.0], range(0, 1000, 25))
    n_checked = 0
    near = 0
    for r in tr:
        if r["K"] == 0 or r["Kp"] == 0:
            continue
        exact = r["Kp"] * r["V"] > r["K"] * r["Vp"]
        if abs(r["t"]) > 1e-9:
            assert bool(r["result"]) == exact, r
            n_checked += 1
        elif abs(r["t"]) <= EPS:
            near += 1
            # a true tie (K' V = K V') must never count as an improvement
            if r["Kp"] * r["V"] == r["K"] * r["Vp"]:
                assert not r["result"]
    assert n_checked > 1000


def test_general_alpha_decimal_redecide(oracle_mod):
    scales = W.log_scales(10)
    tr = _traces(oracle_mod, scales, range(3, 1000, 97))
    rng = np.random.Generator(np.random.PCG64(5))
    cand = [r for r in tr if r["K"] > 0 and r["Kp"] > 0]
    idx = set(rng.choice(len(cand), size=min(1500, len(cand)), replace=False).tolist())
    idx |= {i for i, r in enumerate(cand) if abs(r["t"]) < 1e-6}
    D = decimal.Decimal
    for i in sorted(idx):
        r = cand[i]
        t = (D(r["Kp"]) / D(r["K"])).ln() - D(repr(r["alpha"])) * (D(r["Vp"]) / D(r["V"])).ln()
        exact = t > D(EPS)
        if bool(r["result"]) != exact:
            assert abs(t - D(EPS)) < D("1e-11"), r
        # the computed margin tracks the exact one closely
        assert abs(D(r["t"]) - t) < D("1e-12"), (r, t)
