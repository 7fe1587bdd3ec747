"""Pins for the oracle's normalised mutual information of two covers (the
overlapping-community NMI that Sec. 4 uses to compare community sets across
scales and with the planted ones; the paper cites its definition without
printing it, so these pins come from the definition and its closed forms):

* a four-node case worked by hand (tests/golden/nmi_worked_example.json);
* identical covers give 1; two partitions into halves that cut each other
  in quarters give exactly 0 (every conditional entropy is refused);
* the value is symmetric in the two covers, and does not depend on the
  order of the communities or on a relabelling of the nodes;
* an independent brute-force evaluation from 0/1 membership matrices
  (natural logs from numpy, conditional entropies summed cell by cell)
  agrees to 1e-9 on random overlapping covers;
* the average over p successive scales (reading N5) of a constant sequence
  is 1, and with p = 2 it is the NMI of each consecutive pair."""
import json
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _random_cover(rng, n, k, pmax=0.4):
    out = []
    for _ in range(k):
        m = rng.random(n) < rng.uniform(0.05, pmax)
        if not m.any():
            m[rng.integers(n)] = True
        out.append(np.flatnonzero(m).astype(np.int32))
    return out


def _brute(n, X, Y):
    """H(X|Y)_norm and H(Y|X)_norm from 0/1 membership matrices."""
    def mat(cover):
        M = np.zeros((len(cover), n), dtype=np.int64)
        for k, c in enumerate(cover):
            M[k, c] = 1
        return M

    def plogp(p):
        return np.where(p > 0, -p * np.log(np.where(p > 0, p, 1.0)), 0.0)

    def half(A, B):
        terms = []
        for x in A:
            px1 = x.mean()
            hx = plogp(px1) + plogp(1 - px1)
            best = None
            for y in B:
                cells = {(i, j): np.mean((x == i) & (y == j)) for i in (0, 1) for j in (0, 1)}
                if not (plogp(cells[1, 1]) + plogp(cells[0, 0]) > plogp(cells[1, 0]) + plogp(cells[0, 1])):
                    continue
                # conditional entropy cell by cell: -sum P(x, y) log P(x | y)
                cond = 0.0
                for j in (0, 1):
                    py = cells[0, j] + cells[1, j]
                    for i in (0, 1):
                        if cells[i, j] > 0:
                            cond -= cells[i, j] * np.log(cells[i, j] / py)
                best = cond if best is None else min(best, cond)
            if best is None:
                best = hx
            terms.append(best / hx if hx > 0 else 0.0)
        return float(np.mean(terms))

    MX, MY = mat(X), mat(Y)
    return 1.0 - (half(MX, MY) + half(MY, MX)) / 2.0


def _margins(n, X, Y):
    """Smallest |h(a) + h(e) - h(b) - h(c)| over all pairs (in nats)."""
    def h(c):
        return 0.0 if c == 0 else -(c / n) * np.log(c / n)
    m = np.inf
    for x in X:
        sx = set(x.tolist())
        for y in Y:
            a = len(sx & set(y.tolist()))
            b, c = len(x) - a, len(y) - a
            e = n - a - b - c
            m = min(m, abs(h(a) + h(e) - h(b) - h(c)))
    return m


def test_worked_example(oracle_mod):
    g = json.load(open(os.path.join(HERE, "golden", "nmi_worked_example.json")))
    v = oracle_mod.nmi(g["n"], g["cover_x"], g["cover_y"])
    assert abs(v - g["nmi"]) <= 1e-12
    assert oracle_mod.nmi(g["n"], g["cover_y"], g["cover_x"]) == v


@pytest.mark.parametrize("seed", range(4))
def test_identical_covers_give_one(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(20, 200))
    X = _random_cover(rng, n, int(rng.integers(1, 12)))
    assert abs(oracle_mod.nmi(n, X, X) - 1.0) <= 1e-12
    part = [np.arange(i, n, 7, dtype=np.int32) for i in range(7)]
    assert abs(oracle_mod.nmi(n, part, part) - 1.0) <= 1e-12


@pytest.mark.parametrize("n", [8, 40, 400])
def test_crossing_halves_give_zero(oracle_mod, n):
    idx = np.arange(n, dtype=np.int32)
    X = [idx[: n // 2], idx[n // 2:]]
    Y = [idx[idx % 2 == 0], idx[idx % 2 == 1]]
    assert oracle_mod.nmi(n, X, Y) == 0.0


@pytest.mark.parametrize("seed", range(6))
def test_symmetry_and_relabelling(oracle_mod, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(30, 150))
    X = _random_cover(rng, n, int(rng.integers(2, 9)))
    Y = _random_cover(rng, n, int(rng.integers(2, 9)))
    v = oracle_mod.nmi(n, X, Y)
    assert oracle_mod.nmi(n, Y, X) == v
    assert abs(oracle_mod.nmi(n, X[::-1], [Y[i] for i in rng.permutation(len(Y))]) - v) <= 1e-12
    perm = rng.permutation(n).astype(np.int32)
    Xp = [np.sort(perm[c]) for c in X]
    Yp = [np.sort(perm[c]) for c in Y]
    assert abs(oracle_mod.nmi(n, Xp, Yp) - v) <= 1e-12
    assert 0.0 <= v <= 1.0 + 1e-12


@pytest.mark.parametrize("seed", range(8))
def test_matches_brute_force(oracle_mod, seed):
    rng = np.random.default_rng(200 + seed)
    for _ in range(50):
        n = int(rng.integers(12, 60))
        X = _random_cover(rng, n, int(rng.integers(1, 6)), pmax=0.7)
        Y = _random_cover(rng, n, int(rng.integers(1, 6)), pmax=0.7)
        if _margins(n, X, Y) > 1e-9:          # no admission test at a tie
            break
    assert abs(oracle_mod.nmi(n, X, Y) - _brute(n, X, Y)) <= 1e-9


def test_empty_covers(oracle_mod):
    assert oracle_mod.nmi(10, [], []) == 1.0
    assert oracle_mod.nmi(10, [np.array([1, 2], np.int32)], []) == 0.0
    empty = np.zeros(0, np.int32)
    assert oracle_mod.nmi(10, [empty], [empty, empty]) == 1.0


def test_empty_communities_are_skipped(oracle_mod):
    rng = np.random.default_rng(11)
    n = 50
    X = _random_cover(rng, n, 4)
    Y = _random_cover(rng, n, 3)
    empty = np.zeros(0, np.int32)
    v = oracle_mod.nmi(n, X, Y)
    assert oracle_mod.nmi(n, X[:2] + [empty] + X[2:], [empty] + Y + [empty]) == v


def test_successive_average(oracle_mod):
    rng = np.random.default_rng(7)
    n = 80
    X = _random_cover(rng, n, 5)
    assert np.allclose(oracle_mod.nmi_successive(n, [X] * 6, 3), 1.0, atol=1e-12)
    covers = [_random_cover(rng, n, 4) for _ in range(5)]
    pairs = [oracle_mod.nmi(n, covers[t], covers[t + 1]) for t in range(4)]
    assert np.array_equal(oracle_mod.nmi_successive(n, covers, 2), np.array(pairs))
    w3 = oracle_mod.nmi_successive(n, covers, 3)
    assert w3.size == 3 and abs(w3[1] - (pairs[1] + pairs[2]) / 2) <= 1e-15
