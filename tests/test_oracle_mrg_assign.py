"""Pins of the oracle's assignment (k-center objective, Section 1.1) and MRG
(Algorithm 1, Lemmas 1-3) against a hand-worked example, library distances,
brute-force optimum and the special cases where MRG reduces to Gonzalez."""
import json
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

GOLD = os.path.join(os.path.dirname(__file__), "golden", "gon_mrg_hand6.json")


def test_assign_hand_example(orc):
    g = json.load(open(GOLD))
    X = np.array(g["points"], np.float32)
    lab, R = orc.assign(X, np.array(g["assign"]["centers"]))
    assert lab.tolist() == g["assign"]["labels"]
    assert R == g["assign"]["radius"]


def test_assign_matches_library(orc):
    rng = np.random.default_rng(21)
    for d in (1, 3, 16):
        X = rng.normal(size=(700, d)).astype(np.float32)
        C = rng.choice(700, 37, replace=False)
        lab, R, mind = orc.assign(X, C, want_mind=True)
        D = cdist(X.astype(np.float64), X[C].astype(np.float64), "sqeuclidean")
        ref = D.min(axis=1)
        assert np.allclose(mind, ref, rtol=1e-12, atol=0)
        # label: lowest position among the (numerically) nearest
        for i in range(700):
            near = np.flatnonzero(D[i] <= ref[i] * (1 + 1e-12))
            assert lab[i] == near[0] or (len(near) > 1 and lab[i] in near)
        assert R == pytest.approx(np.sqrt(ref.max()), rel=1e-12)


def test_assign_ties_lowest_position(orc):
    X = np.array([[0, 0], [2, 0], [-2, 0], [1, 0]], np.float32)
    lab, R = orc.assign(X, np.array([1, 2]))
    assert lab[0] == 0      # equidistant from both centers
    lab2, _ = orc.assign(X, np.array([2, 1]))
    assert lab2[0] == 0


def test_assign_radius_equals_gon_trace(orc):
    X = np.random.default_rng(22).random((3000, 5)).astype(np.float32)
    c, tr, got = orc.gon(X, 30, 0)
    _, R = orc.assign(X, c[:got])
    assert R == tr[got - 1]


def test_mrg_hand_example(orc):
    g = json.load(open(GOLD))["mrg"]
    X = np.array(json.load(open(GOLD))["points"], np.float32)
    r = orc.mrg(X, np.array(g["offsets"]), g["k"])
    assert r["round1"].tolist() == g["round1"]
    assert np.allclose(r["r1"], g["r1"], rtol=1e-15)
    assert r["union"].tolist() == g["union"]
    assert r["centers"][:r["n_centers"]].tolist() == g["centers"]
    assert r["r2"] == g["r2"] and r["radius"] == g["radius"]


def _random_offsets(rng, n, m):
    cuts = np.sort(rng.integers(0, n + 1, m - 1))
    return np.r_[0, cuts, n].astype(np.int64)


def test_mrg_four_approximation_bruteforce(orc):
    # Lemma 2: two-round MRG is within 4 * OPT, for any partition
    rng = np.random.default_rng(31)
    worst = 0.0
    for trial in range(80):
        n = int(rng.integers(5, 13))
        d = int(rng.integers(1, 3))
        k = int(rng.integers(1, 4))
        m = int(rng.integers(1, 5))
        X = rng.normal(size=(n, d)).astype(np.float32)
        opt = orc.opt_bruteforce(X, k)
        perm = rng.permutation(n)
        Xp = X[perm]
        off = _random_offsets(rng, n, m)
        r = orc.mrg(Xp, off, k)
        assert r["radius"] <= 4 * opt * (1 + 1e-12) + 1e-12
        assert r["radius"] >= opt * (1 - 1e-12)
        # the triangle-inequality chain of the proof
        assert r["radius"] <= r["r1"].max() + r["r2"] + 1e-9
        if opt > 0:
            worst = max(worst, r["radius"] / opt)
    assert worst > 1.0


def test_lemma1_gon_on_subsets(orc):
    # Gonzalez on any subset S covers S within 2 * OPT(V)
    rng = np.random.default_rng(32)
    for trial in range(40):
        n = int(rng.integers(6, 12))
        k = int(rng.integers(1, 4))
        X = rng.normal(size=(n, 2)).astype(np.float32)
        opt = orc.opt_bruteforce(X, k)
        S = np.sort(rng.choice(n, int(rng.integers(1, n + 1)), replace=False))
        c, tr, got = orc.gon(X[S], k, 0)
        assert tr[got - 1] <= 2 * opt * (1 + 1e-12) + 1e-12


def test_mrg_one_partition_is_gon(orc):
    X = np.random.default_rng(33).random((2000, 3)).astype(np.float32)
    k = 20
    r = orc.mrg(X, np.array([0, 2000]), k)
    c, tr, got = orc.gon(X, k, 0)
    assert set(r["centers"].tolist()) == set(c.tolist())
    assert r["radius"] == tr[-1]


def test_mrg_small_partitions_is_gon(orc):
    # every partition holds at most k points: the union is all of V
    X = np.random.default_rng(34).random((300, 2)).astype(np.float32)
    k = 12
    off = np.arange(0, 301, 10)
    r = orc.mrg(X, off, k)
    assert r["union"].tolist() == list(range(300))
    c, tr, got = orc.gon(X, k, 0)
    assert np.array_equal(r["centers"], c)


def test_mrg_empty_partitions(orc):
    X = np.random.default_rng(35).random((500, 2)).astype(np.float32)
    off = np.array([0, 0, 200, 200, 500, 500])
    r = orc.mrg(X, off, 10)
    assert np.all(r["round1"][[0, 2, 4]] == -1)
    assert r["n_centers"] == 10 and np.all(r["r1"][[0, 2, 4]] == 0)


def test_multi_round_bound_bruteforce(orc):
    # Lemma 3: i rounds of the loop give a 2(i+1) approximation; here
    # "rounds" counts the final round too, so the bound is 2 * rounds
    rng = np.random.default_rng(36)
    seen = set()
    for trial in range(60):
        n = int(rng.integers(8, 15))
        k = int(rng.integers(1, 3))
        c = int(rng.integers(2 * k + 1, 7))
        X = rng.normal(size=(n, 2)).astype(np.float32)
        opt = orc.opt_bruteforce(X, k)
        r = orc.mrg_rounds(X, k, c)
        assert r["radius"] >= 0
        assert r["radius"] <= 2 * r["rounds"] * opt * (1 + 1e-12) + 1e-12
        seen.add(r["rounds"])
    assert max(seen) >= 3


def test_multi_round_capacity_above_n_is_gon(orc):
    X = np.random.default_rng(37).random((400, 3)).astype(np.float32)
    r = orc.mrg_rounds(X, 9, 400)
    c, tr, got = orc.gon(X, 9, 0)
    assert r["rounds"] == 1 and np.array_equal(r["centers"], c)


def test_min_dist2_to_set_matches_library(orc):
    # d(x, S) of the EIM distance pass and of Select: squared FP64 distance to
    # the nearest listed point and the lowest list position attaining it
    rng = np.random.default_rng(38)
    for d in (1, 2, 8, 32):
        X = rng.normal(size=(400, d)).astype(np.float32)
        for trial in range(6):
            S = rng.choice(400, int(rng.integers(1, 60)), replace=False)
            x = int(rng.integers(0, 400))
            v, a = orc.min_dist2_to_set(X, x, S)
            D = cdist(X[x:x + 1].astype(np.float64), X[S].astype(np.float64),
                      "sqeuclidean")[0]
            assert v == pytest.approx(D.min(), rel=1e-12, abs=0)
            assert D[a] <= D.min() * (1 + 1e-12)
            # integer coordinates: every distance exact, so value and the
            # lowest position are exact too
            Xi = rng.integers(-20, 21, (400, d)).astype(np.float32)
            v, a = orc.min_dist2_to_set(Xi, x, S)
            Di = cdist(Xi[x:x + 1].astype(np.float64), Xi[S].astype(np.float64),
                       "sqeuclidean")[0]
            assert v == Di.min() and a == int(np.flatnonzero(Di == Di.min())[0])
    # a repeated member ties with itself: the first position wins
    X = np.array([[0, 0], [3, 4], [3, 4], [6, 8]], np.float32)
    assert orc.min_dist2_to_set(X, 0, np.array([3, 2, 1])) == (25.0, 1)
    assert orc.min_dist2_to_set(X, 3, np.array([0])) == (100.0, 0)
    # the empty set is at infinite distance
    v, a = orc.min_dist2_to_set(X, 0, np.array([], np.int64))
    assert v == np.inf and a == -1


@pytest.mark.parametrize("n,c,k", [(3001, 1000, 40), (2500, 700, 25), (999, 250, 12)])
def test_multi_round_one_pass_equals_two_round(orc, n, c, k):
    # one pass of the loop (Algorithm 1) is two-round MRG on the blocks of
    # the ascending order, whose sizes differ by at most one: partition p is
    # [p*n // mi, (p+1)*n // mi) with mi = ceil(n / c).  Clustered data, so
    # that block boundaries and first centers change the result.
    X = np.random.default_rng(39).normal(size=(n, 3)).astype(np.float32)
    X[: n // 3] += 40.0
    X[n // 3: n // 2] -= 25.0
    mi = -(-n // c)
    off = np.array([p * n // mi for p in range(mi + 1)], np.int64)
    assert np.diff(off).max() - np.diff(off).min() <= 1
    r = orc.mrg_rounds(X, k, c)
    q = orc.mrg(X, off, k)
    assert r["rounds"] == 2
    assert np.array_equal(r["centers"], q["centers"])
    assert r["n_centers"] == q["n_centers"] and r["radius"] == q["radius"]
    # the union is ascending and is exactly the blocks' Gonzalez centers, each
    # block started at its smallest index (computed here block by block)
    S = r["sample"]
    assert np.all(np.diff(S) > 0)
    blocks = []
    for p in range(mi):
        cc, _, got = orc.gon(X[off[p]:off[p + 1]], k, 0)
        blocks.append(cc[:got] + off[p])
    assert np.array_equal(S, np.sort(np.concatenate(blocks)))
    assert np.array_equal(S, q["union"])
    # the last round starts from the smallest index of S
    assert r["centers"][0] == S[0]


def test_multi_round_two_passes_compose(orc):
    # two passes of the loop: the second pass splits the first pass's union
    # (ascending) into ceil(|S|/c) blocks and runs Gonzalez on each
    n, c, k = 4000, 250, 20
    X = np.random.default_rng(40).normal(size=(n, 2)).astype(np.float32)
    r = orc.mrg_rounds(X, k, c)
    assert r["rounds"] == 3
    S = np.arange(n)
    for _ in range(2):
        mi = -(-len(S) // c)
        nxt = []
        for p in range(mi):
            blk = S[p * len(S) // mi:(p + 1) * len(S) // mi]
            cc, _, got = orc.gon(X[blk], k, 0)
            nxt.append(blk[cc[:got]])
        S = np.sort(np.concatenate(nxt))
    assert np.array_equal(r["sample"], S)
    cc, tr, got = orc.gon(X[S], k, 0)
    assert np.array_equal(r["centers"][:got], S[cc[:got]])
