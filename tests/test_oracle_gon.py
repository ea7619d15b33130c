"""Pins of the oracle's Gonzalez traversal (Section 3.1) against facts that
do not come from the oracle itself: a hand-worked example, closed forms on a
1-D lattice, brute-force optimum (the 2-approximation), the separation
argument behind it, metamorphic relations and library distances."""
import itertools
import json
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

GOLD = os.path.join(os.path.dirname(__file__), "golden", "gon_mrg_hand6.json")


def test_hand_example(orc):
    g = json.load(open(GOLD))
    X = np.array(g["points"], np.float32)
    c, tr, got = orc.gon(X, g["gon"]["k"], g["gon"]["first"])
    assert got == 3
    assert c.tolist() == g["gon"]["centers"]
    assert np.array_equal(tr, np.array(g["gon"]["trace"]))


@pytest.mark.parametrize("L", [1, 2, 5, 8, 9, 100, 101])
def test_lattice_closed_form(orc, L):
    # points 0..L on a line, first = 0: the farthest is L, then the middle
    # (lower of the two middles when L is odd), radius floor(L/2) after it
    X = np.arange(L + 1, dtype=np.float32)[:, None]
    k = 3 if L >= 2 else 2
    c, tr, got = orc.gon(X, k, 0)
    assert c[0] == 0 and c[1] == L
    assert tr[0] == L
    if L >= 2:
        assert c[2] == L // 2
        assert tr[1] == L // 2
        # after 0, L/2, L the radius is ceil(L/2)/2 rounded per half
        half = L // 2
        assert tr[2] == max(half // 2, (L - half) // 2)
    else:
        assert tr[1] == 0 and got == 2


def test_k1_is_max_distance_to_first(orc):
    rng = np.random.default_rng(11)
    X = rng.normal(size=(500, 5)).astype(np.float32)
    for first in (0, 17, 499):
        c, tr, got = orc.gon(X, 1, first)
        ref = cdist(X[first:first + 1].astype(np.float64),
                    X.astype(np.float64)).max()
        assert got == 1 and c[0] == first
        assert abs(tr[0] - ref) <= 1e-12 * ref


def test_two_approximation_bruteforce(orc):
    # Gonzalez's radius is at most twice the optimum, for every first center
    rng = np.random.default_rng(5)
    worst = 0.0
    for trial in range(60):
        n = int(rng.integers(4, 12))
        d = int(rng.integers(1, 4))
        k = int(rng.integers(1, 4))
        X = rng.normal(size=(n, d)).astype(np.float32)
        opt = orc.opt_bruteforce(X, k)
        for first in range(n):
            c, tr, got = orc.gon(X, k, first)
            r = tr[got - 1]
            assert r >= opt * (1 - 1e-12)
            assert r <= 2 * opt * (1 + 1e-12)
            if opt > 0:
                worst = max(worst, r / opt)
    assert worst > 1.0   # the bound is exercised, not vacuous


def test_bruteforce_itself_on_known_optimum(orc):
    # the enumeration on a configuration whose optimum is known by hand:
    # two tight pairs far apart, k = 2 -> radius = half-gap within a pair
    X = np.array([[0, 0], [0, 2], [100, 0], [100, 2]], np.float32)
    assert orc.opt_bruteforce(X, 2) == 2.0
    assert orc.opt_bruteforce(X, 4) == 0.0
    assert orc.opt_bruteforce(X, 1) == pytest.approx(np.hypot(100, 2))


def test_separation_certificate(orc):
    # the k centers and the final farthest point are pairwise at least the
    # final radius apart (the argument behind the factor 2)
    rng = np.random.default_rng(7)
    X = rng.normal(size=(3000, 3)).astype(np.float32)
    k = 25
    c, tr, got, mind = orc.gon(X, k, 0, want_mind=True)
    a = int(np.argmax(mind))
    P = X[np.r_[c, a]].astype(np.float64)
    D = cdist(P, P)
    iu = np.triu_indices(len(P), 1)
    assert D[iu].min() >= tr[k - 1] * (1 - 1e-12)


def test_invariants(orc):
    rng = np.random.default_rng(8)
    X = rng.random((2000, 4)).astype(np.float32)
    k = 40
    c, tr, got, mind = orc.gon(X, k, 5, want_mind=True)
    assert got == k
    assert np.all(np.diff(tr) <= 0)                 # trace never increases
    assert len(set(c.tolist())) == k                # no center twice
    assert np.all(mind[c] == 0)                     # centers cover themselves
    assert np.sqrt(mind.max()) == tr[-1]
    # each chosen center is a farthest point at its step (library distances)
    D = cdist(X.astype(np.float64), X[c].astype(np.float64), "sqeuclidean")
    for t in range(k - 1):
        m = D[:, :t + 1].min(axis=1)
        far = np.flatnonzero(m >= m.max() * (1 - 1e-12))
        assert c[t + 1] in far


def test_prefix_property(orc):
    X = np.random.default_rng(9).random((5000, 3)).astype(np.float32)
    c1, t1, g1 = orc.gon(X, 10, 0)
    c2, t2, g2 = orc.gon(X, 60, 0)
    assert np.array_equal(c1, c2[:10]) and np.array_equal(t1, t2[:10])


def test_early_stop_on_duplicates(orc):
    base = np.array([[0, 0], [1, 1], [2, 0]], np.float32)
    X = np.repeat(base, 5, axis=0)
    c, tr, got = orc.gon(X, 10, 0)
    assert got == 3
    assert np.all(c[3:] == -1)
    assert tr[2] == 0 and np.all(tr[3:] == 0)
    assert sorted(X[c[:3]].tolist()) == sorted(base.tolist())


def test_tie_goes_to_lowest_index(orc):
    # four corners of a square seen from the center point: all tie
    X = np.array([[1, 1], [0, 0], [2, 0], [0, 2], [2, 2]], np.float32)
    c, tr, got = orc.gon(X, 2, 0)
    assert c[1] == 1


def test_translation_and_scaling(orc):
    X = points = np.random.default_rng(2).integers(0, 20, (800, 6)).astype(
        np.float32)
    c, tr, _ = orc.gon(X, 30, 3)
    shift = np.arange(6, dtype=np.float32) * 7 - 11
    c2, tr2, _ = orc.gon(points + shift, 30, 3)
    assert np.array_equal(c, c2) and np.array_equal(tr, tr2)
    Y = np.random.default_rng(3).normal(size=(800, 6)).astype(np.float32)
    c3, tr3, _ = orc.gon(Y, 30, 0)
    c4, tr4, _ = orc.gon(Y * np.float32(8.0), 30, 0)
    assert np.array_equal(c3, c4) and np.array_equal(tr3 * 8, tr4)


def test_replay_accepts_own_and_rejects_wrong(orc):
    X = np.random.default_rng(4).random((1000, 2)).astype(np.float32)
    k = 15
    c, tr, got = orc.gon(X, k, 0)
    bad, ties, tr2 = orc.gon_replay(X, k, c, 0.0)
    assert bad == -1 and ties == 0 and np.array_equal(tr, tr2)
    wrong = c.copy()
    wrong[5] = c[3]              # a point already chosen
    assert orc.gon_replay(X, k, wrong, 1e-6)[0] == 5
    near = c.copy()
    # the second farthest point at step 4 is not a certified tie at band 0
    _, _, _, mind = orc.gon(X, 5, 0, want_mind=True)
    order = np.argsort(-mind, kind="stable")
    near[5] = order[1]
    assert orc.gon_replay(X, k, near, 0.0)[0] == 5
    # a truncated sequence violates the stopping rule
    assert orc.gon_replay(X, k, c[:7], 1e-6)[0] == 7


def test_replay_accepts_certified_tie(orc):
    # two points at squared distances 100 and 100*(1 - 1e-7) from the first
    X = np.array([[0.0], [10.0], [-np.sqrt(100 * (1 - 1e-7))]], np.float32)
    m = (X[:, 0].astype(np.float64)) ** 2
    assert m[2] < m[1]
    band = 1e-6
    bad, ties, _ = orc.gon_replay(X, 2, np.array([0, 2]), band)
    assert bad == -1 and ties == 1
    assert orc.gon_replay(X, 2, np.array([0, 2]), 0.0)[0] == 1


def test_resume_single_first_is_gon(orc):
    X = np.random.default_rng(41).normal(size=(800, 4)).astype(np.float32)
    for first in (0, 313):
        c, tr, got = orc.gon_resume(X, 25, [first])
        c2, tr2, got2 = orc.gon(X, 25, first)
        assert got == got2 and np.array_equal(c, c2) and np.array_equal(tr, tr2)


def test_resume_from_own_prefix_is_longer_run(orc):
    # the traversal adds one center per step from the current set alone, so a
    # saved prefix extends to the longer run (Section 3.1)
    X = np.random.default_rng(42).normal(size=(1500, 3)).astype(np.float32)
    c, tr, got = orc.gon(X, 60, 7)
    for p in (2, 17, 59, 60):
        cr, trr, gr = orc.gon_resume(X, 60, c[:p])
        assert gr == got and np.array_equal(cr, c) and np.array_equal(trr, tr)


def test_resume_arbitrary_prefix_by_library_distances(orc):
    # an arbitrary prefix (not a traversal's): the prefix is kept, every
    # later center is the lowest-index farthest point by library distances,
    # trace[t] is the next center's distance to centers 0..t and the last
    # entry is the covering radius (integer coordinates: all exact)
    rng = np.random.default_rng(43)
    for trial in range(20):
        n = int(rng.integers(5, 60))
        X = rng.integers(0, 9, (n, 2)).astype(np.float32)
        k = int(rng.integers(1, 12))
        p = int(rng.integers(1, k + 1))
        pre = rng.choice(n, min(p, n), replace=False)
        p = len(pre)
        if p > k:
            continue
        c, tr, got = orc.gon_resume(X, k, pre)
        D = cdist(X.astype(np.float64), X.astype(np.float64), "sqeuclidean")
        assert np.array_equal(c[:min(p, got)], pre[:min(p, got)])
        m = np.full(n, np.inf)
        for t in range(got):
            m = np.minimum(m, D[c[t]])
            if t + 1 < got:
                nxt = c[t + 1]
                if t + 1 >= p:
                    assert nxt == int(np.flatnonzero(m == m.max())[0])
                assert (m[nxt] > 0 or t + 1 < p) and tr[t] == np.sqrt(m[nxt])
            else:
                assert tr[t] == np.sqrt(m.max())
                # ended at k, or after the prefix with every point covered
                if got < k:
                    assert got >= p and m.max() == 0
        assert np.all(c[got:] == -1) and np.all(tr[got:] == 0)


def test_resume_covered_prefix_center_is_kept(orc):
    # a forced center at distance 0 from the centers before it is still a
    # center (the prefix is taken as given); the run stops only at a free
    # step whose farthest point is covered
    X = np.array([[0, 0], [5, 0], [0, 0], [9, 9]], np.float32)
    c, tr, got = orc.gon_resume(X, 4, [0, 1, 2])
    assert got == 4 and c.tolist() == [0, 1, 2, 3]
    # trace: next center's distance to the centers before it, then the
    # covering radius (0: every point is a center)
    assert tr.tolist() == [5.0, 0.0, np.sqrt(4 * 4 + 9 * 9), 0.0]
    c, tr, got = orc.gon_resume(X, 6, [0, 2, 1])
    assert got == 4 and c.tolist() == [0, 2, 1, 3, -1, -1]
    assert tr.tolist() == [0.0, 5.0, np.sqrt(4 * 4 + 9 * 9), 0.0, 0.0, 0.0]


def test_resume_rejects_bad_prefix(orc):
    X = np.zeros((10, 2), np.float32)
    for pre, k in (([], 3), ([0, 1, 2, 3], 3), ([10], 3), ([-1], 3)):
        with pytest.raises(ValueError):
            orc.gon_resume(X, k, pre)
