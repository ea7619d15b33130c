"""Pins of the oracle's EIM pass (Algorithm 2 with Select, Algorithm 3, and
the Section 4.1 termination changes): the counter-based generator against
numpy's Philox, each draw and the Select threshold recomputed with library
routines, the special cases the paper names (no sampling falls back to
Gonzalez; all-equal points end after one iteration), per-iteration
invariants and the sample-size distribution.  The 10-approximation holds
only with sufficient probability: per instance it is parity unpinned."""
import math

import numpy as np
import pytest
from scipy.spatial.distance import cdist


def _numpy_philox(ctr, key):
    # numpy advances the 256-bit counter before each block, so start it one
    # below the wanted counter
    c = [int(x) for x in ctr]
    v = c[0] | (c[1] << 64) | (c[2] << 128) | (c[3] << 192)
    v = (v - 1) % (1 << 256)
    prev = [(v >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
    bg = np.random.Philox(counter=prev, key=[int(key[0]), int(key[1])])
    return bg.random_raw(4)


def test_philox_matches_numpy(orc):
    rng = np.random.default_rng(1)
    cases = [([0, 0, 0, 0], [0, 0]),
             ([2**64 - 1] * 4, [2**64 - 1] * 2)]
    for _ in range(20):
        cases.append((rng.integers(0, 2**63, 4, dtype=np.uint64).tolist(),
                      rng.integers(0, 2**63, 2, dtype=np.uint64).tolist()))
    for ctr, key in cases:
        assert np.array_equal(orc.philox4x64_10(ctr, key),
                              _numpy_philox(ctr, key))


def _uniforms_numpy(seed, xs, it):
    out = np.empty((len(xs), 2))
    for j, x in enumerate(xs):
        w = _numpy_philox([x, it, 0, 0], [seed, 0])
        out[j] = [(int(w[0]) >> 11) * 2.0**-53, (int(w[1]) >> 11) * 2.0**-53]
    return out


def test_uniform_pair_matches_numpy(orc):
    for x, it in [(0, 0), (5, 0), (123456, 3), (2**31 + 7, 1)]:
        u = orc.eim_uniform_pair(77, x, it)
        assert np.array_equal(u, _uniforms_numpy(77, [x], it)[0])


def _consts(n, k, eps, phi):
    L = math.log(n)
    ne = n ** eps
    return dict(A_S=9 * k * ne * L, A_H=4 * ne * L,
                thr=(4 / eps) * k * ne * L, r=max(1, math.ceil(phi * L)))


def test_no_sampling_falls_back_to_gon(orc):
    # |V| below the loop threshold: the sample is V and the result is
    # Gonzalez on V from point 0
    X = np.random.default_rng(41).normal(size=(1000, 3)).astype(np.float32)
    k = 10
    assert 1000 <= _consts(1000, k, 0.1, 8)["thr"]
    e = orc.eim(X, k, 0.1, 8.0, seed=1)
    assert e["iters"] == [] and len(e["sample"]) == 1000
    c, tr, got = orc.gon(X, k, 0)
    assert np.array_equal(e["centers"], c) and e["radius"] == tr[-1]


def test_all_equal_points_end_in_one_iteration(orc):
    # with the removal rule "distance <= d(v,S)" every point leaves R in the
    # first iteration; the strict rule would never remove any
    n, k, eps = 10000, 1, 0.5
    assert n > _consts(n, k, eps, 1)["thr"]
    X = np.ones((n, 2), np.float32)
    e = orc.eim(X, k, eps, 1.0, seed=3)
    assert len(e["iters"]) == 1 and len(e["R"]) == 0
    assert e["iters"][0]["tau"] == 0.0
    assert np.array_equal(e["sample"], e["S"]) and e["radius"] == 0.0


def _one_iteration_case(orc):
    X = np.random.default_rng(42).normal(size=(20000, 2)).astype(np.float32)
    n, k, eps, phi, seed = 20000, 2, 0.1, 1.0, 1234
    e = orc.eim(X, k, eps, phi, seed)
    return X, n, k, eps, phi, seed, e


def test_draws_and_select_recomputed(orc):
    X, n, k, eps, phi, seed, e = _one_iteration_case(orc)
    assert len(e["iters"]) == 1
    cst = _consts(n, k, eps, phi)
    it = e["iters"][0]
    assert it["p_s"] == min(1.0, cst["A_S"] / n)
    assert it["p_h"] == min(1.0, cst["A_H"] / n)
    U = _uniforms_numpy(seed, range(n), 0)
    S = np.flatnonzero(U[:, 0] < it["p_s"])
    H = np.flatnonzero(U[:, 1] < it["p_h"])
    assert np.array_equal(S, e["S"])
    assert it["h_size"] == len(H) and it["ds_size"] == len(S)
    Xd = X.astype(np.float64)
    dH = cdist(Xd[H], Xd[S], "sqeuclidean").min(axis=1)
    tau = np.sort(dH)[::-1][min(cst["r"], len(H)) - 1]
    assert it["tau"] == pytest.approx(tau, rel=1e-12)
    dR = cdist(Xd, Xd[S], "sqeuclidean").min(axis=1)
    notS = np.ones(n, bool)
    notS[S] = False
    keep = np.flatnonzero(notS & (dR > it["tau"]))
    assert np.array_equal(keep, e["R"])
    assert np.array_equal(np.union1d(S, keep), e["sample"])


def test_iteration_invariants(orc):
    rng = np.random.default_rng(43)
    for trial in range(4):
        X = rng.normal(size=(30000, 3)).astype(np.float32)
        e = orc.eim(X, 3, 0.1, [1.0, 4.0, 6.0, 8.0][trial], seed=trial)
        its = e["iters"]
        assert len(its) >= 1 and e["radius"] >= 0
        sizes = [s["r_size"] for s in its]
        assert all(b < a for a, b in zip(sizes, sizes[1:]))   # R shrinks
        S, R = e["S"], e["R"]
        assert len(np.intersect1d(S, R)) == 0
        Xd = X.astype(np.float64)
        d = cdist(Xd, Xd[S], "sqeuclidean").min(axis=1)
        assert np.all(d[R] > its[-1]["tau"])
        gone = np.setdiff1d(np.arange(len(X)), np.union1d(S, R))
        assert np.all(d[gone] <= max(s["tau"] for s in its) * (1 + 1e-12))
        assert e["n_centers"] == 3
        assert np.all(np.isin(e["centers"], e["sample"]))


def test_sample_sizes_binomial(orc):
    n, k, eps = 50000, 4, 0.1
    cst = _consts(n, k, eps, 4)
    X = np.random.default_rng(44).random((n, 2)).astype(np.float32)
    for seed in range(5):
        it = orc.eim(X, k, eps, 4.0, seed)["iters"][0]
        for cnt, p in ((it["ds_size"], it["p_s"]), (it["h_size"], it["p_h"])):
            mu, sd = n * p, math.sqrt(n * p * (1 - p))
            assert abs(cnt - mu) <= 6 * sd


def test_draw_flags_match_uniform_pairs(orc):
    # the vectorised draws are the per-point uniforms compared with p_S, p_H
    rng = np.random.default_rng(44)
    for it in (0, 3):
        R = np.sort(rng.choice(10**6, 500, replace=False))
        seed = 5 * 2**32 + 17
        f = orc.eim_draw_flags(seed, it, R, 0.3, 0.05)
        for j, x in enumerate(R):
            uS, uH = orc.eim_uniform_pair(seed, int(x), it)
            assert bool(f[j] & 1) == (uS < 0.3) and bool(f[j] & 2) == (uH < 0.05)
    # probability 1 draws everything, 0 nothing
    assert np.all(orc.eim_draw_flags(1, 0, np.arange(100), 1.0, 0.0) == 1)
