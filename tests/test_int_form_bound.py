"""Host check of the arithmetic behind the resident engine's exact-integer
form (no GPU).  For integer coordinates of magnitude at most M with
5 d M^2 <= 2^24 and K = d M^2, every partial sum the kernel forms must be an
integer of magnitude at most 2^24, hence exact in FP32, in each of its
accumulation orders:

- a worker applying center c: K + |c|^2, then + (-2 x_j) c_j in order,
  against a kept minimum m' = (m - |x|^2) + K;
- the leader updating a candidate: (K + |c|^2) + sum of (-2 x_j) c_j, then
  + (|x|^2 - K);
- the canonical distance: sum of (x_j - c_j)^2 in order, which the leader's
  certification compares against;
- a key: (m' - K) + |x|^2, with |x|^2 taken as 0.25 * sum of (-2 x_j)^2.

Section 3.1's traversal then sees the same FP32 keys in both forms.  The
extreme inputs (every coordinate at +-M) reach the largest partial sums."""
import itertools

import numpy as np
import pytest

LIM = 2 ** 24


def int_bound(d):
    m = 0
    while 5 * d * (m + 1) ** 2 <= LIM:
        m += 1
    return m


def partials_ok(seq):
    return all(abs(v) <= LIM for v in seq)


def worker_partials(x, c, K):
    s = K + sum(v * v for v in c)
    out = [s]
    for xj, cj in zip(x, c):
        s += (-2 * xj) * cj
        out.append(s)
    return out


def leader_partials(x, c, K):
    out = worker_partials(x, c, K)
    xx = sum(v * v for v in x)
    out.append(out[-1] + (xx - K))
    return out


def canonical_partials(x, c):
    s, out = 0, []
    for xj, cj in zip(x, c):
        s += (xj - cj) ** 2
        out.append(s)
    return out


def check_pair(x, c, m_prev, K):
    """m_prev: an earlier canonical min-distance of x (an exact integer)."""
    xx = sum(v * v for v in x)
    w = worker_partials(x, c, K)
    l = leader_partials(x, c, K)
    k = canonical_partials(x, c)
    conv = [m_prev - xx, m_prev - xx + K]           # m' from m
    m1 = min(m_prev - xx + K, w[-1])                # the worker's min
    key = [m1 - K, m1 - K + xx]                     # (m' - K) + |x|^2
    sq = [4 * xx, xx]                               # sum of (-2 x)^2, times 0.25
    assert partials_ok(w) and partials_ok(l) and partials_ok(k)
    assert partials_ok(conv) and partials_ok(key) and partials_ok(sq)
    assert w[-1] >= 0 and m1 >= 0                   # the unsigned-bits min stays valid
    assert l[-1] == k[-1]                           # both forms, one distance
    assert key[-1] == min(m_prev, k[-1])            # the key is the canonical minimum


@pytest.mark.parametrize("d", [8, 10, 16, 32, 41, 64])
def test_extreme_sign_patterns(d):
    M = int_bound(d)
    K = d * M * M
    assert 5 * d * M * M <= LIM < 5 * d * (M + 1) ** 2   # M is the largest
    pats = [np.full(d, M), np.full(d, -M), np.array([M if j % 2 else -M for j in range(d)]),
            np.zeros(d, dtype=np.int64)]
    for x, c in itertools.product(pats, pats):
        x = [int(v) for v in x]
        c = [int(v) for v in c]
        far = sum((a - b) ** 2 for a, b in zip(x, c))
        check_pair(x, c, far, K)
        check_pair(x, c, 0, K)


@pytest.mark.parametrize("d", [8, 10, 16, 41])
def test_random_integers_within_bound(d):
    M = int_bound(d)
    K = d * M * M
    rng = np.random.default_rng(d)
    for _ in range(300):
        x = [int(v) for v in rng.integers(-M, M + 1, d)]
        c = [int(v) for v in rng.integers(-M, M + 1, d)]
        c0 = [int(v) for v in rng.integers(-M, M + 1, d)]
        m_prev = sum((a - b) ** 2 for a, b in zip(x, c0))
        check_pair(x, c, m_prev, K)


@pytest.mark.parametrize("d", [8, 10, 16, 41])
def test_bound_rule_margin(d):
    # every partial sum above is at most 4 d M^2, so the rule 5 d M^2 <= 2^24
    # keeps a margin; one past the 4 d M^2 limit, two opposite extreme
    # points are farther apart than 2^24 and the distance is no longer exact
    M = int_bound(d)
    M4 = 0
    while 4 * d * (M4 + 1) ** 2 <= LIM:
        M4 += 1
    assert M <= M4
    x = [M4 + 1] * d
    c = [-(M4 + 1)] * d
    assert not partials_ok(canonical_partials(x, c))
