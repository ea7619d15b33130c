"""Seeded synthetic workloads for the k-center hot path.

This module only draws inputs; it holds none of the method's arithmetic.
The tests, the smoke check and the benchmark all draw their inputs from it,
so the oracle and the HIP library always see the same points.

Every generator uses numpy's PCG64 ``default_rng(seed)``, draws in FP64 and
casts to FP32 (the precision the library consumes).  Shapes follow the
paper's experimental data (Section 7.3): uniform points in a square, Gaussian
blobs, and an unbalanced mixture where one blob holds most points.  The two
public datasets the paper also uses are absent; ``points_int_grid`` and
``points_mixed_scale`` are synthetic stand-ins with the same schema shape
(10 small-integer features; 41 mixed-scale features).
"""
import math

import numpy as np


def points_uniform(n, d=2, seed=1):
    """n points uniform in [0,1)^d (the paper's uniform-square data)."""
    rng = np.random.default_rng(seed)
    return rng.random((n, d), dtype=np.float32)


def points_int_grid(n, seed=2):
    """n points with d = 10 integer coordinates stored as FP32: five columns
    uniform in {1..4} interleaved with five uniform in {1..13}.  Squared
    distances are at most 5*3^2 + 5*12^2 = 765, exact in FP32."""
    rng = np.random.default_rng(seed)
    X = np.empty((n, 10), np.float32)
    for c in range(5):
        X[:, 2 * c] = rng.integers(1, 5, n)
        X[:, 2 * c + 1] = rng.integers(1, 14, n)
    return X


def points_gauss_mixture(n, d=16, n_comp=50, lo=-100.0, hi=100.0,
                         sig_lo=0.5, sig_hi=5.0, seed=3, heavy=None):
    """Isotropic Gaussian mixture: component centers uniform in [lo,hi]^d,
    per-component sigma uniform in [sig_lo, sig_hi].  Components are equally
    likely, unless ``heavy`` (a fraction) is given: then component 0 holds
    that fraction of the points and the rest are spread uniformly over the
    others (the paper's unbalanced data)."""
    rng = np.random.default_rng(seed)
    cen = rng.uniform(lo, hi, (n_comp, d))
    sig = rng.uniform(sig_lo, sig_hi, n_comp)
    if heavy is None:
        comp = rng.integers(0, n_comp, n)
    else:
        comp = np.where(rng.random(n) < heavy, 0,
                        rng.integers(1, n_comp, n))
    X = np.empty((n, d), np.float32)
    step = 1 << 20
    for s in range(0, n, step):
        e = min(n, s + step)
        c = comp[s:e]
        X[s:e] = cen[c] + sig[c, None] * rng.standard_normal((e - s, d))
    return X


def partition_offsets(n, m, alpha=0.5, seed=3):
    """Offsets [m+1] of m contiguous partitions with Dirichlet(alpha) sizes:
    floor(w_p * n), the remainder handed out by largest fractional part
    (ties to the lower index).  Empty partitions are allowed."""
    rng = np.random.default_rng(seed + 1000)
    w = rng.dirichlet([alpha] * m)
    raw = w * n
    sz = np.floor(raw).astype(np.int64)
    rem = n - int(sz.sum())
    frac = raw - sz
    order = np.lexsort((np.arange(m), -frac))
    sz[order[:rem]] += 1
    off = np.zeros(m + 1, np.int64)
    off[1:] = np.cumsum(sz)
    return off


def points_mixed_scale(n, seed=4):
    """n points, d = 41, mixed-scale columns z-scored per column in FP64:
    7 log-normal (sigma 3), 20 Bernoulli(p_j) with p_j ~ U[0.01, 0.5],
    14 uniform integers {0..v_j} with v_j ~ U{2..10}.  A zero-variance
    column becomes 0."""
    rng = np.random.default_rng(seed)
    X = np.empty((n, 41), np.float32)
    cols = []
    for _ in range(7):
        cols.append(("ln", None))
    for _ in range(20):
        cols.append(("b", rng.uniform(0.01, 0.5)))
    for _ in range(14):
        cols.append(("i", int(rng.integers(2, 11))))
    for j, (kind, par) in enumerate(cols):
        if kind == "ln":
            v = rng.lognormal(0.0, 3.0, n)
        elif kind == "b":
            v = (rng.random(n) < par).astype(np.float64)
        else:
            v = rng.integers(0, par + 1, n).astype(np.float64)
        mu = v.mean()
        sd = v.std()
        X[:, j] = 0.0 if sd == 0 else (v - mu) / sd
    return X


def to_bf16_rne(X):
    """Round FP32 to BF16 (round to nearest even), returned as uint16 bits.
    Used to hand the library a BF16 copy of the points."""
    b = np.ascontiguousarray(X, np.float32).view(np.uint32)
    lsb = (b >> 16) & 1
    r = (b + 0x7FFF + lsb) >> 16
    return r.astype(np.uint16)


# ---------------------------------------------------------------------------
# The five benchmark workloads.

CONFIG1 = dict(name="gon_uniform_n20000_d2_k20", n=20000, d=2, k=20, first=0)
CONFIG2 = dict(name="gon_intgrid_n1000000_d10", n=1_000_000, d=10,
               ks=(100, 1000), first=0)
CONFIG3 = dict(name="mrg_gauss50_n8000000_d16_m64_k200", n=8_000_000, d=16,
               m=64, k=200)
CONFIG4 = dict(name="gon_mixed41_n5000000_k500", n=5_000_000, d=41, k=500)
CONFIG5 = dict(name="batch256_unbalanced_gon_mrg_eim", count=256)


def config1(n=20000):
    return points_uniform(n, 2, seed=1)


# The three synthetic graph types of the paper's comparison (Section 8.1,
# Tables 2-4), 2-D, at the scale the printed radii imply: Unif uniform in
# [0, 100)^2; Gau 25 clusters with centers uniform in [0, 100]^2 and
# sigma 0.1, points spread evenly; UnB the same with about half the points
# in cluster 0.
QUALITY_SETS = {"unif": 100_000, "gau": 1_000_000, "unb": 200_000}


def quality_points(kind, seed, n=None):
    """One data set of graph type `kind` ('unif', 'gau', 'unb'); n defaults
    to the paper's size for that type."""
    n = QUALITY_SETS[kind] if n is None else n
    if kind == "unif":
        rng = np.random.default_rng(seed)
        return (rng.random((n, 2)) * 100.0).astype(np.float32)
    heavy = 0.5 if kind == "unb" else None
    return points_gauss_mixture(n, 2, 25, 0.0, 100.0, 0.1, 0.1, seed=seed, heavy=heavy)


def equal_offsets(n, m):
    """Offsets [m+1] of m contiguous partitions of sizes differing by at most
    one (the points are i.i.d., so contiguous blocks are random subsets)."""
    return np.array([p * n // m for p in range(m + 1)], np.int64)


def config2(n=1_000_000):
    return points_int_grid(n, seed=2)


def config3(n=8_000_000, m=64):
    X = points_gauss_mixture(n, 16, 50, seed=3)
    return X, partition_offsets(n, m, 0.5, seed=3)


def config4(n=5_000_000):
    X = points_mixed_scale(n, seed=4)
    return X, to_bf16_rne(X)


def config5_instances(count=256, n_lo=1e3, n_hi=2e6, seed=5):
    """Instance descriptors of the mixed batch: n log-uniform in
    [n_lo, n_hi], d in {2, 8, 32}, k in [10, 400], algorithm drawn 40% GON /
    30% MRG (m in {8,16,32,64}) / 30% EIM (eps in {0.1, 0.5}, phi in
    {1,4,6,8}, Philox seed 5*2^32 + id).  Points come from
    ``config5_points``."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(math.floor(math.exp(rng.uniform(math.log(n_lo),
                                                math.log(n_hi)))))
        d = int(rng.choice([2, 8, 32]))
        k = int(rng.integers(10, 401))
        u = rng.random()
        inst = dict(id=i, n=n, d=d, k=k, data_seed=5_000 + i)
        if u < 0.4:
            inst["algo"] = "gon"
        elif u < 0.7:
            inst["algo"] = "mrg"
            inst["m"] = int(rng.choice([8, 16, 32, 64]))
        else:
            inst["algo"] = "eim"
            inst["eps"] = float(rng.choice([0.1, 0.5]))
            inst["phi"] = float(rng.choice([1.0, 4.0, 6.0, 8.0]))
            inst["seed"] = 5 * (1 << 32) + i
        out.append(inst)
    return out


def config5_points(inst):
    """Points of one batch instance: 25 Gaussian blobs in [-100,100]^d,
    sigma in [0.5, 5], blob 0 holding 90% of the points."""
    X = points_gauss_mixture(inst["n"], inst["d"], 25, seed=inst["data_seed"],
                             heavy=0.9)
    if inst["algo"] == "mrg":
        off = partition_offsets(inst["n"], inst["m"], 0.5,
                                seed=inst["data_seed"])
        return X, off
    return X, None
