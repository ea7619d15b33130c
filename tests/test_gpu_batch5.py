"""Oracle parity of kcenter_batch on the mixed-batch workload: Gonzalez, MRG
(Algorithm 1) and EIM (Algorithms 2 and 3) instances of d in {2, 8, 32}
with unbalanced Gaussian blobs (one blob holds 90% of the points).

* Integer coordinates (the blobs rounded; squared distances below 2^24, so
  exact in FP32): every instance's centers and radius equal the oracle's bit
  for bit, EIM's sample too.
* The full 256-instance float batch: within a fixed oracle budget, at least
  15 instances per algorithm (at least 3 of them at d = 32) are checked
  against the oracle -- Gonzalez sequences replayed (certified ties only)
  with the exact radius; MRG's first round per partition, union and second
  round replayed; EIM's samples and iteration records equal the oracle's, and
  on the larger instances its first iteration's draws, threshold and a
  seeded sample of keep / remove decisions."""
import math

import numpy as np
import pytest

from paper_1604_03228_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def band(d):
    m = d + 2
    return 2 * m * U32 / (1 - m * U32) + 1e-12


@pytest.fixture(scope="module")
def kc():
    import paper_1604_03228_amd as kc
    assert torch.cuda.is_available()
    return kc


def on_stream(fn):
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        out = fn()
    st.synchronize()
    return out


def run_batch(kc, probs):
    h = kc.Handle()
    outs = on_stream(lambda: kc.batch(probs, handle=h))
    assert h.device_status() == 0
    res = [(c.cpu().numpy(), int(nc.item()), float(r.item())) for c, nc, r in outs]
    return h, res


def _int_instances():
    """Two instances per (algorithm, d): EIM with eps = 0.1 enters its
    sampling loop, with eps = 0.5 it runs Gonzalez on all points."""
    out = []
    i = 0
    for d in (2, 8, 32):
        for rep in range(2):
            i += 1
            n = 6_000 + 3_137 * rep + 1_000 * d
            out.append(dict(id=i, algo="gon", n=n, d=d, k=17 + 23 * rep, first=rep * 11))
            i += 1
            out.append(dict(id=i, algo="mrg", n=n + 501, d=d, k=12 + 9 * rep,
                            m=(8, 32)[rep]))
            i += 1
            eps = (0.1, 0.5)[rep]
            out.append(dict(id=i, algo="eim", n=(20_000, 7_000)[rep], d=d, k=10 + rep,
                            eps=eps, phi=(4.0, 8.0)[rep], seed=5 * 2**32 + i))
    return out


def test_batch_mixed_integer_exact(kc, orc):
    orc.set_threads(16)
    insts = _int_instances()
    probs, hosts, offs = [], [], []
    for inst in insts:
        X = np.round(W.points_gauss_mixture(inst["n"], inst["d"], 25, seed=9_000 + inst["id"],
                                            heavy=0.9)).astype(np.float32)
        pr = dict(X=torch.from_numpy(X).cuda(), algo=inst["algo"], k=inst["k"])
        off = None
        if inst["algo"] == "gon":
            pr["first"] = inst["first"]
        elif inst["algo"] == "mrg":
            off = W.partition_offsets(inst["n"], inst["m"], 0.5, seed=inst["id"])
            pr["offsets"] = off
        else:
            pr.update(eps=inst["eps"], phi=inst["phi"], seed=inst["seed"])
        probs.append(pr)
        hosts.append(X)
        offs.append(off)
    h, res = run_batch(kc, probs)
    h.close()
    loops = 0
    for inst, X, off, (c, nc, r) in zip(insts, hosts, offs, res):
        k = inst["k"]
        if inst["algo"] == "gon":
            oc, otr, og = orc.gon(X, k, inst["first"])
            assert nc == og and np.array_equal(c, oc) and r == otr[og - 1], inst
        elif inst["algo"] == "mrg":
            o = orc.mrg(X, off, k)
            assert nc == o["n_centers"] and np.array_equal(c, o["centers"]), inst
            assert r == o["radius"], inst
        else:
            o = orc.eim(X, k, inst["eps"], inst["phi"], inst["seed"])
            assert nc == o["n_centers"] and np.array_equal(c, o["centers"]), inst
            assert r == o["radius"], inst
            loops += len(o["iters"]) > 0
    assert loops == 3   # the eps = 0.1 instance of every d samples


def _mrg_check(kc, orc, X, off, k, h):
    """MRG through the single-problem call with its details: every round-1
    partition's sequence and round 2's are certified farthest points
    (oracle replay); the union is the ascending set of round-1 centers; the
    radius is the exact covering radius of the centers."""
    Xd = torch.from_numpy(X).cuda()
    c, nc, r, det = on_stream(lambda: kc.mrg(Xd, off, k, handle=h, details=True))
    c = c.cpu().numpy()
    nc = int(nc.item())
    r1 = det["round1"].cpu().numpy().reshape(len(off) - 1, k)
    uni = det["union"].cpu().numpy()[:int(det["n_union"].item())]
    allc = []
    for p in range(len(off) - 1):
        lo, hi = int(off[p]), int(off[p + 1])
        if hi == lo:
            continue
        seq = r1[p][r1[p] >= 0]
        allc.append(seq)
        bad, _, _ = orc.gon_replay(X[lo:hi], k, seq - lo, band(X.shape[1]))
        assert bad == -1, "partition %d" % p
    assert np.array_equal(uni, np.sort(np.concatenate(allc)))
    loc = np.searchsorted(uni, c[:nc])
    bad, _, _ = orc.gon_replay(X[uni], k, loc, band(X.shape[1]))
    assert bad == -1
    _, R = orc.assign(X, c[:nc])
    assert float(r.item()) == R
    return c, nc, float(r.item())


def _eim_first_iteration(kc, orc, X, inst, h):
    """A larger EIM instance: its first iteration's draws (sizes), threshold
    over all of H, and 10,000 seeded keep / remove decisions equal the
    oracle's; the final Gonzalez is replayed on the sample."""
    n, k = len(X), inst["k"]
    Xd = torch.from_numpy(X).cuda()
    c, nc, r, smp, its = on_stream(lambda: kc.eim(Xd, k, inst["eps"], inst["phi"],
                                                  inst["seed"], handle=h))
    smp = smp.cpu().numpy()
    assert len(its) >= 1
    it0 = its[0]
    L = math.log(n)
    ne = math.pow(n, inst["eps"])
    assert it0["p_s"] == min(1.0, 9.0 * k * ne * L / n)
    assert it0["p_h"] == min(1.0, 4.0 * ne * L / n)
    f = orc.eim_draw_flags(inst["seed"], 0, np.arange(n), it0["p_s"], it0["p_h"])
    S = np.flatnonzero(f & 1)
    H = np.flatnonzero(f & 2)
    assert len(S) == it0["ds_size"] and len(H) == it0["h_size"]
    dH = np.sort([orc.min_dist2_to_set(X, int(x), S)[0] for x in H])[::-1]
    rr = min(max(1, math.ceil(inst["phi"] * L)), len(H))
    assert it0["tau"] == dH[rr - 1]
    # S joins the sample; a point outside S stays iff d(x,S)^2 > tau (after
    # one iteration the sample is S and the kept points; after more, a point
    # removed in the first is still outside it)
    assert np.all(np.isin(S, smp))
    rest = np.setdiff1d(np.arange(n), S)
    pick = np.random.default_rng(inst["id"]).choice(rest, min(10_000, len(rest)), replace=False)
    # d(x, S)^2 of the picked points: the oracle's assignment of [X[pick];
    # X[S]] to the S rows (its per-point minimum, FP64)
    Y = np.concatenate([X[pick], X[S]])
    _, _, md = orc.assign(Y, np.arange(len(pick), len(Y)), want_mind=True)
    in_smp = np.isin(pick, smp)
    for x, dm, got in zip(pick, md[:len(pick)], in_smp):
        keep = dm > it0["tau"]
        if len(its) == 1 or not keep:
            assert keep == bool(got), x
    # the final Gonzalez on the sample, replayed; exact radius
    nc = int(nc.item())
    cc = c.cpu().numpy()[:nc]
    loc = np.searchsorted(smp, cc)
    bad, _, _ = orc.gon_replay(X[smp], k, loc, band(X.shape[1]))
    assert bad == -1
    _, R = orc.assign(X, cc)
    assert float(r.item()) == R


def _pick(idx, insts, cost, count=15, d32=3):
    """The `count` cheapest instances by oracle cost, at least `d32` of them
    at d = 32."""
    order = sorted(idx, key=cost)
    with32 = [i for i in order if insts[i]["d"] == 32][:d32]
    rest = [i for i in order if i not in with32][:count - len(with32)]
    return with32 + rest


@pytest.mark.slow
def test_batch_config5_oracle(kc, orc):
    orc.set_threads(16)
    insts = W.config5_instances()
    probs, hosts = [], []
    for inst in insts:
        X, off = W.config5_points(inst)
        pr = dict(X=torch.from_numpy(X).cuda(), algo=inst["algo"], k=inst["k"])
        if off is not None:
            pr["offsets"] = off
        if inst["algo"] == "eim":
            pr.update(eps=inst["eps"], phi=inst["phi"], seed=inst["seed"])
        probs.append(pr)
        hosts.append(X)
    h, res = run_batch(kc, probs)

    def loops(i):
        t = insts[i]
        return t["n"] > (4 / t["eps"]) * t["k"] * t["n"] ** t["eps"] * math.log(t["n"])

    gon = [i for i, t in enumerate(insts) if t["algo"] == "gon"]
    mrg = [i for i, t in enumerate(insts) if t["algo"] == "mrg"]
    eim = [i for i, t in enumerate(insts) if t["algo"] == "eim"]
    cost = lambda i: insts[i]["n"] * insts[i]["k"] * insts[i]["d"]
    checked = {"gon": 0, "mrg": 0, "eim": 0}
    d32 = {"gon": 0, "mrg": 0, "eim": 0}
    for i in _pick(gon, insts, cost):
        X, (c, nc, r) = hosts[i], res[i]
        bad, _, _ = orc.gon_replay(X, insts[i]["k"], c[:nc], band(X.shape[1]))
        assert bad == -1, insts[i]
        _, R = orc.assign(X, c[:nc])
        assert r == R
        checked["gon"] += 1
        d32["gon"] += insts[i]["d"] == 32
    for i in _pick(mrg, insts, cost):
        c, nc, r = _mrg_check(kc, orc, hosts[i], probs[i]["offsets"], insts[i]["k"], h)
        assert (nc, r) == res[i][1:] and np.array_equal(c, res[i][0]), insts[i]
        checked["mrg"] += 1
        d32["mrg"] += insts[i]["d"] == 32
    # EIM: the cheapest instances in full (sample, records, replay), two
    # sampling ones among them; two larger sampling ones by their first
    # iteration
    small_loop = sorted([i for i in eim if loops(i)], key=lambda i: insts[i]["n"])
    full = _pick([i for i in eim if not loops(i)], insts, cost, 13) + small_loop[:2]
    for i in full:
        t = insts[i]
        o = orc.eim(hosts[i], t["k"], t["eps"], t["phi"], t["seed"])
        c, nc, r = res[i]
        C = o["sample"]
        loc = np.searchsorted(C, c[:nc])
        assert np.array_equal(C[loc], c[:nc]), t
        bad, _, _ = orc.gon_replay(hosts[i][C], t["k"], loc, band(t["d"]))
        assert bad == -1, t
        _, R = orc.assign(hosts[i], c[:nc])
        assert r == R
        checked["eim"] += 1
        d32["eim"] += t["d"] == 32
    one_iter = [i for i in small_loop[2:] if insts[i]["n"] < 700_000][:2]
    for i in one_iter:
        _eim_first_iteration(kc, orc, hosts[i], insts[i], h)
        d32["eim"] += insts[i]["d"] == 32
    h.close()
    assert all(v >= 15 for v in checked.values()), checked
    assert all(v >= 3 for v in d32.values()), d32
