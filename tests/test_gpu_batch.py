"""GPU parity of kcenter_batch: every problem of a mixed batch (Gonzalez,
MRG, EIM; d in {2, 8, 32}; uneven n and k) must give exactly the outputs of
its single-problem entry point, and those are checked against the FP64
oracle (bit-exact on integer coordinates, replay on floats)."""
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


def single(kc, pr, h):
    X = pr["X"]
    if pr["algo"] == "gon":
        c, tr, nc = kc.gonzalez(X, pr["k"], pr.get("first", 0), handle=h)
        g = int(nc.item())
        return c.cpu().numpy(), g, float(tr[g - 1].item())
    if pr["algo"] == "mrg":
        c, nc, r = kc.mrg(X, pr["offsets"], pr["k"], handle=h)
        return c.cpu().numpy(), int(nc.item()), float(r.item())
    c, nc, r, _, _ = kc.eim(X, pr["k"], pr["eps"], pr["phi"], pr["seed"],
                            handle=h)
    return c.cpu().numpy(), int(nc.item()), float(r.item())


def make_batch(insts):
    probs = []
    for inst in insts:
        X, off = W.config5_points(inst)
        pr = dict(X=torch.from_numpy(X).cuda(), Xh=X, algo=inst["algo"],
                  k=inst["k"])
        if off is not None:
            pr["offsets"] = off
        if inst["algo"] == "eim":
            pr.update(eps=inst["eps"], phi=inst["phi"], seed=inst["seed"])
        probs.append(pr)
    return probs


def run_and_compare(kc, probs):
    h = kc.Handle()
    outs = on_stream(lambda: kc.batch(probs, handle=h))
    assert h.device_status() == 0
    res = []
    for pr, (c, nc, r) in zip(probs, outs):
        got = (c.cpu().numpy(), int(nc.item()), float(r.item()))
        ref = on_stream(lambda: single(kc, pr, h))
        assert h.device_status() == 0
        assert got[1] == ref[1], pr["algo"]
        assert np.array_equal(got[0][:got[1]], ref[0][:ref[1]]), pr["algo"]
        assert got[2] == ref[2], pr["algo"]
        res.append(got)
    return res


def test_batch_small_mixed(kc, orc):
    insts = W.config5_instances(24, n_lo=500, n_hi=30_000, seed=11)
    probs = make_batch(insts)
    res = run_and_compare(kc, probs)
    # the oracle on every problem
    for inst, pr, (c, nc, r) in zip(insts, probs, res):
        X = pr["Xh"]
        k = inst["k"]
        if inst["algo"] == "gon":
            bad, _, _ = orc.gon_replay(X, k, c[:nc], band(X.shape[1]))
            assert bad == -1
        elif inst["algo"] == "mrg":
            o = orc.mrg(X, pr["offsets"], k)
            assert nc == o["n_centers"]
        else:
            o = orc.eim(X, k, inst["eps"], inst["phi"], inst["seed"])
            assert np.all(np.isin(c[:nc], o["sample"]))
        _, R = orc.assign(X, c[:nc])
        assert r == R


def test_batch_integer_exact(kc, orc):
    # integer coordinates: Gonzalez and MRG results equal the oracle exactly
    rng = np.random.default_rng(5)
    probs, hosts = [], []
    for i in range(10):
        n = int(rng.integers(300, 20_000))
        d = int(rng.choice([2, 8]))
        X = rng.integers(-60, 61, (n, d)).astype(np.float32)
        k = int(rng.integers(3, 60))
        pr = dict(X=torch.from_numpy(X).cuda(), algo="gon" if i % 2 else "mrg",
                  k=k)
        if pr["algo"] == "mrg":
            pr["offsets"] = W.partition_offsets(n, int(rng.integers(1, 9)),
                                                0.5, seed=i)
        else:
            pr["first"] = int(rng.integers(0, n))
        probs.append(pr)
        hosts.append(X)
    res = run_and_compare(kc, probs)
    for pr, X, (c, nc, r) in zip(probs, hosts, res):
        if pr["algo"] == "gon":
            oc, otr, og = orc.gon(X, pr["k"], pr["first"])
            assert nc == og and np.array_equal(c[:nc], oc[:og])
            assert r == otr[og - 1]
        else:
            o = orc.mrg(X, pr["offsets"], pr["k"])
            assert np.array_equal(c, o["centers"]) and r == o["radius"]


def test_batch_streamed_group_on_bf16_copy(kc, orc):
    # option resident = 0 streams every group; a streamed group of n points
    # with n (2d - 4) >= 1e8 runs on a BF16 copy the library rounds, with
    # exact rescoring: its centers and radii equal the FP32 single calls'
    # (both streamed); here 1.8e6 points at d = 32
    rng = np.random.default_rng(77)
    probs = []
    for i, (n, algo, k) in enumerate([(900_000, "gon", 60), (600_000, "mrg", 40),
                                      (300_000, "gon", 25)]):
        X = W.points_gauss_mixture(n, 32, 30, seed=500 + i)
        pr = dict(X=torch.from_numpy(X).cuda(), Xh=X, algo=algo, k=k)
        if algo == "mrg":
            pr["offsets"] = W.partition_offsets(n, 8, 0.5, seed=i)
        else:
            pr["first"] = int(rng.integers(0, n))
        probs.append(pr)
    h = kc.Handle(resident=False)
    outs = on_stream(lambda: kc.batch(probs, handle=h))
    assert h.device_status() == 0
    assert h.counter("bf16_listed") > 0    # the group did run the BF16 stream
    for pr, (c, nc, r) in zip(probs, outs):
        ref = on_stream(lambda: single(kc, pr, h))
        g = int(nc.item())
        assert g == ref[1]
        assert np.array_equal(c.cpu().numpy()[:g], ref[0][:g])
        assert float(r.item()) == ref[2]
    # the smallest against the oracle: a replay of its traversal
    pr, (c, nc, _) = probs[2], outs[2]
    g = int(nc.item())
    bad, _, _ = orc.gon_replay(pr["Xh"], pr["k"], c.cpu().numpy()[:g], band(32))
    assert bad == -1


@pytest.mark.slow
def test_batch_config5_full(kc, orc):
    orc.set_threads(16)
    insts = W.config5_instances()
    probs = make_batch(insts)
    res = run_and_compare(kc, probs)
    # sampled oracle checks: the smallest Gonzalez and MRG instances
    gon = sorted([i for i, t in enumerate(insts) if t["algo"] == "gon"],
                 key=lambda i: insts[i]["n"])[:3]
    for i in gon:
        X = probs[i]["Xh"]
        c, nc, r = res[i]
        bad, _, _ = orc.gon_replay(X, insts[i]["k"], c[:nc], band(X.shape[1]))
        assert bad == -1
        _, R = orc.assign(X, c[:nc])
        assert r == R
