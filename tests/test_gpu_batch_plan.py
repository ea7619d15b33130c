"""kcenter_batch_plan / run / free: a batch planned once and run several
times returns, on every run, what kcenter_batch returns for the same
problems (whose results test_gpu_batch5.py checks against the oracle);
runs read the points' current values; errors are reported on the host."""
import numpy as np
import pytest

from paper_1604_03228_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def problems(seed=0):
    """GON, MRG and EIM problems at d in {2, 8, 32} with integer coordinates
    (exact FP32 distances), one of them too large for the resident grid at
    d = 32 so that both groups of that dimension run."""
    out = []
    for j, d in enumerate((2, 8, 32)):
        n = 9_000 + 1_000 * d
        X = np.round(W.points_gauss_mixture(n, d, 25, seed=seed + d, heavy=0.9)).astype(np.float32)
        Xd = torch.from_numpy(X).cuda()
        out.append(dict(X=Xd, algo="gon", k=23 + j, first=5))
        out.append(dict(X=Xd, algo="mrg", k=17, offsets=W.partition_offsets(n, 8, 0.5, seed=d)))
        out.append(dict(X=Xd, algo="eim", k=10, eps=0.1, phi=4.0, seed=7 * 2**32 + d))
    big = np.round(W.points_gauss_mixture(1_200_000, 32, 25, seed=seed + 99,
                                          heavy=0.9)).astype(np.float32)
    out.append(dict(X=torch.from_numpy(big).cuda(), algo="gon", k=12, first=1))
    return out


def host(outs):
    return [(c.cpu().numpy(), int(nc.item()), float(r.item())) for c, nc, r in outs]


def test_plan_runs_equal_batch(kc):
    probs = problems()
    h = kc.Handle()
    ref = host(on_stream(lambda: kc.batch(probs, handle=h)))
    assert h.device_status() == 0
    plan = kc.BatchPlan(probs, handle=h)
    for _ in range(3):
        got = host(on_stream(plan.run))
        assert h.device_status() == 0
        for (a, na, ra), (b, nb, rb) in zip(ref, got):
            assert na == nb and np.array_equal(a[:na], b[:nb]) and ra == rb
    # new values, same shapes: coordinates doubled (still exact in FP32)
    # keep every center sequence and double every radius
    for X in {id(pr["X"]): pr["X"] for pr in probs}.values():   # shared tensors once
        X.mul_(2.0)
    got = host(on_stream(plan.run))
    for (a, na, ra), (b, nb, rb) in zip(ref, got):
        assert na == nb and np.array_equal(a[:na], b[:nb]) and rb == 2.0 * ra
    plan.close()
    plan.close()   # idempotent
    h.close()


def test_plan_matches_oracle(kc, orc):
    orc.set_threads(16)
    probs = problems(seed=3)[:9]
    plan = kc.BatchPlan(probs)
    got = host(on_stream(plan.run))
    plan.close()
    for pr, (c, nc, r) in zip(probs, got):
        X = pr["X"].cpu().numpy()
        if pr["algo"] == "gon":
            oc, otr, og = orc.gon(X, pr["k"], pr["first"])
            assert nc == og and np.array_equal(c[:nc], oc[:og]) and r == otr[og - 1]
        elif pr["algo"] == "mrg":
            o = orc.mrg(X, pr["offsets"], pr["k"])
            assert nc == o["n_centers"] and np.array_equal(c, o["centers"]) and r == o["radius"]
        else:
            o = orc.eim(X, pr["k"], pr["eps"], pr["phi"], pr["seed"])
            assert nc == o["n_centers"] and np.array_equal(c, o["centers"]) and r == o["radius"]


def test_plan_rejects_bad_problems(kc):
    X = torch.zeros(100, 3, device="cuda")
    with pytest.raises(kc.KCenterError):
        kc.BatchPlan([dict(X=X, algo="gon", k=5, first=100)])
    with pytest.raises(kc.KCenterError):
        kc.BatchPlan([dict(X=X, algo="mrg", k=5, offsets=[0, 50, 99])])
    plan = kc.BatchPlan([])
    assert plan.run() == []
    plan.close()
