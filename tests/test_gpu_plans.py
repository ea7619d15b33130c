"""Calls that share a handle: the cached HIP graphs must follow each call's
plan (partition offsets, problem sizes), and table uploads must be ordered on
the caller's stream after the work already queued there.  Integer-coordinate
inputs, so every result is compared with the FP64 oracle bit for bit."""
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


def _intpts(n, d, seed):
    rng = np.random.default_rng(seed)
    X = rng.integers(0, 14, (n, d)).astype(np.float32)
    X[: n // 4] += 40.0          # clusters, so partitions differ
    return X


@pytest.mark.parametrize("resident", [True, False])
def test_mrg_same_sizes_different_offsets(kc, orc, resident):
    # equal n, m and k; the second call's partitions hold more 1024-point
    # tiles in all than the first call's
    n, m, k = 60_000, 4, 24
    X = _intpts(n, 6, 71)
    Xd = torch.from_numpy(X).cuda()
    offs = [np.array([0, 1000, 2000, 3000, n], np.int64),
            np.array([0, 14_500, 29_500, 44_500, n], np.int64)]
    h = kc.Handle(resident=resident)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    outs = []
    with torch.cuda.stream(st):
        for off in offs + offs:
            c, nc, r = kc.mrg(Xd, off, k, handle=h)
            st.synchronize()
            outs.append((c.cpu().numpy(), int(nc.item()), float(r.item())))
        assert h.device_status() == 0
    h.close()
    for (c, nc, r), off in zip(outs, offs + offs):
        o = orc.mrg(X, off, k)
        assert nc == o["n_centers"]
        assert np.array_equal(c, o["centers"]) and r == o["radius"]


def test_batch_prefix_views(kc, orc):
    # the same array, first as its first n1 rows, then as its first n2
    X = _intpts(40_000, 8, 72)
    Xd = torch.from_numpy(X).cuda()
    h = kc.Handle()
    res = []
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        for n in (9_000, 37_000, 9_000):
            off = W.equal_offsets(n, 8)
            probs = [dict(X=Xd[:n], algo="gon", k=30, first=3),
                     dict(X=Xd[:n], algo="mrg", k=20, offsets=off)]
            outs = kc.batch(probs, handle=h)
            st.synchronize()
            res.append((n, off, [(o[0].cpu().numpy(), int(o[1].item()),
                                  float(o[2].item())) for o in outs]))
        assert h.device_status() == 0
    h.close()
    for n, off, ((cg, ng, rg), (cm, nm, rm)) in res:
        oc, otr, og = orc.gon(X[:n], 30, 3)
        assert ng == og and np.array_equal(cg, oc) and rg == otr[og - 1]
        o = orc.mrg(X[:n], off, 20)
        assert nm == o["n_centers"] and np.array_equal(cm, o["centers"])
        assert rm == o["radius"]


@pytest.mark.parametrize("resident", [True, False])
def test_back_to_back_calls_one_sync(kc, orc, resident):
    # calls with different first centers and offsets enqueued back to back
    # on one stream and synchronised once: each reports its own arguments
    n = 30_000
    X = _intpts(n, 10, 73)
    Xd = torch.from_numpy(X).cuda()
    h = kc.Handle(resident=resident)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    firsts = (0, 5, 29_999, 5)
    offs = [W.equal_offsets(n, 3), np.array([0, 100, 20_000, n], np.int64)]
    with torch.cuda.stream(st):
        g = [kc.gonzalez(Xd, 40, f, handle=h) for f in firsts]
        mr = [kc.mrg(Xd, off, 16, handle=h) for off in offs]
        st.synchronize()
        assert h.device_status() == 0
    h.close()
    for f, (c, tr, nc) in zip(firsts, g):
        oc, otr, og = orc.gon(X, 40, f)
        assert int(nc.item()) == og
        assert np.array_equal(c.cpu().numpy(), oc)
        assert np.array_equal(tr.cpu().numpy(), otr)
    for off, (c, nc, r) in zip(offs, mr):
        o = orc.mrg(X, off, 16)
        assert np.array_equal(c.cpu().numpy(), o["centers"])
        assert float(r.item()) == o["radius"]
