"""The autotuner measures variants that must give identical results: a
handle that tunes (and so runs every feasible variant of the first call of
each shape bucket) returns exactly what an untuned handle returns, on the
tuning call and on the calls that reuse the cached choice; the report names
the buckets it measured."""
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


def host(t):
    return [x.cpu().numpy() if isinstance(x, torch.Tensor) else x for x in t]


@pytest.mark.parametrize("n,d,k", [(300_000, 8, 64), (120_000, 32, 200), (5_000, 3, 17)])
def test_gonzalez_tuned_equals_untuned(kc, n, d, k):
    X = torch.from_numpy(W.points_gauss_mixture(n, d, 20, seed=n + d)).cuda()
    ref_h = kc.Handle()
    ref_h.set_option("autotune", 0)
    ref = host(on_stream(lambda: kc.gonzalez(X, k, first=3, handle=ref_h)))
    h = kc.Handle()
    for _ in range(3):   # tuning call, then the cached choice
        got = host(on_stream(lambda: kc.gonzalez(X, k, first=3, handle=h)))
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
        assert h.device_status() == 0
    rep = h.tune_report()
    keys = [key for key in rep if key.startswith("gon/%d/" % d)]
    assert len(keys) == 1
    var, ms = rep[keys[0]]
    assert 0 <= var < len(ms) and ms[var] >= 0
    assert all(ms[var] <= t for t in ms if t >= 0)
    ref_h.close()
    h.close()


@pytest.mark.parametrize("d", [8, 32])
def test_eim_tuned_equals_untuned(kc, d):
    n, k = 150_000, 10
    X = torch.from_numpy(W.points_gauss_mixture(n, d, 25, seed=77 + d, heavy=0.9)).cuda()
    seed = 3 * 2**32 + d

    def run(h):
        c, nc, r, smp, its = on_stream(lambda: kc.eim(X, k, 0.1, 4.0, seed, handle=h))
        assert h.device_status() == 0
        return c.cpu().numpy(), int(nc.item()), float(r.item()), smp.cpu().numpy(), its

    ref_h = kc.Handle()
    ref_h.set_option("autotune", 0)
    ref = run(ref_h)
    assert len(ref[4]) >= 1   # the instance samples
    h = kc.Handle()
    for _ in range(2):
        got = run(h)
        assert np.array_equal(ref[0], got[0]) and ref[1:3] == got[1:3]
        assert np.array_equal(ref[3], got[3])
        assert ref[4] == got[4]
    rep = h.tune_report()
    keys = [key for key in rep if key.startswith("eim/%d/" % d)]
    assert len(keys) >= 1
    for key in keys:
        var, ms = rep[key]
        assert ms[var] >= 0
        if d > 8:
            assert ms[0] == -1   # the direct pass is for d <= 8 only
    ref_h.close()
    h.close()


def test_tune_report_size_query(kc):
    h = kc.Handle()
    assert h.tune_report() == {}
    h.close()
