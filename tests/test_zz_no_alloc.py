"""kcenter_gonzalez_noalloc (the entry point that allocates no device memory)
against kcenter_gonzalez: two calls in a row on one handle, the second with
a smaller input, each compared element by element with the allocating entry
point's outputs on the same points (and, on integer coordinates, with the
FP64 oracle bit for bit)."""
import ctypes

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


def _pair(kc, h, Xd, k, first):
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        a = kc.gonzalez_noalloc(Xd, k, first, handle=h)
        b = kc.gonzalez(Xd, k, first, handle=h)
        st.synchronize()
        assert h.device_status() == 0
    return [tuple(t.cpu().numpy() for t in r) for r in (a, b)]


def _same(a, b):
    assert np.array_equal(a[0], b[0])          # centers
    assert np.array_equal(a[1], b[1])          # trace, bit for bit
    assert np.array_equal(a[2], b[2])          # n_chosen


@pytest.mark.parametrize("resident", [True, False])
def test_intgrid_two_calls_shrinking(kc, orc, resident, rows_layout):
    h = kc.Handle(resident=resident)
    X = W.config2(300_000)
    for n, k, first, layout in ((300_000, 400, 0, "dense"), (70_001, 150, 9, "odd")):
        Xn = np.ascontiguousarray(X[:n])
        Xd = rows_layout(Xn, layout)
        a, b = _pair(kc, h, Xd, k, first)
        _same(a, b)
        oc, otr, og = orc.gon(Xn, k, first)
        assert int(a[2][0]) == og
        assert np.array_equal(a[0], oc) and np.array_equal(a[1], otr)
    h.close()


@pytest.mark.parametrize("resident", [True, False])
def test_float_two_calls_shrinking(kc, resident):
    h = kc.Handle(resident=resident)
    X = W.points_gauss_mixture(200_000, 16, 20, seed=77)
    for n, k, first in ((200_000, 256, 0), (5_000, 37, 4_999)):
        Xd = torch.from_numpy(np.ascontiguousarray(X[:n])).cuda()
        a, b = _pair(kc, h, Xd, k, first)
        _same(a, b)
    h.close()


def test_early_stop_and_tiny(kc, orc):
    # fewer distinct points than k: the run stops, then a one-point input
    h = kc.Handle()
    X = np.repeat(np.arange(6, dtype=np.float32)[:, None], 3, axis=1)
    X = np.repeat(X, 50, axis=0)
    for Xn, k in ((X, 20), (X[:1], 3)):
        Xd = torch.from_numpy(np.ascontiguousarray(Xn)).cuda()
        a, b = _pair(kc, h, Xd, k, 0)
        _same(a, b)
        oc, otr, og = orc.gon(Xn, k, 0)
        assert int(a[2][0]) == og and np.array_equal(a[0], oc)
    h.close()


def test_rejects_beyond_scratch(kc):
    # the size check runs on the host before any work: a request needing
    # more than the fixed array is refused with KC_EINVAL, and a BF16 one
    # with KC_EUNSUPPORTED
    h = kc.Handle()
    Xd = torch.zeros((8, 4), dtype=torch.float32, device="cuda")
    L = kc.load_library()
    p = kc.points(Xd)
    p.n = 3_000_000          # 36 MB of min-distances and candidates alone
    out = [torch.empty(4, dtype=torch.int64, device="cuda"),
           torch.empty(4, dtype=torch.float64, device="cuda"),
           torch.empty(1, dtype=torch.int64, device="cuda")]
    rc = L.kcenter_gonzalez_noalloc(h._h, ctypes.byref(p), 4, 0,
                                    *[ctypes.c_void_p(t.data_ptr()) for t in out],
                                    ctypes.c_void_p(None))
    assert rc == -1 and b"limit" in L.kc_last_error(h._h)
    p = kc.points(Xd, Xd.to(torch.bfloat16))
    rc = L.kcenter_gonzalez_noalloc(h._h, ctypes.byref(p), 4, 0,
                                    *[ctypes.c_void_p(t.data_ptr()) for t in out],
                                    ctypes.c_void_p(None))
    assert rc == -6
    h.close()
