"""GPU parity of kcenter_mrg_rounds (Algorithm 1 with its loop and machine
capacity c) against the FP64 oracle.

On integer coordinates (exact FP32 squared distances) every pass chooses the
oracle's centers, so the final centers, their count, the number of rounds and
the covering radius must be equal.  On float coordinates the radius must be
the exact covering radius of the GPU's centers."""
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


def run(kc, X, k, c, resident=True):
    h = kc.Handle(resident=resident)
    Xd = torch.from_numpy(X).cuda()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        cen, nc, r, rounds = kc.mrg_rounds(Xd, k, c, handle=h)
        assert h.device_status() == 0
    st.synchronize()
    out = cen.cpu().numpy(), int(nc.item()), float(r.item()), rounds
    h.close()
    return out


def int_points(n, d, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(-60, 61, (n, d)).astype(np.float32)


# (n, k, c): several passes of many small blocks; one pass; capacity >= n
# (plain Gonzalez, one round); blocks smaller than k in a later pass
@pytest.mark.parametrize("n,k,c,resident", [
    (120_000, 40, 1_000, True),
    (120_000, 40, 1_000, False),
    (20_000, 7, 100, True),
    (50_000, 20, 25_000, True),
    (30_000, 25, 30_000, True),
    (9_000, 30, 70, True),
])
def test_mrg_rounds_integer_exact(kc, orc, n, k, c, resident):
    X = int_points(n, 8, n + k + c)
    cen, nc, r, rounds = run(kc, X, k, c, resident)
    o = orc.mrg_rounds(X, k, c)
    assert rounds == o["rounds"]
    assert nc == o["n_centers"]
    assert np.array_equal(cen, o["centers"])
    assert r == o["radius"]


@pytest.mark.parametrize("layout", ["wide", "shift"])
def test_mrg_rounds_row_layouts(kc, orc, rows_layout, layout):
    # the first pass reads the caller's (strided or misaligned) rows
    X = int_points(60_000, 10, 13)
    k, c = 30, 4_000
    h = kc.Handle()
    Xd = rows_layout(X, layout)
    cen, nc, r, rounds = kc.mrg_rounds(Xd, k, c, handle=h)
    torch.cuda.synchronize()
    assert h.device_status() == 0
    o = orc.mrg_rounds(X, k, c)
    assert int(nc.item()) == o["n_centers"] and rounds == o["rounds"]
    assert np.array_equal(cen.cpu().numpy()[:o["n_centers"]], o["centers"][:o["n_centers"]])
    assert float(r.item()) == o["radius"]
    h.close()


def test_mrg_rounds_no_progress(kc, orc):
    # blocks of at most 40 points and k = 50: a pass keeps every point
    X = int_points(5_000, 4, 3)
    assert orc.mrg_rounds(X, 50, 40)["radius"] == -1
    with pytest.raises(kc.KCenterError) as e:
        run(kc, X, 50, 40)
    assert e.value.status == -4


def test_mrg_rounds_gauss(kc, orc):
    X, _ = W.config3(200_000, 16)
    cen, nc, r, rounds = run(kc, X, 30, 2_000)
    o = orc.mrg_rounds(X, 30, 2_000)
    assert rounds == o["rounds"] == 3
    _, R = orc.assign(X, cen[:nc])
    assert r == R
    if np.array_equal(cen, o["centers"]):
        assert r == o["radius"]
