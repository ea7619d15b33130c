"""GPU parity of kcenter_gonzalez against the FP64 oracle.

Integer-coordinate inputs (exact FP32 squared distances) must match the
oracle bit for bit: centers, trace and radius.  Float inputs are replayed
through the oracle: every GPU choice must be a farthest point up to the FP32
error band 2*gamma_{d+2} (a certified tie), and the final radius -- the exact
FP64 covering radius of the GPU's centers -- must equal the oracle's value
for those centers."""
import numpy as np
import pytest

from paper_1604_03228_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def band(d):
    m = d + 2
    g = m * U32 / (1 - m * U32)
    return 2 * g + 1e-12


@pytest.fixture(scope="module")
def kc():
    import paper_1604_03228_amd as kc
    assert torch.cuda.is_available()
    return kc


def run_gon(kc, X, k, first=0, resident=True, graphs=True):
    # a non-default stream, so that graph capture is exercised
    h = kc.Handle(graphs=graphs, resident=resident)
    Xd = torch.from_numpy(X).cuda()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        c, tr, nch = kc.gonzalez(Xd, k, first, handle=h)
        assert h.device_status() == 0
    torch.cuda.synchronize()
    out = c.cpu().numpy(), tr.cpu().numpy(), int(nch.item())
    h.close()
    return out


def check_float(orc, X, k, first, c, tr, got):
    seq = c[:got]
    bad, ties, otr = orc.gon_replay(X, k, seq, band(X.shape[1]))
    assert bad == -1, "step %d not a certified farthest point" % bad
    # final radius: exact FP64 covering radius of the GPU's centers
    _, R = orc.assign(X, seq)
    assert tr[got - 1] == R
    # trace entries: FP64 distance of each chosen point, within the band of
    # the oracle's maximum along the same sequence
    rel = np.abs(tr[:got] - otr) / np.maximum(otr, 1e-300)
    assert np.all(rel <= band(X.shape[1]))
    assert np.all(tr[got:] == 0)
    return ties


@pytest.mark.parametrize("resident", [True, False])
def test_config1_uniform(kc, orc, resident):
    X = W.config1()
    c, tr, got = run_gon(kc, X, 20, 0, resident=resident)
    assert got == 20
    ties = check_float(orc, X, 20, 0, c, tr, got)
    oc, otr, _ = orc.gon(X, 20, 0)
    if ties == 0:
        assert np.array_equal(c, oc)
    assert abs(tr[-1] - otr[-1]) <= 1e-6 * otr[-1]


@pytest.mark.parametrize("n,resident", [(50_000, True), (50_000, False),
                                        (1_000_000, True), (1_000_000, False)])
def test_config2_intgrid_bitexact(kc, orc, n, resident):
    X = W.config2(n)
    k = 1000 if n == 1_000_000 else 300
    orc.set_threads(16)
    oc, otr, og = orc.gon(X, k, 0)
    c, tr, got = run_gon(kc, X, k, 0, resident=resident)
    assert got == og
    assert np.array_equal(c, oc)
    assert np.array_equal(tr, otr)


def test_resident_candidate_cap(kc, orc):
    # Two far points inside every wave's share of the register-resident
    # layout (d = 10: point g*4096 + p*256 + w*64 + lane sits in lane `lane`
    # of wave w of block g), the rest on the {0,1} grid, first center on the
    # grid: every wave's two largest keys are far points and its third is a
    # grid point, so about 600 published keys exceed the round's bound and
    # the candidate cap (a raised bound) applies.  Exact integer distances.
    rng = np.random.default_rng(7)
    n, d = 300_000, 10
    X = rng.integers(0, 2, (n, d)).astype(np.float32)
    far = np.array([g * 4096 + w * 64 + l for g in range((n + 4095) // 4096)
                    for w in range(4) for l in (0, 1)])
    far = far[far < n]
    X[far] = rng.integers(100, 1000, (len(far), d)).astype(np.float32)
    k = 800
    orc.set_threads(16)
    oc, otr, og = orc.gon(X, k, 2)
    assert set(far) <= set(oc[:len(far) + 1])
    for resident in (True, False):
        c, tr, got = run_gon(kc, X, k, 2, resident=resident)
        assert got == og
        assert np.array_equal(c, oc)
        assert np.array_equal(tr, otr)


# The resident engine's large variant (4,032 points per block at d = 16
# instead of 2,688) takes inputs beyond the balanced variant's grid: forced
# by a 4-block cap at 15,000 points, and at 800,000 points by the
# co-resident grid itself (at most 256 blocks hold 688,128 points).
@pytest.mark.parametrize("n,cap", [(15_000, 4), (800_000, 0)])
def test_resident_large_variant(kc, orc, n, cap):
    rng = np.random.default_rng(n)
    X = rng.integers(-50, 51, (n, 16)).astype(np.float32)
    k = 64
    h = kc.Handle()
    h.set_option("resident_blocks", cap)
    h.set_option("autotune", 0)   # the resident engine, not a measured choice
    h.set_option("timing", 1)
    Xd = torch.from_numpy(X).cuda()
    c, tr, nch = kc.gonzalez(Xd, k, 3, handle=h)
    assert h.device_status() == 0
    _, la, iv = h.timing_read("gon_resident")
    assert (la, iv) == (1, 1)
    oc, otr, og = orc.gon(X, k, 3)
    assert int(nch.item()) == og
    assert np.array_equal(c.cpu().numpy(), oc)
    assert np.array_equal(tr.cpu().numpy(), otr)
    h.close()


@pytest.mark.parametrize("d", [3, 10, 16])
@pytest.mark.parametrize("layout", ["dense", "wide", "odd", "shift"])
def test_resident_row_layouts(kc, orc, rows_layout, d, layout):
    # integer coordinates: centers and trace bit-exact against the oracle;
    # several tiles per block and a ragged tail
    rng = np.random.default_rng(7 * d + len(layout))
    n = 50_037
    X = rng.integers(-20, 21, (n, d)).astype(np.float32)
    k = 48
    h = kc.Handle()
    h.set_option("autotune", 0)   # the resident engine, not a measured choice
    h.set_option("timing", 1)
    Xd = rows_layout(X, layout)
    c, tr, nch = kc.gonzalez(Xd, k, 5, handle=h)
    assert h.device_status() == 0
    _, la, _ = h.timing_read("gon_resident")
    assert la == 1
    oc, otr, og = orc.gon(X, k, 5)
    assert int(nch.item()) == og
    assert np.array_equal(c.cpu().numpy(), oc)
    assert np.array_equal(tr.cpu().numpy(), otr)
    h.close()


def test_config2_prefix(kc):
    X = W.config2(200_000)
    c1, t1, _ = run_gon(kc, X, 100, 0)
    c2, t2, _ = run_gon(kc, X, 1000, 0)
    assert np.array_equal(c1, c2[:100])
    assert np.array_equal(t1[:99], t2[:99])


@pytest.mark.parametrize("d", [1, 2, 3, 5, 8, 10, 16, 32, 41, 70])
@pytest.mark.parametrize("resident", [True, False])
def test_dims_ragged(kc, orc, d, resident):
    # n not a multiple of 4, 64 or the tile; generic and unrolled dims
    rng = np.random.default_rng(100 + d)
    n = 7_919
    X = rng.normal(size=(n, d)).astype(np.float32)
    k = 37
    c, tr, got = run_gon(kc, X, k, 11, resident=resident)
    assert got == k and c[0] == 11
    check_float(orc, X, k, 11, c, tr, got)


@pytest.mark.parametrize("resident", [True, False])
def test_early_stop_duplicates(kc, orc, resident):
    base = np.random.default_rng(5).integers(0, 9, (13, 3)).astype(np.float32)
    base = np.unique(base, axis=0)
    X = np.repeat(base, 40, axis=0)
    k = 50
    c, tr, got = run_gon(kc, X, k, 0, resident=resident)
    oc, otr, og = orc.gon(X, k, 0)
    assert got == og == len(base)
    assert np.array_equal(c, oc) and np.array_equal(tr, otr)
    assert np.all(c[got:] == -1)


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 1023, 1024, 1025])
def test_tiny_and_tile_edges(kc, orc, n):
    X = np.random.default_rng(n).integers(-50, 50, (n, 4)).astype(np.float32)
    k = min(n + 2, 30)
    for resident in (True, False):
        c, tr, got = run_gon(kc, X, k, n // 2, resident=resident)
        oc, otr, og = orc.gon(X, k, n // 2)
        assert got == og and np.array_equal(c, oc) and np.array_equal(tr, otr)


def test_graphs_off_and_repeat(kc):
    X = W.config2(100_000)
    a = run_gon(kc, X, 200, 3, resident=False, graphs=False)
    b = run_gon(kc, X, 200, 3, resident=False, graphs=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    h = kc.Handle(resident=False)
    Xd = torch.from_numpy(X).cuda()
    outs = []
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    for _ in range(3):   # replays of one captured graph, eager work between
        with torch.cuda.stream(st):
            c, tr, nch = kc.gonzalez(Xd, 200, 3, handle=h)
        st.synchronize()
        outs.append((c.cpu().numpy().copy(), tr.cpu().numpy().copy()))
        torch.zeros(1000, device="cuda").sum().item()
    for o in outs:
        assert np.array_equal(o[0], a[0]) and np.array_equal(o[1], a[1])


def test_invalid_arguments(kc):
    h = kc.Handle()
    X = torch.zeros(10, 3, device="cuda")
    with pytest.raises(kc.KCenterError) as e:
        kc.gonzalez(X, 0, 0, handle=h)
    assert e.value.status == -1
    with pytest.raises(kc.KCenterError):
        kc.gonzalez(X, 3, 10, handle=h)
    with pytest.raises(kc.KCenterError):
        kc.gonzalez(X, 3, -1, handle=h)
    with pytest.raises(ValueError):
        kc.gonzalez(X.t(), 3, 0, handle=h)


# The one-workgroup engine (tune_force = 3; it holds up to 1,024 lanes x
# 20 / 16 / 8 / 7 / 4 points at d = 2 / 3 / 8 / 10 / 16): integer
# coordinates, centers, trace and count bit-exact against the oracle, at
# ragged sizes up to its capacity, with k = 1, early stops and a first
# center past the middle.
@pytest.mark.parametrize("d,n", [(2, 1), (2, 1025), (2, 20_000), (2, 20_480), (3, 16_384),
                                 (8, 5_000), (10, 7_168), (16, 4_096)])
@pytest.mark.parametrize("k", [1, 7, 200])
def test_block_engine(kc, orc, d, n, k):
    X = np.random.default_rng(n + d).integers(-30, 31, (n, d)).astype(np.float32)
    h = kc.Handle()
    h.set_option("tune_force", 3)
    h.set_option("timing", 1)
    Xd = torch.from_numpy(X).cuda()
    first = (2 * n) // 3
    c, tr, nch = kc.gonzalez(Xd, k, first, handle=h)
    assert h.device_status() == 0
    _, la, _ = h.timing_read("gon_block")
    assert la == 1
    oc, otr, og = orc.gon(X, k, first)
    assert int(nch.item()) == og
    assert np.array_equal(c.cpu().numpy(), oc)
    assert np.array_equal(tr.cpu().numpy(), otr)
    h.close()


def test_block_engine_early_stop(kc, orc):
    base = np.random.default_rng(9).integers(0, 9, (11, 2)).astype(np.float32)
    base = np.unique(base, axis=0)
    X = np.repeat(base, 700, axis=0)
    h = kc.Handle()
    h.set_option("tune_force", 3)
    c, tr, nch = kc.gonzalez(torch.from_numpy(X).cuda(), 40, 0, handle=h)
    oc, otr, og = orc.gon(X, 40, 0)
    got = int(nch.item())
    assert got == og == len(base)
    assert np.array_equal(c.cpu().numpy(), oc) and np.array_equal(tr.cpu().numpy(), otr)
    h.close()
