"""GPU parity of kcenter_assign (MFMA + FP64 certification) and kcenter_mrg
(two-round MRG) against the FP64 oracle.

Assignment labels must equal the oracle's exactly (certified points by the
error bound, the rest rescored in FP64 with the oracle's arithmetic), and
the radius must equal the oracle's exact FP64 covering radius.  MRG on
integer coordinates (exact FP32 distances) must match the oracle in every
output; on float coordinates every round is replayed through the oracle
(certified ties only) and the radius is the exact one of the GPU's centers.
"""
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


def gpu_assign(kc, X, C, bf16=False, handle=None):
    h = handle or kc.Handle()
    Xd = torch.from_numpy(X).cuda()
    B = torch.from_numpy(W.to_bf16_rne(X).view(np.int16)).cuda() if bf16 else None
    Cd = torch.from_numpy(np.asarray(C, np.int64)).cuda()
    lab, r = on_stream(lambda: kc.assign(Xd, Cd, bf16=B, handle=h))
    assert h.device_status() == 0
    return lab.cpu().numpy(), float(r.item())


def mode_handle(kc, mode):
    """FP32 inputs run the distance pass on split BF16 MFMAs by default, or on
    the FP32 MFMA (option mfma_split = 0); "bf16" passes a BF16 copy."""
    h = kc.Handle()
    if mode == "fp32":
        h.set_option("mfma_split", 0)
    return h


@pytest.mark.parametrize("d", [1, 2, 5, 16, 41, 70])
@pytest.mark.parametrize("k", [1, 7, 200])
@pytest.mark.parametrize("mode", ["split", "fp32", "bf16"])
def test_assign_random(kc, orc, d, k, mode):
    rng = np.random.default_rng(1000 * d + k)
    n = 9_999
    X = (rng.normal(size=(n, d)) * rng.uniform(0.1, 50, d)).astype(np.float32)
    C = rng.choice(n, k, replace=False)
    lab, R = gpu_assign(kc, X, C, mode == "bf16", handle=mode_handle(kc, mode))
    olab, oR = orc.assign(X, C)
    assert np.array_equal(lab, olab)
    assert R == oR


@pytest.mark.parametrize("mode", ["split", "fp32", "bf16"])
def test_assign_ties_and_duplicates(kc, orc, mode):
    # integer grid: many exactly equal distances; duplicate centers too
    X = W.config2(30_000)
    c, _, _ = orc.gon(X, 64, 0)
    C = np.r_[c, c[:5], c[10:12]]
    lab, R = gpu_assign(kc, X, C, mode == "bf16", handle=mode_handle(kc, mode))
    olab, oR = orc.assign(X, C)
    assert np.array_equal(lab, olab) and R == oR


# BF16 inputs: the points whose label or radius bound the BF16 pass leaves
# open run a second MFMA pass on their FP32 rows (split, packed at 2,048
# centers, or the FP32 MFMA), FP64 after that; with and without labels
@pytest.mark.parametrize("d,k", [(3, 100), (16, 2048), (41, 500)])
@pytest.mark.parametrize("split", [1, 0])
@pytest.mark.parametrize("labels", [True, False])
def test_assign_bf16_second_pass(kc, orc, d, k, split, labels):
    X = W.points_gauss_mixture(12_000, d, 25, 0.0, 100.0, 0.2, 1.0, seed=60 + d)
    C = np.random.default_rng(d + k).choice(len(X), k, replace=False)
    h = kc.Handle()
    h.set_option("mfma_split", split)
    Xd = torch.from_numpy(X).cuda()
    B = torch.from_numpy(W.to_bf16_rne(X).view(np.int16)).cuda()
    lab, r = on_stream(lambda: kc.assign(Xd, torch.from_numpy(C), labels=labels, bf16=B,
                                         handle=h))
    assert h.device_status() == 0
    olab, oR = orc.assign(X, C)
    assert float(r.item()) == oR
    if labels:
        assert np.array_equal(lab.cpu().numpy(), olab)


def test_assign_radius_equals_gon(kc, orc):
    X = W.config1()
    c, tr, got = orc.gon(X, 20, 0)
    lab, R = gpu_assign(kc, X, c)
    assert R == tr[-1]


# Radius only (no labels): at d <= 8 the canonical FP32 distances bound each
# point's min-distance tightly (the direct pass); above, the MFMA bound.
# Data far from the origin with small clusters makes the MFMA bound loose;
# k = 1500 spans two chunks of the direct pass's staged centers.
@pytest.mark.parametrize("d", [1, 2, 5, 8, 16])
@pytest.mark.parametrize("k", [1, 7, 200, 1500])
def test_radius_only_far_from_origin(kc, orc, d, k):
    X = W.points_gauss_mixture(20_011, d, 25, 0.0, 100.0, 0.1, 0.1, seed=31 + d)
    C = np.random.default_rng(k + d).choice(len(X), k, replace=False)
    h = kc.Handle()
    h.set_option("timing", 1)
    Xd = torch.from_numpy(X).cuda()
    lab, r = on_stream(lambda: kc.assign(Xd, torch.from_numpy(C), labels=False, handle=h))
    assert lab is None and h.device_status() == 0
    _, la, _ = h.timing_read("assign_direct")
    assert la == (1 if d <= 8 else 0)
    _, oR = orc.assign(X, C)
    assert float(r.item()) == oR


# more centers than one LDS chunk holds, in both passes and with labels, in
# every block shape of the MFMA pass (tune_force: 4 / 8 waves per block with
# 64 KiB of staged centers, then with 32 KiB)
@pytest.mark.parametrize("d", [2, 16, 41])
@pytest.mark.parametrize("labels", [True, False])
@pytest.mark.parametrize("var", [0, 1, 2, 3])
def test_assign_many_centers(kc, orc, d, labels, var):
    rng = np.random.default_rng(50 + d)
    X = (rng.normal(size=(20_000, d)) * 10.0).astype(np.float32)
    C = rng.choice(len(X), 5_000, replace=False)
    h = kc.Handle()
    h.set_option("tune_force", var)
    Xd = torch.from_numpy(X).cuda()
    lab, r = on_stream(lambda: kc.assign(Xd, torch.from_numpy(C), labels=labels, handle=h))
    assert h.device_status() == 0
    olab, oR = orc.assign(X, C)
    assert float(r.item()) == oR
    if labels:
        assert np.array_equal(lab.cpu().numpy(), olab)


# the split pass over 2,048 or more centers packs its three products along
# one K range where that saves MFMAs (d <= 21 and 33..53): the part
# boundaries at d, 2d, 3d fall in every place of the 32-wide K steps; 2,032
# centers and d = 22, 54 keep three chains
@pytest.mark.parametrize("d,k", [(3, 2048), (10, 2048), (11, 2048), (21, 2048), (22, 2048),
                                 (33, 2048), (43, 2048), (53, 2048), (54, 2048), (16, 2032)])
def test_assign_packed_split(kc, orc, d, k):
    rng = np.random.default_rng(70 + d)
    X = (rng.normal(size=(6_000, d)) * 4.0 + 300.0).astype(np.float32)
    C = rng.choice(len(X), k, replace=False)
    Xd = torch.from_numpy(X).cuda()
    olab, oR = orc.assign(X, C)
    for labels in (True, False):
        h = kc.Handle()
        lab, r = on_stream(lambda: kc.assign(Xd, torch.from_numpy(C), labels=labels, handle=h))
        assert h.device_status() == 0
        assert float(r.item()) == oR
        if labels:
            assert np.array_equal(lab.cpu().numpy(), olab)


def test_mrg_fewer_centers_than_k_small_d(kc, orc):
    # 13 distinct points, repeated: fewer than k centers exist, and the
    # covering radius (direct pass, d = 2) sees the device-side center count
    base = np.random.default_rng(8).integers(0, 50, (13, 2)).astype(np.float32)
    X = np.repeat(base, 500, axis=0)[np.random.default_rng(9).permutation(6500)]
    off = W.partition_offsets(len(X), 5, 0.5, seed=9)
    k = 20
    g = gpu_mrg(kc, X, off, k)
    o = orc.mrg(X, off, k)
    assert g["n_centers"] == 13
    assert np.array_equal(g["centers"], o["centers"])
    assert g["radius"] == o["radius"] == 0.0


def test_assign_bad_center_is_reported(kc):
    h = kc.Handle()
    X = np.random.default_rng(3).random((1000, 3)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    Cd = torch.tensor([0, 5, 5000], dtype=torch.int64, device="cuda")
    on_stream(lambda: kc.assign(Xd, Cd, handle=h))
    assert h.device_status() & 4


def gpu_mrg(kc, X, off, k, bf16=False, handle=None):
    h = handle or kc.Handle()
    Xd = torch.from_numpy(X).cuda()
    B = torch.from_numpy(W.to_bf16_rne(X).view(np.int16)).cuda() if bf16 else None
    c, nc, r, ex = on_stream(lambda: kc.mrg(Xd, off, k, bf16=B, handle=h,
                                            details=True))
    assert h.device_status() == 0
    m = len(off) - 1
    nu = int(ex["n_union"].item())
    return dict(centers=c.cpu().numpy(), n_centers=int(nc.item()),
                radius=float(r.item()),
                round1=ex["round1"].cpu().numpy().reshape(m, k),
                r1=ex["r1"].cpu().numpy(),
                union=ex["union"].cpu().numpy()[:nu], r2=float(ex["r2"].item()))


def int_points(n, d, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(-100, 101, (n, d)).astype(np.float32)


# resident = False forces round 1 onto the streaming engines (FP32, or BF16
# with exact rescoring); with it the partitions are register-resident in
# either precision
@pytest.mark.parametrize("resident", [True, False])
@pytest.mark.parametrize("bf16", [False, True])
def test_mrg_integer_exact(kc, orc, bf16, resident):
    X = int_points(60_000, 16, 7)
    off = W.partition_offsets(60_000, 12, 0.5, seed=7)
    off = np.r_[off[:3], off[3], off[3:]]   # an extra empty partition
    k = 25
    g = gpu_mrg(kc, X, off, k, bf16, handle=kc.Handle(resident=resident))
    o = orc.mrg(X, off, k)
    assert np.array_equal(g["round1"], o["round1"])
    assert np.array_equal(g["r1"], o["r1"])
    assert np.array_equal(g["union"], o["union"])
    assert g["n_centers"] == o["n_centers"]
    assert np.array_equal(g["centers"], o["centers"])
    assert g["r2"] == o["r2"] and g["radius"] == o["radius"]


def test_mrg_small_partitions_and_k_above(kc, orc):
    # partitions smaller than k (all their points are centers), k > |U|
    X = int_points(3_000, 4, 9)
    off = np.r_[0, 5, 5, 17, 40, 3000]
    k = 30
    g = gpu_mrg(kc, X, off, k)
    o = orc.mrg(X, off, k)
    assert np.array_equal(g["round1"], o["round1"])
    assert np.array_equal(g["centers"], o["centers"])
    assert g["radius"] == o["radius"]


def test_mrg_union_shorter_than_round2_grid(kc, orc):
    # 15 tiny partitions and 5 large ones: the union (1,150 points) is far
    # below the capacity m*k = 4,000 that sizes round 2's resident grid, so
    # its trailing blocks own no point and must still pass every barrier
    rng = np.random.default_rng(17)
    sizes = [10] * 15 + [7_000] * 5
    n = sum(sizes)
    X = rng.integers(-80, 81, (n, 16)).astype(np.float32)
    off = np.r_[0, np.cumsum(sizes)]
    k = 200
    g = gpu_mrg(kc, X, off, k)   # checks the device status word
    o = orc.mrg(X, off, k)
    assert len(g["union"]) == len(o["union"]) == 15 * 10 + 5 * 200
    assert np.array_equal(g["centers"], o["centers"])
    assert g["radius"] == o["radius"]


# Round 1 on the resident engine packs the partitions first-fit decreasing
# into cooperative launches.  With d = 16 a block holds 2,688 points in the
# balanced variant and 4,032 in the large one.  Uncapped, all partitions
# share one launch; a cap of 3 blocks per launch spreads them over six
# (all on the large variant) or seven (balanced, plus the 11,000-point
# partition on the large one), whichever the cost model prefers; at 2 the
# 11,000-point partition fits no grid, so the round streams (20 step
# launches).
@pytest.mark.parametrize("cap,launches", [(0, (1,)), (3, (6, 7)), (2, (20,))])
def test_mrg_resident_packing(kc, orc, cap, launches):
    rng = np.random.default_rng(23)
    sizes = [0, 1, 19, 20, 21, 2688, 2689, 5000, 8064, 11000, 300, 0, 7000]
    n = sum(sizes)
    X = rng.integers(-60, 61, (n, 16)).astype(np.float32)
    off = np.r_[0, np.cumsum(sizes)]
    k = 20
    h = kc.Handle()
    h.set_option("resident_blocks", cap)
    h.set_option("timing", 1)
    g = gpu_mrg(kc, X, off, k, handle=h)
    _, la, iv = h.timing_read("mrg_round1")
    assert la in launches and iv == 1
    o = orc.mrg(X, off, k)
    assert np.array_equal(g["round1"], o["round1"])
    assert np.array_equal(g["r1"], o["r1"])
    assert np.array_equal(g["union"], o["union"])
    assert np.array_equal(g["centers"], o["centers"])
    assert g["r2"] == o["r2"] and g["radius"] == o["radius"]
    h.close()


@pytest.mark.parametrize("layout", ["wide", "odd", "shift"])
def test_mrg_row_layouts(kc, orc, rows_layout, layout):
    # strided and misaligned rows: round 1 loads the partitions straight from
    # the rows where their layout allows, else from the staging copy
    X = int_points(40_000, 16, 11)
    off = W.partition_offsets(40_000, 9, 0.5, seed=11)
    k = 18
    h = kc.Handle()
    h.set_option("timing", 1)
    Xd = rows_layout(X, layout)
    c, nc, r, ex = on_stream(lambda: kc.mrg(Xd, off, k, handle=h, details=True))
    assert h.device_status() == 0
    _, la, _ = h.timing_read("mrg_round1")
    assert la >= 1
    o = orc.mrg(X, off, k)
    m = len(off) - 1
    assert np.array_equal(ex["round1"].cpu().numpy().reshape(m, k), o["round1"])
    assert np.array_equal(ex["r1"].cpu().numpy(), o["r1"])
    assert np.array_equal(c.cpu().numpy(), o["centers"])
    assert float(r.item()) == o["radius"]
    h.close()


def check_mrg_float(orc, X, off, k, g):
    # every partition's round-1 sequence is a certified farthest-first run
    b = band(X.shape[1])
    for p in range(len(off) - 1):
        lo, hi = off[p], off[p + 1]
        if hi == lo:
            assert np.all(g["round1"][p] == -1)
            continue
        seq = g["round1"][p]
        seq = seq[seq >= 0] - lo
        bad, _, _ = orc.gon_replay(X[lo:hi], k, seq, b)
        assert bad == -1, "partition %d step %d" % (p, bad)
        _, R = orc.assign(X[lo:hi], seq)
        assert g["r1"][p] == R
    U = np.sort(g["round1"][g["round1"] >= 0])
    assert np.array_equal(U, g["union"])
    loc = np.searchsorted(U, g["centers"][:g["n_centers"]])
    bad, _, _ = orc.gon_replay(X[U], k, loc, b)
    assert bad == -1
    _, R2 = orc.assign(X[U], loc)
    assert g["r2"] == R2
    _, R = orc.assign(X, g["centers"][:g["n_centers"]])
    assert g["radius"] == R


def test_mrg_gauss_small(kc, orc):
    X, off = W.config3(200_000, 16)
    k = 40
    g = gpu_mrg(kc, X, off, k)
    check_mrg_float(orc, X, off, k, g)
    for resident in (True, False):
        gb = gpu_mrg(kc, X, off, k, bf16=True, handle=kc.Handle(resident=resident))
        assert np.array_equal(g["round1"], gb["round1"])
        assert np.array_equal(g["centers"], gb["centers"])
        assert g["radius"] == gb["radius"]


@pytest.mark.slow
def test_mrg_config3_full(kc, orc):
    orc.set_threads(16)
    X, off = W.config3()
    k = W.CONFIG3["k"]
    h = kc.Handle()
    g = gpu_mrg(kc, X, off, k, handle=h)
    check_mrg_float(orc, X, off, k, g)
    hs = kc.Handle(resident=False)
    for bf in (False, True):   # both streaming engines
        gs = gpu_mrg(kc, X, off, k, bf16=bf, handle=hs)
        assert np.array_equal(g["centers"], gs["centers"])
        assert np.array_equal(g["round1"], gs["round1"])
        assert g["radius"] == gs["radius"]
