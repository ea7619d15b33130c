"""GPU parity of kcenter_eim against the FP64 oracle.

Every draw (Philox4x64-10) and every keep/remove decision is certified, so
the sample C = S u R and the per-iteration records (sizes, probabilities,
the threshold tau) must equal the oracle's exactly.  The final Gonzalez on
the sample is replayed through the oracle (certified ties only) and the
radius is the exact FP64 covering radius of the GPU's centers."""
import numpy as np
import pytest

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


def gpu_eim(kc, X, k, eps, phi, seed, max_iters=64, split=True, force=-1):
    h = kc.Handle()
    h.set_option("mfma_split", int(split))
    h.set_option("tune_force", force)
    Xd = torch.from_numpy(X).cuda()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        c, nc, r, smp, its = kc.eim(Xd, k, eps, phi, seed, max_iters, handle=h)
        assert h.device_status() == 0
    st.synchronize()
    return dict(centers=c.cpu().numpy(), n_centers=int(nc.item()),
                radius=float(r.item()), sample=smp.cpu().numpy(), iters=its,
                exact=h.counter("eim_exact"), refined=h.counter("eim_refined"))


def check(orc, X, k, eps, phi, seed, g):
    o = orc.eim(X, k, eps, phi, seed)
    assert np.array_equal(g["sample"], o["sample"])
    assert len(g["iters"]) == len(o["iters"])
    for a, b in zip(g["iters"], o["iters"]):
        for key in ("r_size", "ds_size", "h_size", "s_size"):
            assert a[key] == b[key], key
        assert a["p_s"] == b["p_s"] and a["p_h"] == b["p_h"]
        assert a["tau"] == b["tau"]
    C = o["sample"]
    got = g["n_centers"]
    loc = np.searchsorted(C, g["centers"][:got])
    assert np.array_equal(C[loc], g["centers"][:got])
    bad, ties, _ = orc.gon_replay(X[C], k, loc, band(X.shape[1]))
    assert bad == -1
    _, R = orc.assign(X, g["centers"][:got])
    assert g["radius"] == R
    if ties == 0:
        assert np.array_equal(g["centers"], o["centers"])
        assert g["radius"] == o["radius"]
    return o


def test_no_sampling_is_gon(kc, orc):
    X = np.random.default_rng(41).normal(size=(1000, 3)).astype(np.float32)
    g = gpu_eim(kc, X, 10, 0.1, 8.0, 1)
    o = check(orc, X, 10, 0.1, 8.0, 1, g)
    assert g["iters"] == [] and len(g["sample"]) == 1000


def test_one_iteration(kc, orc):
    X = np.random.default_rng(42).normal(size=(20000, 2)).astype(np.float32)
    g = gpu_eim(kc, X, 2, 0.1, 1.0, 1234)
    check(orc, X, 2, 0.1, 1.0, 1234, g)
    assert len(g["iters"]) == 1


@pytest.mark.parametrize("phi", [1.0, 4.0, 6.0, 8.0])
def test_iterations_gauss(kc, orc, phi):
    rng = np.random.default_rng(int(phi))
    X = (rng.normal(size=(60000, 3)) * 10).astype(np.float32)
    g = gpu_eim(kc, X, 3, 0.1, phi, 7 + int(phi))
    check(orc, X, 3, 0.1, phi, 7 + int(phi), g)
    assert len(g["iters"]) >= 1


def test_all_duplicates(kc, orc):
    X = np.ones((10000, 2), np.float32)
    g = gpu_eim(kc, X, 1, 0.5, 1.0, 3)
    check(orc, X, 1, 0.5, 1.0, 3, g)
    assert len(g["iters"]) == 1 and g["radius"] == 0.0


# d <= 8 runs the distance pass in canonical FP32 (tight relative bounds);
# above, on MFMA, whose bounds scale with the norms, so the unbalanced blobs
# leave many candidates whose interval contains tau and the exact FP64 pass
# decides them: tiled for d <= 64, one block per candidate above (d = 70).
@pytest.mark.parametrize("d,split", [(2, True), (8, True), (32, True), (32, False),
                                     (70, True)])
def test_unbalanced_blobs(kc, orc, d, split):
    from paper_1604_03228_amd import workloads as W
    X = W.points_gauss_mixture(100_000, d, 25, seed=77, heavy=0.9)
    g = gpu_eim(kc, X, 20, 0.1, 4.0, 5 * 2**32 + 1, split=split)
    check(orc, X, 20, 0.1, 4.0, 5 * 2**32 + 1, g)
    if d > 8:
        assert g["exact"] + g["refined"] > 0


# Every variant of the distance pass (tune_force): 0 the direct canonical
# FP32 pass (d <= 8; elsewhere the first feasible variant), 1 the FP32 MFMA,
# 2-5 the split MFMA with 4 / 8 waves per block and 64 KiB of staged
# samples, then 8 / 4 waves with 32 KiB; the MFMA variants' undecided
# candidates go through the canonical FP32 refinement, then FP64.
# Samples, records and the final Gonzalez equal the oracle's in every one.
@pytest.mark.parametrize("d", [2, 8, 32])
@pytest.mark.parametrize("var", [0, 1, 2, 3, 4, 5])
def test_forced_variants(kc, orc, d, var):
    from paper_1604_03228_amd import workloads as W
    X = W.points_gauss_mixture(60_000, d, 25, seed=91 + d, heavy=0.9)
    g = gpu_eim(kc, X, 12, 0.1, 4.0, 3 * 2**32 + d, force=var)
    check(orc, X, 12, 0.1, 4.0, 3 * 2**32 + d, g)
    assert len(g["iters"]) >= 1


def test_max_iters_reports_noconv(kc):
    X = np.random.default_rng(5).normal(size=(60000, 3)).astype(np.float32)
    with pytest.raises(kc.KCenterError) as e:
        gpu_eim(kc, X, 3, 0.1, 8.0, 9, max_iters=1)
    assert e.value.status == -4


# The parameter-study shape (Gaussian data, n = 200,000, d = 2, 25 clusters
# of sigma 0.1 in [0, 100]^2, eps = 0.1): samples, iterations and centers
# equal the oracle's at the extremes of phi and k.
@pytest.mark.parametrize("k,phi", [(2, 1.0), (25, 8.0)])
def test_study_shape(kc, orc, k, phi):
    from paper_1604_03228_amd import workloads as W
    X = W.points_gauss_mixture(200_000, 2, 25, 0.0, 100.0, 0.1, 0.1, seed=600)
    g = gpu_eim(kc, X, k, 0.1, phi, 7 * 2**32)
    check(orc, X, k, 0.1, phi, 7 * 2**32, g)
    assert len(g["iters"]) >= 1
