"""GPU parity of the BF16-stream + exact FP32 rescoring Gonzalez path: its
center sequence must equal the FP32 path's exactly (both on the GPU), the
FP32 path's must pass the oracle replay, and the radius trace and exact
radius must agree."""
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


def run(kc, X, k, first, bf16, h):
    Xd = torch.from_numpy(X).cuda()
    B = torch.from_numpy(W.to_bf16_rne(X).view(np.int16)).cuda() if bf16 else None
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        c, tr, nch = kc.gonzalez(Xd, k, first, bf16=B, handle=h)
        assert h.device_status() == 0
    st.synchronize()
    return c.cpu().numpy(), tr.cpu().numpy(), int(nch.item())


# d = 70 takes the generic-d kernels and stages in two passes of columns
@pytest.mark.parametrize("d", [2, 5, 16, 41, 70])
def test_bf16_matches_fp32(kc, orc, d):
    rng = np.random.default_rng(d)
    n = 50_021
    X = (rng.normal(size=(n, d)) * rng.uniform(0.5, 20, d)).astype(np.float32)
    k = 60
    h = kc.Handle()
    c32, t32, g32 = run(kc, X, k, 3, False, h)
    cbf, tbf, gbf = run(kc, X, k, 3, True, h)
    assert g32 == gbf == k
    assert np.array_equal(c32, cbf)
    assert np.array_equal(t32, tbf)
    bad, _, _ = orc.gon_replay(X, k, c32, band(d))
    assert bad == -1


def test_bf16_integer_grid_exact(kc, orc):
    # exact ties everywhere: the rescoring must break them like the oracle
    X = W.config2(100_000)
    k = 200
    h = kc.Handle()
    cbf, tbf, gbf = run(kc, X, k, 0, True, h)
    oc, otr, og = orc.gon(X, k, 0)
    assert gbf == og and np.array_equal(cbf, oc) and np.array_equal(tbf, otr)


def test_bf16_early_stop(kc, orc):
    base = np.random.default_rng(2).normal(size=(9, 6)).astype(np.float32)
    X = np.repeat(base, 50, axis=0)
    h = kc.Handle()
    c, tr, got = run(kc, X, 20, 0, True, h)
    oc, otr, og = orc.gon(X, 20, 0)
    assert got == og == 9 and np.array_equal(c, oc) and np.array_equal(tr, otr)


@pytest.mark.slow
def test_config4_full(kc, orc):
    orc.set_threads(16)
    X, _ = W.config4()
    k = W.CONFIG4["k"]
    h = kc.Handle()
    c32, t32, _ = run(kc, X, k, 0, False, h)
    cbf, tbf, _ = run(kc, X, k, 0, True, h)
    assert np.array_equal(c32, cbf) and np.array_equal(t32, tbf)
    bad, _, otr = orc.gon_replay(X, k, c32, band(41))
    assert bad == -1
    olab, R = orc.assign(X, c32)
    assert t32[-1] == R
    assert abs(t32[-1] - otr[-1]) <= 1e-6 * otr[-1]
    # the n x k assignment of the objective (Section 1.1) at full shape:
    # BF16 MFMA distances with certified labels, FP64 rescoring of the rest;
    # labels equal the oracle's and the radius is the exact FP64 one
    Xd = torch.from_numpy(X).cuda()
    B = torch.from_numpy(W.to_bf16_rne(X).view(np.int16)).cuda()
    cd = torch.from_numpy(c32).cuda()
    for bf in (B, None):
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            lab, rad = kc.assign(Xd, cd, bf16=bf, handle=h)
            assert h.device_status() == 0
        st.synchronize()
        assert np.array_equal(lab.cpu().numpy(), olab)
        assert float(rad.item()) == R
