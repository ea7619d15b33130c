"""GPU: option "validate" scans a call's points for non-finite coordinates
on the device and sets bit 3 of the device status word, with no host wait.
Non-finite inputs go through the assignment only (no engine here depends
on them for its control flow); finite inputs leave the word clear, and with
the option off nothing is scanned."""
import numpy as np
import pytest

from paper_1604_03228_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NONFINITE = 8


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


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
@pytest.mark.parametrize("pad", [0, 3])        # contiguous rows, and ld = d + 3
@pytest.mark.parametrize("bf16", [False, True])
def test_assign_flags_nonfinite(kc, bad, pad, bf16):
    rng = np.random.default_rng(4)
    n, d = 5000, 7
    A = rng.normal(size=(n, d + pad)).astype(np.float32)
    A[1234, 5] = bad
    X = torch.from_numpy(A).cuda()[:, :d]
    B = None
    if bf16:
        Ab = W.to_bf16_rne(np.ascontiguousarray(A)).view(np.int16)
        B = torch.from_numpy(Ab).cuda()[:, :d]
    C = torch.arange(0, 40, dtype=torch.int64)
    h = kc.Handle()
    on_stream(lambda: kc.assign(X, C, bf16=B, handle=h))
    assert h.device_status() == 0          # option off: nothing scanned
    h.set_option("validate", 1)
    on_stream(lambda: kc.assign(X, C, bf16=B, handle=h))
    assert h.device_status() & NONFINITE
    A[1234, 5] = 0.5                       # finite again: the word stays clear
    X = torch.from_numpy(A).cuda()[:, :d]
    if bf16:
        B = torch.from_numpy(W.to_bf16_rne(np.ascontiguousarray(A)).view(np.int16)).cuda()[:, :d]
    on_stream(lambda: kc.assign(X, C, bf16=B, handle=h))
    assert h.device_status() == 0


def test_finite_calls_stay_clear(kc):
    # every entry point scans when the option is on; finite points pass
    X = torch.from_numpy(W.points_gauss_mixture(30_000, 8, 10, seed=3)).cuda()
    h = kc.Handle()
    h.set_option("validate", 1)
    on_stream(lambda: kc.gonzalez(X, 20, 0, handle=h))
    on_stream(lambda: kc.mrg(X, W.partition_offsets(30_000, 4, 0.5, seed=1), 10, handle=h))
    on_stream(lambda: kc.eim(X, 5, 0.1, 4.0, 11, handle=h))
    on_stream(lambda: kc.batch([dict(X=X, algo="gon", k=7, first=3),
                                dict(X=X, algo="eim", k=4, eps=0.1, phi=4.0, seed=5)],
                               handle=h))
    assert h.device_status() == 0


def test_validate_option_range(kc):
    h = kc.Handle()
    with pytest.raises(kc.KCenterError):
        h.set_option("validate", 2)
