import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size case")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


def _rows_layout(X, layout):
    """X (n x d, FP32) on the GPU as rows of a wider array ("wide": ld = d+4,
    "odd": ld = d+1) or starting one float past an aligned address ("shift");
    "dense" is a plain copy.  The resident engine loads points straight from
    rows whose stride and base suit its vector loads, else from a staging
    copy, so these layouts reach both paths."""
    import torch
    n, d = X.shape
    if layout == "dense":
        return torch.from_numpy(X).cuda()
    if layout in ("wide", "odd"):
        ld = d + 4 if layout == "wide" else d + 1
        B = torch.full((n, ld), float("nan"), dtype=torch.float32)
        B[:, :d] = torch.from_numpy(X)
        return B.cuda()[:, :d]
    assert layout == "shift"
    flat = torch.full((n * d + 1,), float("nan"), dtype=torch.float32)
    flat[1:] = torch.from_numpy(X).reshape(-1)
    return flat.cuda()[1:].view(n, d)


@pytest.fixture(scope="session")
def rows_layout():
    return _rows_layout
