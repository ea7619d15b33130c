"""CPU checks of the C ABI: the library loads without a GPU and exports every
function that include/kcenter.h declares (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kcenter.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", text,
                       flags=re.M)
    return sorted(set(names))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("kcenter_gonzalez", "kcenter_mrg", "kcenter_eim",
              "kcenter_assign", "kcenter_batch", "kc_create", "kc_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1604_03228_amd as kc
    L = kc.load_library()
    for n in declared_functions():
        assert hasattr(L, n), n
    assert set(declared_functions()) <= set(kc.EXPORTS)


def test_strerror_without_gpu():
    import paper_1604_03228_amd as kc
    L = kc.load_library()
    assert L.kc_strerror(0) == b"ok"
    assert L.kc_strerror(-1) == b"invalid argument"
    assert L.kc_create(None) == -1


def test_product_path_does_not_touch_oracle():
    pkg = os.path.join(ROOT, "paper_1604_03228_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                for bad in ("import oracle", "from oracle", "kc_oracle",
                            "orc_"):
                    assert bad not in src, (f, bad)
