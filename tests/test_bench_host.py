"""Host logic of bench.py (no GPU): the roofline arithmetic of the dominant
Gonzalez kernel in both of the resident engine's forms and for the
streaming engine, and the rule that a stored HBM-traffic record counts only
while the kernel's sources are unchanged."""
import json
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def resident(ms, launches, integer_form):
    return {"engine": "k_gon_resident", "kern_ms": ms * launches, "launches": launches,
            "integer_form": integer_form}


@pytest.mark.parametrize("form,opu", [(True, 11), (False, 21)])
def test_resident_roofline(form, opu):
    n, d, k = 1_000_000, 10, 1000
    kern, roof = bench.gon_roofline(n, d, k, resident(0.8, 20, form))
    assert kern == "k_gon_resident" and roof["bound"] == "alu"
    flops = n * k * 3 * d                      # sub, multiply, add per coordinate
    assert roof["achieved"] == pytest.approx(flops / 0.8e-3 / 1e12)
    assert roof["frac"] == pytest.approx(roof["achieved"] / 157.3)
    ir = roof["issue_rate"]
    assert ir["ops_per_update"] == opu         # d + 1 exact-integer, 2d + 1 canonical
    assert ir["form"] == ("exact-integer" if form else "canonical")
    assert ir["achieved"] == pytest.approx(n * k * opu / 0.8e-3 / 1e12)
    assert ir["peak"] == pytest.approx(256 * 4 * 32 * 2.4e9 / 1e12)


def test_streaming_roofline_is_hbm_bound():
    n, d, k = 1_000_000, 10, 1000
    g = {"engine": "k_gon_step", "kern_ms": 11.0, "launches": 1000}   # 11 µs each
    kern, roof = bench.gon_roofline(n, d, k, g)
    assert kern == "k_gon_step" and roof["bound"] == "hbm"
    # per launch: read d coordinates and the min-distance, write it back
    assert roof["achieved"] == pytest.approx(n * (4 * d + 8) / 11e-6 / 1e9)
    assert roof["frac"] == pytest.approx(roof["achieved"] / 8000.0)


def test_stored_traffic_needs_matching_sources(tmp_path, monkeypatch):
    srcs = ["kc_resident.hip", "kc_device.h"]
    good = bench.kernel_source_hash(srcs)
    rec = {"k_gon_resident|w": {"bytes_per_launch": 123.0, "source_hash": good},
           "k_gon_resident|stale": {"bytes_per_launch": 456.0, "source_hash": "0" * 16}}
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "PROFILE_TRAFFIC", str(p))
    assert bench.stored_traffic("k_gon_resident", "w", srcs) == 123.0
    assert bench.stored_traffic("k_gon_resident", "stale", srcs) is None
    assert bench.stored_traffic("k_gon_resident", "absent", srcs) is None
    monkeypatch.setattr(bench, "PROFILE_TRAFFIC", str(tmp_path / "missing.json"))
    assert bench.stored_traffic("k_gon_resident", "w", srcs) is None
