"""Host-side logic of bench.py: the roofline of the two-iteration CG from
the library's profile counters, and the gating of committed HBM counter
figures on the kernel source hash and the launch shape."""
import json

import pytest

import bench

G = 256 ** 3


def prof(n, total_ms, update_ms, key="fp32"):
    return {f"{key}_sweep": (n, total_ms), f"{key}_update_ms": update_ms}


def test_sstep_roofline_splits_basis_and_update():
    r = bench.roofline("fp32_sweep", prof(10, 1.5, 0.9), G, "fp32",
                       {"ppt": 4, "cx": 22, "nwg": 768,
                        "basis": {"threads": 1024, "ppt": 4, "cx": 16, "nwg": 256}}, sstep=True)
    assert r["kernel"].startswith("k_sstep update")
    assert r["basis_kernel"]["launch_shape"]["grid_threads"] == 256 * 1024
    assert r["avg_launch_us"] == pytest.approx(90.0)
    assert r["achieved"] == pytest.approx(24 * G / 90e-6 / 1e9, rel=1e-3)
    b = r["basis_kernel"]
    assert b["avg_launch_us"] == pytest.approx(60.0)
    assert b["algorithmic_bytes_per_launch"] == 8 * G
    assert r["outer_step_us"] == pytest.approx(150.0)
    assert r["launch_shape"]["grid_threads"] == 768 * 256


def test_sstep_roofline_512_thread_update_shape():
    r = bench.roofline("fp32_sweep", prof(10, 1.5, 0.9), G, "fp32",
                       {"ppt": 4, "cx": 32, "nwg": 256, "segment": 2048,
                        "basis": {"threads": 1024, "ppt": 4, "cx": 16, "nwg": 256}}, sstep=True)
    assert r["launch_shape"]["threads"] == 512
    assert r["launch_shape"]["grid_threads"] == 256 * 512


def test_sweep_roofline_unchanged():
    r = bench.roofline("fp64_sweep", {"fp64_sweep": (4, 0.8)}, G, "fp64")
    assert r["avg_launch_us"] == pytest.approx(200.0)
    assert r["algorithmic_bytes_per_launch"] == 48 * G
    assert "basis_kernel" not in r


def test_traffic_needs_matching_source_and_shape(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source")
    t = {"stencil_sha": bench.source_hash(str(src)),
         "fp32_update": {"hbm_bytes_per_launch": 111, "launch_shape": {"ppt": 4, "cx": 22}},
         "fp32_basis": {"hbm_bytes_per_launch": 22,
                        "launch_shape": {"threads": 1024, "ppt": 4, "cx": 16}}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(t))
    monkeypatch.setitem(bench.TRAFFIC, "sstep", (str(f), str(src)))

    def fresh(cx, basis_threads=1024, layout=0):
        r = bench.roofline("fp32_sweep", prof(10, 1.5, 0.9), G, "fp32",
                           {"ppt": 4, "cx": cx, "nwg": 768,
                            "basis": {"threads": basis_threads, "ppt": 4, "cx": 16, "nwg": 256,
                                      "layout": layout}},
                           sstep=True)
        bench.attach_traffic(r, "fp32", "sstep")
        return r

    r = fresh(22)
    assert r["traffic"] == 111 and r["basis_kernel"]["traffic"] == 22
    r = fresh(32)  # another update shape: not the one the counters saw
    assert r["traffic"] is None and r["basis_kernel"]["traffic"] == 22
    r = fresh(22, basis_threads=256)  # another basis shape
    assert r["traffic"] == 111 and r["basis_kernel"]["traffic"] is None
    r = fresh(22, layout=16)  # the same numbers in the wavefront-row layout
    assert r["traffic"] == 111 and r["basis_kernel"]["traffic"] is None
    assert r["basis_kernel"]["launch_shape"]["layout"] == 16
    src.write_text("changed kernel source")  # counters taken with other code
    r = fresh(22)
    assert r["traffic"] is None and r["basis_kernel"]["traffic"] is None


def test_committed_traffic_files_name_their_source():
    for form, (path, src) in bench.TRAFFIC.items():
        t = json.load(open(path))
        assert t["source"].endswith(src.split("/")[-1]), form
        assert t["fetch_scale"] > 0 and t["write_scale"] > 0
