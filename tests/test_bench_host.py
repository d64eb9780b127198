"""Host-side logic of bench.py that needs no GPU.

* The measured HBM traffic is reported only from a profiler record whose
  kernel, workload, precision and library-source hash all match; a record
  taken on other sources gives null.
* The roofline names the kernel class with the largest estimated total time
  (timed launches scaled to all launches of the class), prices a contraction
  against the MFMA peak of its precision, a bandwidth-bound class against HBM,
  and the ID class against the FP64 vector peak, and reports per-launch time.
"""
import json

import pytest

import bench


def _write_record(d, name, **rec):
    (d / name).write_text("# summary\n\n* record: " + json.dumps(rec) + "\n")


def test_traffic_record_is_keyed_by_the_library_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.measured_traffic("butterfly_gemm", "helmholtz128grf", "c128") is None
    sha = bench.library_sources_sha256()
    _write_record(tmp_path, "a.md", kernel="butterfly_gemm", config="helmholtz128grf", precision="c128",
                  traffic_bytes_per_launch=123, sources_sha256="0" * 64)
    assert bench.measured_traffic("butterfly_gemm", "helmholtz128grf", "c128") is None
    _write_record(tmp_path, "b.md", kernel="butterfly_gemm", config="helmholtz128grf", precision="c128",
                  traffic_bytes_per_launch=456, sources_sha256=sha)
    assert bench.measured_traffic("butterfly_gemm", "helmholtz128grf", "c128") == 456
    assert bench.measured_traffic("butterfly_gemm", "helmholtz128grf", "c64") is None
    assert bench.measured_traffic("butterfly_gemm", "helmholtz100", "c128") is None
    assert bench.measured_traffic("schur_gemm", "helmholtz128grf", "c128") is None
    (tmp_path / "notes.txt").write_text("* record: not json and not read\n")
    assert bench.measured_traffic("butterfly_gemm", "helmholtz128grf", "c128") == 456


def test_sources_hash_is_stable_and_sees_every_source(tmp_path, monkeypatch):
    h = bench.library_sources_sha256()
    assert h == bench.library_sources_sha256() and len(h) == 64
    src = tmp_path / "paper_2007_00202_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "k.hip").write_text("a")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h1 = bench.library_sources_sha256()
    (src / "notes.md").write_text("not a source")
    assert bench.library_sources_sha256() == h1
    (src / "k.hip").write_text("b")
    assert bench.library_sources_sha256() != h1


def _classes(**dominant):
    ks = {k: {"seconds": 0.01, "launches": 1, "launches_all": 1, "flops": 1e9, "bytes": 1e6}
          for k in ("assemble", "schur_gemm", "butterfly_gemm", "interp_decomp", "entry_extract", "spmv")}
    for k, v in dominant.items():
        ks[k] = v
    return ks


def test_roofline_scales_sampled_classes_before_choosing(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    # 10 of 80 launches timed (1 s): 8 s estimated, more than the fully timed 5 s class
    ks = _classes(butterfly_gemm={"seconds": 1.0, "launches": 10, "launches_all": 80, "flops": 40e12, "bytes": 1e9},
                  schur_gemm={"seconds": 5.0, "launches": 5, "launches_all": 5, "flops": 400e12, "bytes": 1e9})
    rf, kernels = bench.roofline(ks, 2, "c128", "helmholtz128grf")
    assert rf["kernel"] == "butterfly_gemm" and rf["bound"] == "mfma" and rf["unit"] == "TFLOP/s"
    assert rf["achieved"] == pytest.approx(40.0) and rf["peak"] == 78.6
    assert rf["frac"] == pytest.approx(40.0 / 78.6)
    assert rf["avg_launch_ms"] == pytest.approx(100.0)
    assert rf["timed_launches"] == 10 and rf["launches"] == 80 and rf["traffic"] is None
    assert kernels["butterfly_gemm"]["ms"] == pytest.approx(4000.0)  # 8 s over 2 steps
    assert kernels["butterfly_gemm"]["launches"] == 40 and kernels["butterfly_gemm"]["timed_launches"] == 5
    assert kernels["schur_gemm"]["tflops"] == pytest.approx(80.0)
    # the complex64 form prices the same contraction against the FP32 MFMA peak
    rf64, _ = bench.roofline(ks, 2, "c64", "helmholtz128grf")
    assert rf64["peak"] == 157.3 and rf64["frac"] == pytest.approx(40.0 / 157.3)


def test_roofline_bandwidth_and_id_classes(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    ks = _classes(assemble={"seconds": 2.0, "launches": 4, "launches_all": 4, "flops": 0.0, "bytes": 8e12})
    rf, _ = bench.roofline(ks, 1, "c128", "helmholtz128grf")
    assert rf["kernel"] == "assemble" and rf["bound"] == "hbm" and rf["unit"] == "GB/s"
    assert rf["achieved"] == pytest.approx(4000.0) and rf["peak"] == 8000.0 and rf["frac"] == pytest.approx(0.5)
    ks = _classes(interp_decomp={"seconds": 3.0, "launches": 3, "launches_all": 3, "flops": 3e12, "bytes": 1e9})
    rf, _ = bench.roofline(ks, 1, "c64", "helmholtz128grf")
    assert rf["kernel"] == "interp_decomp" and rf["bound"] == "alu"
    assert rf["peak"] == 78.6 and rf["achieved"] == pytest.approx(1.0)  # IDs run in FP64 in either form
