"""Host logic of bench.py (no GPU): the roofline figures it derives from
kernel times, the ceiling from the measured issue rates, and the lookup of
the committed HBM-traffic counters, which must go stale when the pair-kernel
code changes but not when only its comments do."""
import os
import shutil

import pytest

import bench


def test_roofline_fraction_from_kernel_times():
    n = 4096
    kt = {"fwd_us": 11.0, "adj_us": 19.0}
    r = bench.roofline(n, kt, traffic=123.0, precision="fp32c")
    assert r["kernel"] == "adj_pair" and r["bound"] == "alu" and r["traffic"] == 123.0
    achieved = 62 * n * n / 19.0e-6 / 1e12
    assert r["achieved"] == pytest.approx(achieved, abs=1e-3)
    assert r["frac"] == pytest.approx(achieved / 157.3, abs=1e-4)
    # 38 VALU instructions per adjoint pair against 78.65e12 lane-instructions/s
    assert r["valu_issue_frac"] == pytest.approx(38 * n * n / 19.0e-6 / 78.65e12, abs=1e-4)
    # FP64 against the FP64 peak
    r64 = bench.roofline(n, kt, precision="fp64")
    assert r64["peak"] == 78.6 and r64["frac"] == pytest.approx(achieved / 78.6, abs=1e-4)


def test_issue_ceiling(monkeypatch):
    monkeypatch.setattr(bench, "CEILINGS", {})
    assert bench.issue_ceiling(1e12, "fp32c") is None          # probes did not run
    v, e = 64e12, 18e12
    monkeypatch.setattr(bench, "CEILINGS", {"fp32_fma_vgpr_per_s": v, "exp_f32_per_s": e})
    c = bench.issue_ceiling(1.5e12, "fp32c")
    # one forward pair (16 VALU + exp) and one adjoint pair (37 VALU + exp)
    ceiling = 2 / (16 / v + 1 / e + 37 / v + 1 / e)
    assert c["pairs_per_s"] == pytest.approx(ceiling, rel=1e-9)
    assert c["frac"] == pytest.approx(1.5e12 / ceiling, abs=1e-4)
    assert c["valu_per_pair"] == {"fwd": 16, "adj": 37}
    assert bench.issue_ceiling(1e12, "fp64") is None           # FP64 computes its own 2^x


def _fake_root(tmp_path, kernel_text, traffic_text):
    csrc = tmp_path / "paper_1907_04839_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "shoot_kernels.hip").write_text(kernel_text)
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_adj_pair_w.txt").write_text(traffic_text)
    return str(tmp_path)


def test_traffic_counters_go_stale_with_the_code_not_the_comments(tmp_path, monkeypatch):
    code = "// pair kernels\nint f(int x) { return x + 1; } /* block */\n"
    monkeypatch.setattr(bench, "ROOT", _fake_root(tmp_path, code, ""))
    h = bench.kernel_source_hash()
    summary = ("# traffic\n\nMachine-readable:\nworkload = w\nprecision = fp32c\n"
               f"kernel_source_sha256_16 = {h}\nhbm_bytes_per_launch = 4524961\n")
    (tmp_path / "profiles" / "traffic_adj_pair_w.txt").write_text(summary)
    assert bench.measured_traffic("w", "fp32c") == 4524961.0
    assert bench.measured_traffic("w", "fp64") is None         # other precision
    assert bench.measured_traffic("other", "fp32c") is None    # no summary
    src = tmp_path / "paper_1907_04839_amd" / "csrc" / "shoot_kernels.hip"
    # a comment edit keeps the counters
    src.write_text("// the pair kernels, reworded\nint f(int x) {  return x + 1; }\n")
    assert bench.kernel_source_hash() == h
    assert bench.measured_traffic("w", "fp32c") == 4524961.0
    # a code edit makes them stale
    src.write_text(code.replace("x + 1", "x + 2"))
    assert bench.kernel_source_hash() != h
    assert bench.measured_traffic("w", "fp32c") is None


def test_committed_traffic_summaries_are_machine_readable(tmp_path, monkeypatch):
    # the committed summaries parse (their hash may lag a kernel edit: then
    # bench.py reports traffic null, which this test does not forbid)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for name in ("blobs65536", "ellipsoid4096"):
        path = os.path.join(root, "profiles", f"traffic_adj_pair_{name}.txt")
        vals = {}
        with open(path) as f:
            for line in f:
                if "=" in line and not line.startswith(" "):
                    k, v = line.split("=", 1)
                    vals[k.strip()] = v.strip()
        assert vals["workload"] == name and vals["precision"] == "fp32c"
        assert len(vals["kernel_source_sha256_16"]) == 16
        assert float(vals["hbm_bytes_per_launch"]) > 0
        # and bench.py reads the same value when the hash is current
        fake = tmp_path / name
        csrc = fake / "paper_1907_04839_amd" / "csrc"
        csrc.mkdir(parents=True)
        shutil.copy(os.path.join(root, "paper_1907_04839_amd", "csrc", "shoot_kernels.hip"),
                    csrc / "shoot_kernels.hip")
        (fake / "profiles").mkdir()
        monkeypatch.setattr(bench, "ROOT", str(fake))
        text = open(path).read().replace(vals["kernel_source_sha256_16"],
                                         bench.kernel_source_hash())
        (fake / "profiles" / f"traffic_adj_pair_{name}.txt").write_text(text)
        assert bench.measured_traffic(name, "fp32c") == float(vals["hbm_bytes_per_launch"])
