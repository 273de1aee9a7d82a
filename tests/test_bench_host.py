"""Host logic of bench.py (no GPU): the traffic record's source check and the CPU-baseline sample."""

import json

import bench
from workloads import normal_grid


def _kernel_file(tmp_path, body):
    p = tmp_path / "k.hip"
    p.write_text("// header\n// BEGIN KERNEL SOURCE\n" + body + "// END KERNEL SOURCE\nint host_only;\n")
    return str(p)


def test_source_sha_ignores_comments_and_blank_lines(tmp_path):
    a = _kernel_file(tmp_path, "int f(int x) {\n    return x + 1;  // one\n}\n")
    sha = bench.source_sha(a)
    b = _kernel_file(tmp_path, "int f(int x) {\n\n    return x + 1;    // another comment\n}\n")
    assert bench.source_sha(b) == sha
    c = _kernel_file(tmp_path, "int f(int x) {\n    return x + 2;\n}\n")
    assert bench.source_sha(c) != sha


def test_traffic_record_dropped_when_kernel_changes(tmp_path):
    src = _kernel_file(tmp_path, "int f(int x) { return x; }\n")
    rec = tmp_path / "traffic.json"
    rec.write_text(json.dumps({"source_sha": bench.source_sha(src), "bytes_per_launch": 123.0}))
    assert bench.load_traffic(str(rec), src) == 123.0
    _kernel_file(tmp_path, "int f(int x) { return -x; }\n")  # same path, new code
    assert bench.load_traffic(str(rec), src) is None
    assert bench.load_traffic(str(tmp_path / "missing.json"), src) is None


def test_cpu_baseline_sample():
    r = bench.cpu_baseline(normal_grid(66, 130, seed=1), T_step=10, budget_s=0.2)
    assert r["kind"] == "oracle" and r["unit"] == "GFLOP/s"
    assert r["cores"] == bench.host_cores() and r["value"] > 0
    # GFLOP/s at 4 operations and GB/s at 16 B per point and sweep describe the same sweeps
    assert abs(r["effective_GBps_at_16B"] - 4.0 * r["value"]) <= 5 * 0.0005  # both rounded to 3 decimals
    assert "sweeps in" in r["sample"] and "calls of" in r["sample"]


def test_host_cores_is_nproc():
    import os
    import subprocess

    out = subprocess.run(["nproc"], capture_output=True, text=True)
    if out.returncode == 0:
        assert bench.host_cores() == int(out.stdout.strip())
    assert 1 <= bench.host_cores() <= (os.cpu_count() or 1)


def test_traffic_record_checks_expected_keys(tmp_path):
    """A record taken at another pass size (levels) is not used for this one."""
    src = _kernel_file(tmp_path, "int f(int x) { return x; }\n")
    rec = tmp_path / "traffic.json"
    rec.write_text(json.dumps({"source_sha": bench.source_sha(src), "levels": 10, "bytes_per_launch": 7.0}))
    assert bench.load_traffic(str(rec), src, levels=10) == 7.0
    assert bench.load_traffic(str(rec), src, levels=8) is None
    assert bench.load_traffic(str(rec), src) == 7.0


def test_pressure_pass_levels_follow_the_library_split():
    """The longest pass of nit iterations at the library's default: ceil(nit / 12) passes, as even as they
    go (the first nit % passes passes take one more)."""
    for nit in range(1, 200):
        passes = -(-nit // bench.PRESSURE_MAX_LEVELS)
        base, extra = divmod(nit, passes)
        sizes = [base + (1 if k < extra else 0) for k in range(passes)]
        assert sum(sizes) == nit and max(sizes) <= bench.PRESSURE_MAX_LEVELS
        assert bench.pressure_pass_levels(nit) == max(sizes)
    assert bench.pressure_pass_levels(bench.CAVITY_NIT) == 10
