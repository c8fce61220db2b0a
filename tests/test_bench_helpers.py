"""CPU checks of the measurement helpers in bench.py: the algorithmic byte count of a run and
the device-code hash that keys the committed counter summaries."""
import json

import bench


def test_algorithmic_bytes_of_the_headline():
    # 4 B per element, CSR offsets 4(R+1) B, 20 B of aggregates per region
    n, L = 1 << 26, 4096
    R = n // L
    assert bench.algorithmic_bytes(n, L) == 4 * n + 4 * (R + 1) + 20 * R == 268828676
    assert bench.algorithmic_bytes(10, 3) == 4 * 10 + 4 * 5 + 20 * 4   # a ragged last region


def test_kernel_hash_follows_device_code_only(tmp_path, monkeypatch):
    marker = "// ---------------------------------------------------------------- launch table"
    base = "int a = 1;  // first\n__device__ int f() { return a; }\n" + marker + "\nint host = 0;\n"
    variants = {
        "comment": base.replace("// first", "// reworded"),
        "spacing": base.replace("int a = 1;", "int  a=1 ;").replace("a = 1", "a=1"),
        "host": base.replace("int host = 0;", "int host = 1;"),
        "device": base.replace("return a;", "return a + 1;"),
    }
    hashes = {}
    for name, text in [("base", base)] + list(variants.items()):
        f = tmp_path / f"{name}.hip"
        f.write_text(text)
        monkeypatch.setattr(bench, "KERNEL_SOURCE", str(f))
        hashes[name] = bench.kernel_source_hash()
    assert hashes["comment"] == hashes["base"]
    assert hashes["host"] == hashes["base"]
    assert hashes["device"] != hashes["base"]


def test_measured_traffic_needs_a_matching_entry(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("__device__ int f();\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    h = bench.kernel_source_hash()
    table = tmp_path / "traffic.json"
    table.write_text(json.dumps({"entries": [
        {"kernel_source_sha256_16": h, "strategy": "tag", "ensemble_width": 256, "hbm_bytes_per_launch": 123},
        {"kernel_source_sha256_16": "0" * 16, "strategy": "signal", "ensemble_width": 256,
         "hbm_bytes_per_launch": 456}]}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(table))
    assert bench.measured_traffic("tag", 256) == 123
    assert bench.measured_traffic("tag", 128) is None
    assert bench.measured_traffic("signal", 256) is None   # taken on other device code


def test_width_argument_forms():
    assert bench.parse_widths("0") == {"tag": 0, "signal": 0, "lanes": 0, "enum_tag": 0}
    assert bench.parse_widths("256")["enum_tag"] == 256
    w = bench.parse_widths("tag:128,signal:64,enum_tag:128")
    assert w == {"tag": 128, "signal": 64, "lanes": 0, "enum_tag": 128}
    import pytest
    with pytest.raises(ValueError):
        bench.parse_widths("tags:128")


def test_more_than_one_gpu_is_refused():
    """bench.py measures one GPU: --gpus N above 1 exits with status 2 and says so, before it
    touches a GPU."""
    import os
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.abspath(bench.__file__), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
