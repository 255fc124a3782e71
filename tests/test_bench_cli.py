"""bench.py's host side (CPU only): it refuses more than one GPU with a
message, and its CPU baseline times the oracle and reports the threads used."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_cpu_baseline_reports_the_oracle_and_its_threads():
    sys.path.insert(0, ROOT)
    import bench
    import oracle.orc as orc
    out = bench.cpu_baseline(16, target_s=0.2, single_s=0.1)
    assert out["kind"] == "oracle" and out["unit"] == "MLUPS" and out["value"] > 0
    assert out["cores"] == orc.threads()
    assert out["single_thread"]["cores"] == 1 and out["single_thread"]["value"] > 0
    assert "z-slab" in out["sample"]
    assert orc.threads() == out["cores"]  # thread count restored after the one-thread sample


def test_kernel_hash_ignores_comments():
    """A comment edit is not a kernel change: the traffic record keyed by the
    code hash stays valid; a code edit is a change."""
    import bench
    a = "int f(int x) { // one\n  return x + 1; /* two\n lines */ }\n"
    b = "int f(int x) {\n  // another comment\n  return x + 1;  }"
    c = "int f(int x) { return x + 2; }"
    assert bench._code_of(a) == bench._code_of(b) == "int f(int x) { return x + 1; }"
    assert bench._code_of(c) != bench._code_of(a)
    files = {"fused.hip": a, "device.h": "// h\n", "common.h": ""}
    h1 = bench.kernel_source_hash(files.__getitem__)
    files["fused.hip"] = b
    assert bench.kernel_source_hash(files.__getitem__) == h1
    files["fused.hip"] = c
    assert bench.kernel_source_hash(files.__getitem__) != h1
