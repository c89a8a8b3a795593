"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a message and exit code 2 before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_record_key_ignores_comments_only(tmp_path):
    """The stored counter run is keyed by the pass sources with comments and
    blank space removed: a comment edit keeps the key, a code edit changes it."""
    sys.path.insert(0, ROOT)
    import bench
    src = tmp_path / "k.hpp"
    src.write_text("int f(int x) { return x + 1; }  // one\n")
    saved = list(bench.KERNEL_SOURCES)
    try:
        bench.KERNEL_SOURCES[:] = [str(src)]
        h0 = bench.kernel_hash()
        src.write_text("/* a new\n   comment */ int f(int x)   { return x + 1; }\n// two\n")
        assert bench.kernel_hash() == h0
        src.write_text("int f(int x) { return x + 2; }\n")
        assert bench.kernel_hash() != h0
    finally:
        bench.KERNEL_SOURCES[:] = saved
