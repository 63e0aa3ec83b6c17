"""Host-side helpers of bench.py: the code-only source hash that keys the committed
traffic counters, the counters lookup, and the one-GPU guard (no GPU needed)."""
import os
import shutil
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_code_only_drops_comments_and_whitespace():
    src = 'int a = 1; // note\n/* block\n comment */ const char* s = "x // y";\n'
    assert bench._code_only(src) == 'inta=1;constchar*s="x // y";'
    assert bench._code_only("a/*x*/b") == bench._code_only("a b") == "ab"


def _tree(tmp_path, sha, traffic="123456"):
    for rel in bench.KERNEL_SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, rel), dst)
    (tmp_path / "profiles").mkdir(exist_ok=True)
    (tmp_path / "profiles" / "classify_w_counters.md").write_text(
        f"# t\n\n- kernel_source_sha256: `{sha}`\n- traffic_bytes_per_launch: `{traffic}`\n")


def test_committed_traffic_only_for_the_current_code(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _tree(tmp_path, "0" * 64)
    assert bench.committed_traffic("classify", "w") is None     # taken on other code
    _tree(tmp_path, bench.kernel_source_hash())
    assert bench.committed_traffic("classify", "w") == 123456.0
    # a comment edit keeps the counters valid; a code edit does not
    src = tmp_path / bench.KERNEL_SOURCES[0]
    src.write_text(src.read_text() + "\n// trailing note\n")
    assert bench.committed_traffic("classify", "w") == 123456.0
    src.write_text(src.read_text() + "\nstatic int rmx_unused_ = 0;\n")
    assert bench.committed_traffic("classify", "w") is None
    assert bench.committed_traffic("classify", "absent") is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
