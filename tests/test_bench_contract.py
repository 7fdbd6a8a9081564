"""Host-side pieces of the benchmark that need no GPU: the one-GPU guard and
the provenance hash of the headline kernels (comments do not change it, code
does)."""
import json
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parent.parent
sys.path.insert(0, str(ROOT))

import bench  # noqa: E402


def test_code_only_strips_comments_not_strings():
    src = 'int a = 1; // note\n/* block\n comment */ const char *s = "x // y /* z */";\nint b;'
    assert bench._code_only(src) == 'int a = 1; const char *s = "x // y /* z */"; int b;'


def test_kernel_hash_ignores_comment_edits(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("__global__ void k() { int x = 1; }\n")
    monkeypatch.setattr(bench, "ROOT", tmp_path)
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["k.hip"])
    h0 = bench.kernel_hash()
    src.write_text("// a comment\n__global__ void k() {   int x = 1; /* more */ }\n")
    assert bench.kernel_hash() == h0
    src.write_text("__global__ void k() { int x = 2; }\n")
    assert bench.kernel_hash() != h0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
