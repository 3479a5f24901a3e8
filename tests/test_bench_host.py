"""Host-side parts of bench.py: the one-GPU contract and the key of the
recorded traffic counters."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_kernel_hash_ignores_comments_only(tmp_path, monkeypatch):
    import bench
    src = os.path.join(ROOT, "paper_1007_4895_amd", "csrc")
    d = tmp_path / "paper_1007_4895_amd" / "csrc"
    d.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES:
        (d / f).write_text(open(os.path.join(src, f)).read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_hash()
    k = d / "lb_kernels.hpp"
    text = k.read_text()
    k.write_text("// a new comment line\n" + text.replace("\n", "  // trailing remark\n", 3) + "\n\n")
    assert bench.kernel_hash() == h0
    k.write_text(text.replace("return REG_LOW;", "return REG_HIGH;", 1))
    assert bench.kernel_hash() != h0

