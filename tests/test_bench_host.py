"""Host logic of the measurement script (no GPU): it refuses more than one GPU before
touching the device, and the counter summaries stay valid exactly as long as the sources
of the kernel they were taken on are unchanged."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""  # no bench line


def test_kernel_digest_follows_its_own_sources(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_1910_11110_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "common.h").write_text("// shared declarations\n")
    (csrc / "a.hip").write_text('void f() { ProfScope p(s, "kernel_a"); }\n')
    (csrc / "b.hip").write_text('void g() { ProfScope p(s, "kernel_b"); }\n')
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d_a, d_all = bench.source_digest("kernel_a"), bench.source_digest()
    (csrc / "b.hip").write_text('void g() { ProfScope p(s, "kernel_b"); /* changed */ }\n')
    assert bench.source_digest("kernel_a") == d_a  # another kernel's file changed
    assert bench.source_digest() != d_all
    (csrc / "a.hip").write_text('void f() { ProfScope p(s, "kernel_a"); /* changed */ }\n')
    d_a2 = bench.source_digest("kernel_a")
    assert d_a2 != d_a
    (csrc / "common.h").write_text("// shared declarations, changed\n")
    assert bench.source_digest("kernel_a") != d_a2  # headers count for every kernel
