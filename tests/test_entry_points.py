"""Host-side contracts of the entry points (CPU only): the product path fails
loudly when its HIP library is missing, and the benchmark refuses more than one
GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_binding_raises_without_the_library(monkeypatch, tmp_path):
    from paper_0910_0329_amd import mcdose
    monkeypatch.setattr(mcdose, "LIB_PATH", str(tmp_path / "libmcdose.so"))
    monkeypatch.setattr(mcdose, "_lib", None)
    with pytest.raises(ImportError, match="libmcdose.so is missing"):
        mcdose.lib()
    with pytest.raises(ImportError):
        mcdose.Engine(0)


@pytest.mark.parametrize("n", [2, 8])
def test_bench_refuses_several_gpus(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
