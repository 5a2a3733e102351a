"""Host-side behaviour that needs no GPU: the binding refuses to run
without the built HIP library (there is no fallback path), and bench.py
refuses more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2604_12672_amd import mhd
    monkeypatch.setattr(mhd, "_lib", None)
    monkeypatch.setattr(mhd, "LIB_PATH", str(tmp_path / "libmhd.so"))
    with pytest.raises(ImportError, match="missing"):
        mhd.load()
    with pytest.raises(ImportError):
        mhd.Grid({"nx": 4, "ny": 4, "nz": 4})


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}),
                                      ([], {"WORLD_SIZE": "2"})])
def test_bench_runs_on_one_gpu_only(args, env):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args,
                       env=dict(os.environ, **env), capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
