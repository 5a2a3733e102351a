"""Host-side behaviour that needs no GPU: the binding refuses to run
without the built HIP library (there is no fallback path), bench.py
refuses more than one GPU, prices the roofline on the algorithmic bytes,
and keys its counter tables by the kernels' code, not their comments."""
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


def test_algorithmic_bytes_of_the_roofline():
    """The per-zone byte counts behind bench.py's rooflines, counted array
    by array: a state is 5 cell + 3 face doubles (64 B); stage 1 of an
    SSP-RK scheme reads U^n and writes U^(1), every later stage reads U^n and
    U^(s) and writes one state; the previous-T guess reads and writes T; the
    learned guess stores no temperature (320 B per SSP-RK2 step, as without the gas+radiation EOS),
    so the guess array it reads is the kernel's extra traffic, reported
    apart and not priced as work; forcing modes add no per-zone array."""
    import types

    import bench
    state = 64.0

    def w(rk, T=False, force=False):
        return types.SimpleNamespace(params={"rk_order": rk}, T=object() if T else None,
                                     fmodes=object() if force else None)

    rk2 = ((state + state) + (2 * state + state)) / 2
    rk3 = ((state + state) + 2 * (2 * state + state)) / 3
    assert bench.stage_bytes(w(2), False) == rk2 == 160.0
    assert bench.stage_bytes(w(3), False) == pytest.approx(rk3)
    assert bench.stage_bytes(w(2, T=True), False) == rk2 + 16.0
    assert bench.stage_bytes(w(2, T=True), True) == rk2
    assert bench.stage_bytes(w(2, force=True), False) == rk2
    assert bench.extra_bytes(w(2, T=True), True) == 8.0
    assert bench.extra_bytes(w(2, T=True, force=True), True) == 8.0
    assert bench.extra_bytes(w(2, T=True), False) == 0.0
    # species (SSP-RK3): read rho X^(s), rho, 3 face mass fluxes and, in two
    # of three stages, rho X^n; write rho X
    ns = 12
    assert bench.species_bytes(ns) == pytest.approx(8 * ns + 8 + 24 + (2 / 3) * 8 * ns + 8 * ns)
    assert bench.species_bytes(ns) == pytest.approx(288.0)
    # RKL2 stage: 7 doubles read, 3 (internal-energy form) or 2 (T form) written
    assert bench.BYTES_RKL2_STAGE == {0: 7 * 8.0 + 3 * 8.0, 1: 7 * 8.0 + 2 * 8.0}


def test_kernel_digest_follows_code_not_comments():
    """The counter tables are keyed by a digest of the kernels' code text:
    a comment or blank-space edit keeps it, any code edit changes it, and a
    comment marker inside a literal is code."""
    import bench
    src = 'x = a / b;  // ratio\n/* block */ y = "a // b";\nz = \'/\';\n'
    assert bench.code_text(src) == 'x = a / b; y = "a // b"; z = \'/\';'
    assert bench.code_text(src) == bench.code_text(src.replace("ratio", "quotient").replace("  ", " "))
    assert bench.code_text(src) != bench.code_text(src.replace("a / b", "a * b"))
    assert bench.code_text(src) != bench.code_text(src.replace('"a // b"', '"a / b"'))
    assert len(bench.kernel_digest()) == 16
