import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import build
    if not os.path.exists(build.LIB):
        build.build()
    yield


@pytest.fixture(scope="session")
def kernels_asm(tmp_path_factory):
    """gfx950 assembly of mhd_kernels.hip compiled with the library build's
    flags (lines); skips where hipcc is missing."""
    from paper_2604_12672_amd import build
    if shutil.which(build.HIPCC) is None and not os.path.exists(build.HIPCC):
        pytest.skip("hipcc not available")
    csrc = os.path.join(os.path.dirname(build.__file__), "csrc")
    flags = [f for f in build.FLAGS if f not in ("-shared", "-fPIC")]
    out = tmp_path_factory.mktemp("asm") / "kernels.s"
    subprocess.run([build.HIPCC] + flags + ["-I", csrc, "--cuda-device-only", "-S",
                    os.path.join(csrc, "mhd_kernels.hip"), "-o", str(out)],
                   check=True, capture_output=True)
    return out.read_text().split("\n")
