import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built libfgs.so")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def repo_root():
    return ROOT


@pytest.fixture(scope="session")
def rocrand_probe(tmp_path_factory):
    """The ROCm random-number library's Philox4x32-10, compiled for the host from
    tests/helpers/rocrand_philox_host.cpp: reads counter/key rows, prints output words."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("ROCm random-number library headers not available")
    exe = str(tmp_path_factory.mktemp("philox") / "rocrand_philox_host")
    src = os.path.join(ROOT, "tests", "helpers", "rocrand_philox_host.cpp")
    subprocess.run([hipcc, "-O1", "-o", exe, src], check=True, capture_output=True)
    return exe
