"""The native command-line driver (paper_1402_4247_amd/kgev_driver) solves
synthetic pencils through the C ABI without Python: every call and every
k-point's status must be OK."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_driver_solves_through_the_c_abi():
    drv = os.path.join(ROOT, "paper_1402_4247_amd", "kgev_driver")
    r = subprocess.run([drv, "--n", "300", "--nk", "3", "--steps", "2", "--warmup", "1"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count(": ") >= 3 and "FAILED" not in r.stdout and "solves/s" in r.stdout
