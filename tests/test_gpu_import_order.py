"""The package works whichever of it and PyTorch a process imports first
(PyTorch's bundled ROCm runtime must be the one this library binds to; the
binding loads PyTorch before the library).  Runs in a fresh interpreter, as
a collection-time import of the package would otherwise hide the case."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = """
import paper_2602_20516_amd as lgt          # the library first
import torch
assert torch.cuda.is_available()
lat = lgt.Lattice((4, 4, 4, 4))
U = torch.zeros((4, 4, 4, 4, 4, 3, 3), dtype=torch.complex128, device="cuda")
U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
psi = torch.ones((4, 4, 4, 4, 4, 3), dtype=torch.complex128, device="cuda")
out = lat.dslash(U, psi, 0.0)              # kappa = 0: D = 1
assert torch.equal(out, psi)
print("ok")
"""


def test_package_before_torch():
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, capture_output=True, text=True, timeout=180)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-2000:]
