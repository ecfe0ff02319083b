"""The binding works whatever the caller imports first: torch's HIP runtime
and the library's must be one, so torch's device memory and streams are
valid in the library.  Run in a fresh interpreter (a child process), where
the binding is imported before torch."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = """
from paper_1802_02868_amd import dugks2p as D
from paper_1802_02868_amd import workloads as W
import torch
if not torch.cuda.is_available():
    print("NO_GPU")
else:
    s = D.Simulation.from_case(W.drop_case(16, radius=5.0))
    s.step(3)
    p = s.populations()
    torch.cuda.synchronize()
    print("OK", bool(torch.isfinite(p).all()))
    s.close()
"""


def test_binding_imported_before_torch():
    print("import order: binding first, then torch (child process)", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, capture_output=True, text=True,
                       timeout=180)
    if "NO_GPU" in r.stdout:
        pytest.skip("no GPU")
    assert r.returncode == 0, r.stderr[-2000:]
    assert "OK True" in r.stdout, (r.stdout, r.stderr[-2000:])
