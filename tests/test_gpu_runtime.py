"""One HIP runtime per process: opening the library before anything has
touched PyTorch (here through a host-only call, lbm_lattice) must still give
a working solver. PyTorch carries its own libamdhip64 under the same soname
as the system's; before the bindings loaded PyTorch's runtime first, this
order brought in both runtimes and lbm_init failed with LBM_EDEVICE. Runs in
a fresh process, since the order of the first loads is what matters."""
import os
import subprocess
import sys

import pytest

from gpu_common import say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
from paper_2407_12263_amd import lbm, inputs
lbm.lbm_lattice()                       # the library is opened here, before PyTorch
w = inputs.static_droplet(n=16, R=4.0, sigma=2e-3)
sol = lbm.Solver(dict(w.params(), precision="fp32"), w.phi0, w.u0, w.p0)
sol.step(10)
d = sol.diagnostics()
assert abs(d["sum_phi"] - w.phi0.sum()) < 1e-6 * w.phi0.sum(), d["sum_phi"]
print("CHILD_OK", flush=True)
"""


def test_library_opened_before_pytorch_still_runs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("[runtime] fresh process: lbm_lattice before PyTorch, then a solver")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], capture_output=True, text=True,
                       timeout=240)
    say(r.stdout[-500:] + r.stderr[-1500:])
    assert r.returncode == 0 and "CHILD_OK" in r.stdout
