"""The library and PyTorch in one process share one HIP runtime, whichever is used first:
a fresh process steps a controller through the library, then starts torch's GPU context and
allocates on the device."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu


def test_library_first_then_torch():
    code = ("import numpy as np\n"
            "import paper_1509_01149_amd as P\n"
            "import workloads as W\n"
            "wl = W.cartpole(K=257, T=7)\n"
            "with P.controller_for(wl) as c:\n"
            "    u = c.step(wl.x0)\n"
            "assert np.all(np.isfinite(u))\n"
            "import torch\n"
            "assert torch.cuda.is_available()\n"
            "x = torch.ones(4, device='cuda:0')\n"
            "print('sum', float(x.sum()))\n")
    res = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-2000:]
    assert "sum 4.0" in res.stdout
