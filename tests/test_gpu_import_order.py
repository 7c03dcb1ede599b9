"""The package finds the GPU whether it is imported before or after PyTorch
(both must run on one HIP runtime; the binding loads PyTorch's first)."""
import os
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = """
import numpy as np
import paper_1711_01783_amd as met
import torch
from met_inputs import PROFILES
code = met.Code.build(PROFILES["r0.1"], 4096, 3)
bits = torch.zeros((2, 4096), dtype=torch.uint8, device="cuda:0")
syn = met.syndrome(code, bits)
torch.cuda.synchronize()
assert int(syn.cpu().numpy().astype(np.int64).sum()) == 0
print("ok", flush=True)
"""


def test_package_imported_before_torch_finds_the_device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("fresh process: package imported before torch", flush=True)
    r = subprocess.run([sys.executable, "-c", PROBE], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.strip().endswith("ok")
