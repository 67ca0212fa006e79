"""The library opened before PyTorch is imported: one HIP runtime must serve both.  PyTorch bundles
its own copy of the runtime; the binding imports torch before it opens the library, so the
library binds to that copy instead of loading a second runtime, which would find no device."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

from tests.gpu_util import announce, torch_cuda

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, ".")
from paper_cs_0004013_amd import binding
binding.ap_set_rank_mode(0)            # the first use opens the library; torch not imported by the caller
import numpy as np
import torch
import oracle
from paper_cs_0004013_amd import inputs
keys = inputs.keyset("a", 70_001, seed=3).keys
t = torch.from_numpy(keys.view(np.int32)).to("cuda")
out = torch.empty_like(t)
binding.ap_sort_u32(t, out, 1)
torch.cuda.synchronize()
got = out.cpu().numpy().view(np.uint32)
assert np.array_equal(got, oracle.sort_u32(keys)), "mismatch"
print("load-order ok", flush=True)
"""


def test_library_opened_before_torch():
    torch_cuda()
    announce("library opened before torch (child process)")
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "load-order ok" in r.stdout, (r.stdout[-2000:], r.stderr[-2000:])
