"""Shared helpers of the GPU tests: move seeded inputs to the device, run the oracle beside."""
import sys

import numpy as np
import pytest
import torch

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs an MI355X")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to("cuda", dtype)


def host(t):
    return t.detach().to("cpu", torch.float64).numpy()


def plan_for(mesh, precision="fp64", **opts):
    from paper_1808_04099_amd import Mesh, Plan
    return Plan(Mesh(mesh), precision=precision, **opts)


def rel_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
