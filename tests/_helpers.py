"""Shared helpers of the GPU tests (marshalling between the solver's padded
tensors and the oracle's NumPy arrays; error norms)."""
import sys

import numpy as np

# error groups: mass, momentum (three components share one scale), energy
GROUPS = ((0,), (1, 2, 3), (4,))


def grouped_rel_err(a, b, groups=GROUPS):
    """max over groups of max|a - b| / max|b| inside the group."""
    a = np.asarray(a)
    b = np.asarray(b)
    worst = 0.0
    for g in groups:
        scale = np.abs(b[list(g)]).max()
        if scale == 0.0:
            scale = 1.0
        worst = max(worst, float(np.abs(a[list(g)] - b[list(g)]).max() / scale))
    return worst


def announce(*parts):
    print("[gpu-case]", *parts, flush=True)
    sys.stdout.flush()


def to_np(t):
    return t.detach().to("cpu").numpy()


def make_solver(pb, precision="fp64", keep_metrics=False, params=None):
    from paper_2301_00817_amd.solver import Solver
    return Solver(params or pb["params"], pb["xyz"], pb.get("inflow"), precision=precision,
                  keep_metrics=keep_metrics)
