"""The library driven from plain C: tests/c_client.c (C99, HIP runtime for
device memory, no Python) sets up the jet from its 1-D maps, sets the
entrance data and takes RK5 steps through the C-ABI; the same inputs
through the Python binding give bitwise the same time steps and state
(one library, deterministic kernels), in both precision forms."""
import os
import subprocess

import numpy as np
import pytest
import torch

from _helpers import announce
from cases import flow, problems

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2301_00817_amd", "_lib", "c_client")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c_client_matches_the_python_binding(precision, tmp_path):
    from paper_2301_00817_amd import binding as B
    from paper_2301_00817_amd.solver import Solver
    if not os.path.exists(EXE):
        pytest.skip("C client not built (python -m paper_2301_00817_amd.build)")
    announce("c-client", precision)
    nx, nr, nth, nsteps = 40, 24, 16, 4
    X, R, TH = problems.jet_grid(nx, nr, nth)
    Qi = flow.jet_state(X, R, TH, seed=2).to(torch.float64).contiguous()
    inflow = flow.jet_inflow(R, TH, seed=2).to(torch.float64).contiguous()
    assert Qi.shape == (5, nth, nr, nx) and inflow.shape == (5, nth, nr)
    prec = B.LES_FP32_STORAGE if precision == "fp32" else B.LES_FP64
    src, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(src, "wb") as fh:
        fh.write(np.array([nx, nr, nth, nsteps, prec], dtype=np.int32).tobytes())
        for a in (X, R, TH, Qi, inflow):
            fh.write(a.numpy().astype(np.float64).tobytes())
    r = subprocess.run([EXE, str(src), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stderr)
    got = np.fromfile(out, dtype=np.float64)
    dt_c, q_c = got[:nsteps], got[nsteps:].reshape(5, nth, nr, nx)

    dev = torch.device("cuda:0")
    s = Solver(problems.jet_params(), inflow=inflow.to(dev), precision=precision, device=dev,
               grid=(X, R, TH))
    Q = s.pad(Qi.to(dev), dtype=torch.float64)
    dt_py = s.rk5_step(Q, nsteps).cpu().numpy()
    q_py = s.interior(Q).cpu().numpy()
    s.close()
    assert np.isfinite(q_c).all()
    assert np.array_equal(dt_c, dt_py), (dt_c, dt_py)
    assert np.array_equal(q_c, q_py)
    assert not np.array_equal(q_c, Qi.numpy())       # the steps moved the state
