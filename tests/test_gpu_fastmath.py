"""The kernels' fast arithmetic against correctly rounded results, on the
device, over the argument ranges the kernels meet.

FP64 (every FP64 kernel): 1/x by the hardware estimate refined twice by
Newton-Raphson, sqrt(x) by the reciprocal-root estimate refined by
Goldschmidt iterations and one final correction; asserted within 1 ulp of
the IEEE results (numpy's division and square root are correctly rounded).
Ranges: reciprocals of densities, temperatures, pressure sums and of J^-1,
which reaches about 1e-11 on the 1.0e9-point jet mesh and changes sign
across the axis (ghost cells), so |x| in [1e-13, 1e6] with both signs;
square roots of temperatures, metric norms |S|^2 (down to about 1e-16 on
that mesh), strain invariants and spectral-radius products, so x in
[1e-20, 1e12], plus x = 0 (sqrt(0) = 0).

FP32 (the FP32-storage form only): hardware reciprocal and square root,
within 1 ulp; cube root as exp2(log2(x) / 3) from the hardware base-2
logarithm and exponential, within 32 ulp (4e-6 relative: the absolute
error of the logarithm, about an ulp of log2(x), becomes a relative error
of the result that grows with |log2 x|; 22 ulp measured at x near 1e-13),
for the filter width |J^-1|^(1/3), x in [1e-13, 1e6]."""
import ctypes
import os

import numpy as np
import pytest
import torch

from _helpers import announce

pytestmark = pytest.mark.gpu

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2301_00817_amd", "_lib", "liblesjet_devchecks.so")


def _ulps(a, b):
    """|a - b| in units in the last place (same-sign finite arrays)."""
    if a.dtype == np.float64:
        ia, ib = a.view(np.int64), b.view(np.int64)
    else:
        ia, ib = a.view(np.int32).astype(np.int64), b.view(np.int32).astype(np.int64)
    return np.abs(ia - ib)


def _run(x):
    lib = ctypes.CDLL(LIB)
    lib.lesjet_check_fastmath.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_longlong,
                                          ctypes.c_void_p]
    lib.lesjet_check_fastmath.restype = ctypes.c_int
    xd = torch.from_numpy(x).cuda()
    out = torch.empty(5 * x.size, dtype=torch.float64, device="cuda")
    rc = lib.lesjet_check_fastmath(xd.data_ptr(), out.data_ptr(), x.size,
                                   torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(5, x.size)


def _logspace(lo, hi, n, seed):
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), n)


def test_fp64_reciprocal_and_root_within_one_ulp():
    announce("fastmath fp64")
    special = np.array([1.0, 2.0, 0.5, 3.0, 1.4, 1.0 / 1.4, 0.383134, 1.383134, 2.0 ** 40,
                        2.0 ** -40, np.nextafter(1.0, 2.0), np.nextafter(1.0, 0.0)])
    xr = np.concatenate([special, _logspace(1e-13, 1e6, 200000, 1)])
    xr = np.concatenate([xr, -xr])
    out = _run(xr)
    u_rcp = _ulps(out[0], 1.0 / xr)
    xs = np.concatenate([special, _logspace(1e-20, 1e12, 400000, 2)])
    out_s = _run(xs)
    u_sqrt = _ulps(out_s[1], np.sqrt(xs))
    zero = _run(np.array([0.0]))
    print(f"FP64 rcp max {u_rcp.max()} ulp (mean {u_rcp.mean():.3f}), "
          f"sqrt max {u_sqrt.max()} ulp (mean {u_sqrt.mean():.3f})")
    assert u_rcp.max() <= 1
    assert u_sqrt.max() <= 1
    assert zero[1, 0] == 0.0


def test_fp32_reciprocal_root_and_cube_root():
    announce("fastmath fp32")
    x = np.concatenate([np.array([1.0, 2.0, 0.5, 3.0, 1.4]), _logspace(1e-13, 1e6, 200000, 3)])
    x = x.astype(np.float32).astype(np.float64)        # exactly representable in FP32
    out = _run(x)
    f = x.astype(np.float32)
    u_rcp = _ulps(out[2].astype(np.float32), np.float32(1.0) / f)
    u_sqrt = _ulps(out[3].astype(np.float32), np.sqrt(f))
    u_cbrt = _ulps(out[4].astype(np.float32), np.cbrt(x).astype(np.float32))
    print(f"FP32 rcp max {u_rcp.max()} ulp, sqrt max {u_sqrt.max()} ulp, "
          f"cbrt max {u_cbrt.max()} ulp")
    assert u_rcp.max() <= 1
    assert u_sqrt.max() <= 1
    assert u_cbrt.max() <= 32
