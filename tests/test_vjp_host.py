"""The library's hand-written reverse-mode functions and its dual-number
boundary Jacobians, compiled for the host, against central finite
differences of the same device functions' forward forms (no GPU)."""
import ctypes
import os

import pytest

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2301_00817_amd", "_lib", "liblesjet_checks.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} missing: run `python -m paper_2301_00817_amd.build`")
    lib = ctypes.CDLL(LIB)
    for name, args in (("check_point_vjp", [ctypes.c_uint64, ctypes.c_int]),
                       ("check_face_vjp", [ctypes.c_uint64, ctypes.c_int]),
                       ("check_prim_vjp", [ctypes.c_uint64]),
                       ("check_sensor_vjp", [ctypes.c_uint64]),
                       ("check_bc_jacobian", [ctypes.c_uint64, ctypes.c_int, ctypes.c_double])):
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_double
    return lib


@pytest.mark.parametrize("sgs", [0, 1, 2])
def test_point_quantities_vjp(lib, sgs):
    errs = [lib.check_point_vjp(s, sgs) for s in range(1, 40)]
    assert max(errs) < 1e-6, max(errs)


@pytest.mark.parametrize("regime", [0, 1])
def test_face_flux_vjp(lib, regime):
    errs = [lib.check_face_vjp(s, regime) for s in range(1, 40)]
    assert max(errs) < 1e-6, max(errs)


def test_primitive_and_sensor_vjp(lib):
    assert max(lib.check_prim_vjp(s) for s in range(1, 40)) < 1e-7
    assert max(lib.check_sensor_vjp(s) for s in range(1, 40)) < 1e-6


@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("mach", [0.4, -0.4, 1.6, -1.6])
def test_boundary_jacobians(lib, kind, mach):
    errs = [lib.check_bc_jacobian(s, kind, mach) for s in range(1, 20)]
    assert max(errs) < 1e-6, max(errs)
