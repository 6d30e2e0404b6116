"""The two mesh forms of les_init_grid: coordinates (host or device memory)
and the 1-D maps of a cylindrical product mesh (section "Mesh Generation":
the 3-D jet mesh is an axial-radial mesh rotated about the axis).  The maps
are turned into coordinates with the host C library's cos and sin, as the
test inputs are, so all three forms give the same metrics bitwise; the
metrics also match the oracle's."""
import math

import numpy as np
import pytest
import torch

from _helpers import announce, to_np
from cases import mesh, problems
from oracle import les

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,axis_node", [((37, 22, 20), False), ((64, 40, 96), False),
                                             ((21, 12, 16), True)])
def test_product_maps_host_and_device_coordinates_agree(shape, axis_node):
    """Also a mesh whose first radial row lies on the axis (R = 0)."""
    from paper_2301_00817_amd.solver import Solver
    announce("init forms", shape, "axis node" if axis_node else "")
    pb = problems.jet_problem(*shape, seed=2, axis_node=axis_node)
    X, R, TH = pb["grid"]
    prm = pb["params"]
    out = []
    for form in ("maps", "maps_device", "xyz_host", "xyz_device"):
        if form == "maps":
            s = Solver(prm, grid=(X, R, TH), keep_metrics=True)
        elif form == "maps_device":
            s = Solver(prm, grid=(X.cuda(), R.cuda(), TH.cuda()), keep_metrics=True)
        elif form == "xyz_host":
            s = Solver(prm, pb["xyz"], keep_metrics=True)
        else:
            s = Solver(prm, pb["xyz"].cuda(), keep_metrics=True)
        out.append(to_np(s.metrics64))
        s.close()
    for m in out[1:]:
        assert np.array_equal(m, out[0])
    geo = les.geometry(pb["xyz"].numpy(), prm)
    nx = shape[0]
    M = out[0][..., :nx + 4]
    S = geo["S"].reshape(9, *geo["V"].shape)
    assert np.abs(M[:9] - S).max() <= 1e-14 * np.abs(S).max()
    assert np.abs(M[9] - geo["V"]).max() <= 1e-14 * np.abs(geo["V"]).max()


def test_product_maps_build_the_cylindrical_coordinates():
    """The C library's angles reproduce x = X, y = R cos, z = R sin of the
    input generator exactly (the premise of the bitwise comparisons)."""
    X, R, TH = problems.jet_grid(9, 7, 12)
    xyz = mesh.cylindrical_coords(X, R, TH)
    for k in range(12):
        c, s = math.cos(float(TH[k])), math.sin(float(TH[k]))
        assert float(xyz[1, k, 3, 0]) == float(R[3]) * c
        assert float(xyz[2, k, 3, 0]) == float(R[3]) * s


def test_non_finite_maps_are_rejected():
    from paper_2301_00817_amd import binding as B
    announce("init non-finite maps")
    pb = problems.jet_problem(12, 8, 8)
    p = B.make_params(pb["params"], (12, 8, 8), B.LES_FP64)
    X, R, TH = (t.clone().contiguous() for t in pb["grid"])
    R[3] = float("nan")
    stream = torch.cuda.current_stream().cuda_stream
    with pytest.raises(B.LesError) as e:
        B.les_init_grid(p, None, X.data_ptr(), R.data_ptr(), TH.data_ptr(), stream)
    assert e.value.code == B.LES_EINVAL


def test_query_reports_the_padded_shape():
    from paper_2301_00817_amd.solver import Solver
    announce("query")
    pb = problems.jet_problem(37, 22, 20)
    s = Solver(pb["params"], grid=pb["grid"])
    dims, pitch, held = s.query()
    assert dims == (5,) + s.dims and pitch == s.dims[2] == s.pitch
    assert held >= 10 * s.vs * 8
    s.close()
