"""Input generators: counter-based random numbers and meshes."""
import math

import numpy as np
import torch

from cases import mesh, rng


def test_splitmix64_matches_integer_definition():
    xs = [0, 1, 2, 12345, 2 ** 63 - 1, 2 ** 63, 2 ** 64 - 1, 0xDEADBEEFCAFEBABE]
    t = torch.tensor([x - (1 << 64) if x >= (1 << 63) else x for x in xs], dtype=torch.int64)
    out = rng.splitmix64(t)
    for x, y in zip(xs, out.tolist()):
        assert (y & ((1 << 64) - 1)) == rng.splitmix64_int(x)


def test_splitmix64_known_value():
    # first output of the splitmix64 generator seeded with 0 (published
    # reference sequence of the algorithm): 0xE220A8397B1DCDAF
    assert rng.splitmix64_int(0) == 0xE220A8397B1DCDAF


def test_uniform_range_and_chunk_independence():
    idx = torch.arange(100000, dtype=torch.int64)
    u = rng.uniform(7, 3, idx)
    assert float(u.min()) >= 0.0 and float(u.max()) < 1.0
    assert abs(float(u.mean()) - 0.5) < 0.01
    part = rng.uniform(7, 3, idx[500:900])
    assert torch.equal(part, u[500:900])
    other = rng.uniform(7, 4, idx)
    assert not torch.equal(other, u)


def test_jet_mesh_recipe():
    X = mesh.jet_axial(288)
    assert X[0] == 0.0 and abs(float(X[-1]) - 30.0) < 1e-12
    dx = (X[1:] - X[:-1]).numpy()
    assert np.allclose(dx[1:] / dx[:-1], 1.005, rtol=1e-9, atol=0)
    R = mesh.jet_radial(160).numpy()
    assert abs(R[0] - 0.005) < 1e-15 and abs(R[-1] - 20.0) < 1e-12
    dr = np.diff(R)
    assert np.all(dr > 0)
    # finest spacing sits at the lip line r = 0.5 D
    assert abs(R[np.argmin(dr)] - 0.5) < 0.02
    TH = mesh.azimuth(128).numpy()
    assert abs(TH[1] - 2 * math.pi / 128) < 1e-15
