"""The constants and workloads of this build against the values the paper
prints (tests/golden/paper_values.json, each entry with its passage)."""
import json
import math
import os
from fractions import Fraction

import numpy as np

from cases import flow, problems
from oracle import les

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _v(key):
    return GOLDEN[key]["value"]


def test_physical_and_numerical_constants():
    p = problems.base_params()
    assert p["Pr"] == _v("Pr")
    assert p["Pr_sgs"] == _v("Pr_sgs_static")
    assert p["Cs"] == _v("Cs_lilly")
    assert p["k2"] == _v("k2")
    assert p["k4"] == _v("k4")
    # Sutherland's S1 enters in units of the reference temperature (288.15 K,
    # the jet's static temperature of the dimensionless formulation)
    assert p["suth_S"] == _v("sutherland_S1_kelvin") / 288.15
    alpha = [Fraction(a, b) for a, b in _v("rk_alpha")]
    assert [Fraction(x).limit_denominator(64) for x in p["rk_alpha"]] == alpha
    assert all(abs(x - float(a)) == 0.0 for x, a in zip(p["rk_alpha"], alpha))
    assert flow.JET_UJ == _v("jet_mach")


def test_rk_scheme_stable_up_to_the_printed_bound():
    """The oracle's five-stage scheme with the printed alphas, applied to
    R(Q) = i y Q / dt, keeps |Q^(n+1)| <= |Q^n| for |y| up to the printed
    linear bound 2 sqrt(2)."""
    assert _v("cfl_linear_stability_bound") == "2 sqrt(2)"
    alpha = [a / b for a, b in _v("rk_alpha")]
    for y in np.linspace(0.0, 2.0 * math.sqrt(2.0), 41):
        q1 = les.jameson_rk(np.array([1.0 + 0j]), lambda q: -1j * y * q, 1.0, alpha)[0]
        assert abs(q1) <= 1.0 + 1e-15, y


def test_mesh_family_matches_the_table():
    """Axial and radial counts are the table's; the table's 361 azimuthal
    points repeat the periodic one, so the build runs 360 distinct ones, and
    the table's totals are its products with 361 to the printed digits."""
    table = _v("mesh_family")
    assert set(table) == set(problems.PAPER_MESHES)
    for m, (nx, nr, nth, total) in table.items():
        assert problems.PAPER_MESHES[m] == (nx, nr)
        assert problems.CONFIGS["mesh" + m]["shape"] == (nx, nr, nth - 1)
        n = nx * nr * nth
        scale, digits = (1e9, total[:-1]) if total.endswith("B") else (1e6, total[:-1])
        decimals = len(digits.split(".")[1]) if "." in digits else 0
        assert round(n / scale, decimals) == float(digits), (m, n, total)
