"""The golden closed-form values agree with their formulas (guards the fixture file itself)."""
import math
import os

import pins

HERE = os.path.dirname(os.path.abspath(__file__))


def load_golden():
    vals = {}
    with open(os.path.join(HERE, "golden", "closed_forms.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_golden_values():
    g = load_golden()
    assert abs(g["unit_square_coulomb"] - pins.unit_square_coulomb()) < 1e-14
    assert abs(g["disk_energy"] - 8.0 / 3.0) < 1e-15
    assert abs(g["disk_phi_center"] + 2.0 / math.pi) < 1e-15
    for n, key in ((96, "dofs_crossed96"), (192, "dofs_crossed192")):
        assert g[key] == 3 * ((n - 1) ** 2 - (2 * n - 3)) + 9 * (n - 2) + 7
    assert g["dofs_book48"] == 3 * 47 * 47 + 47 * 2
    assert g["dofs_square16"] == 15 * 15
