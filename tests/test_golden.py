"""Golden values the paper prints (tests/golden/paper_sample_q.txt)."""
import math
import os

from paper_2111_06623_amd import units

HERE = os.path.dirname(__file__)


def _read(name):
    out = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()[:2]
                out[k] = float(v)
    return out


def test_sample_transferred_momentum_matches_figure_caption():
    g = _read("paper_sample_q.txt")
    q = units.q_from_alat_units([g["q1_2pi_over_a"], 0, 0], g["celldm_bohr"])
    qa = units.inv_bohr_to_inv_angstrom(math.hypot(*q))
    # the caption quotes two significant digits
    assert abs(qa - g["Q_inv_angstrom"]) < 0.005


def test_broadening_in_hartree():
    g = _read("paper_sample_q.txt")
    assert abs(units.ry_to_ha(g["eta_Ry"]) - 0.015) < 1e-15
    assert abs(units.ry_to_ha(g["epsil_default_Ry"]) - 0.01) < 1e-15
