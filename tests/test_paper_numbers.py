"""Numbers the paper prints, checked against the DOF counting and the
blending defaults used here (tests/golden/paper_numbers.json)."""
import json
import os

import numpy as np

from paper_2306_12891_amd import inputs as I

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def dof(N, nelem):
    return nelem * (N + 1) ** 3


def test_dof_counts(orc):
    g = GOLD["dof_per_element_N7"]
    assert dof(g["N"], 1) == g["value"]
    U = I.freestream(7, (1, 1, 1))
    assert U.shape[2] * U.shape[3] * U.shape[4] == g["value"]
    h = GOLD["hit_meshes_N5"]
    for ne, m in zip(h["elements"], h["dof_million"]):
        assert abs(dof(h["N"], ne) / 1e6 - m) / m < 0.02
    r = GOLD["rotor37"]
    assert abs(dof(r["N"], r["elements"]) - r["dof"]) / r["dof"] < 1e-3
    w = GOLD["pid_wrles"]
    # 370e6 DOF on 723,132 elements is N = 7 (512 DOF per element)
    assert round((w["dof"] / w["elements"]) ** (1 / 3)) - 1 == 7


def test_blending_defaults(orc):
    s = orc.Setup(N=3, blending=1)
    assert s.alpha_min == GOLD["alpha_bounds"]["alpha_min"]
    assert s.alpha_max == GOLD["alpha_bounds"]["alpha_max"]
    assert s.alpha_spread == GOLD["alpha_spread"]["value"]
