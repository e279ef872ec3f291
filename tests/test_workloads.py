"""The seeded workload definitions: the refinement-level geometry of the
paper's setting keeps every box inside its level with the stated margin and
the finest level holds the body-fitted grid and its motion."""
import math

import pytest

from paper_2006_13631_amd.workloads import paper_levels


@pytest.mark.parametrize("b,nlevels,margin", [(800, 4, 16), (256, 4, 8), (128, 3, 8)])
def test_paper_levels_geometry(b, nlevels, margin):
    d = paper_levels(b=b, nlevels=nlevels, margin=margin)
    assert d["nx0"] == d["ny0"] == (5 * b) // 2 ** (nlevels - 1) + 1  # 5L x 5L at level 0
    nx, ny = d["nx0"], d["ny0"]
    for x0, y0, x1, y1 in d["boxes"]:
        assert x0 >= margin and y0 >= margin and x1 <= nx - 1 - margin and y1 <= ny - 1 - margin
        assert x1 - x0 >= 4 and y1 - y0 >= 4
        nx, ny = 2 * (x1 - x0) + 1, 2 * (y1 - y0) + 1
    assert (nx, ny) == d["finest"]
    f = d["fine"]
    A = f["kc"] * b / (2 * math.pi)
    # the grid (4b x b nodes, spacing 1) and its motion stay inside the finest lattice
    assert nx // 2 - f["nux"] // 2 >= 1 and nx // 2 + (f["nux"] - 1 - f["nux"] // 2) <= nx - 2
    assert (ny - 1) / 2 - (f["nuy"] - 1) / 2 - abs(A) >= 1


def test_paper_levels_too_small_a_domain():
    with pytest.raises(ValueError):
        paper_levels(b=64, nlevels=4, margin=16)
