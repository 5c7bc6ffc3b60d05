"""The swelling strip and the membrane plate against the values the paper
prints for its fluid-structure examples (tests/golden/fsi_paper.txt, each
line citing its passage): density, diffusion and pressure coefficients,
porosity, thickness and the wetted region.  Young's modulus and Poisson's
ratio (100 MPa, 0.4) and the lattice counts are the workload's own, not the
paper's Nafion values; the strip wets its whole top row."""
import os

import numpy as np
import pytest

from paper_2309_04010_amd import cases

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fsi_paper.txt")


@pytest.fixture(scope="module")
def g():
    vals = {}
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split()
                vals[k] = float(v)
    return vals


@pytest.mark.parametrize("name", ["strip2d", "plate3d"])
def test_material_and_saturation(g, name):
    c = cases.by_name(name)
    assert c.material["rho0"] == g["rho"]
    assert c.material["C_swell"] == g["C"]
    assert c.run["D"] == g["D"]
    assert c.run["c_bc"] == g["porosity"]
    wet = (c.flags & cases.CDIR) != 0
    assert np.all(c.c_init[wet] == g["porosity"]) and not np.any(c.c_init[~wet])


def test_strip_width(g):
    c = cases.strip2d()
    assert c.shape[1] * c.dp == pytest.approx(g["W_strip"], rel=1e-12)


def test_plate_thickness_and_wetted_region(g):
    c = cases.plate3d()
    nx, ny, nz = c.shape
    assert nz * c.dp == pytest.approx(g["Lz_plate"], rel=1e-12)
    _, idx = cases.lattice(c.shape, c.dp)
    wet = (c.flags & cases.CDIR) != 0
    assert len(np.unique(idx[0][wet])) == pytest.approx(g["patch_plate"] * nx, abs=1)
    assert len(np.unique(idx[1][wet])) == pytest.approx(g["patch_plate"] * ny, abs=1)
    assert len(np.unique(idx[2][wet])) == g["wet_depth_plate"] * nz
    assert idx[2][wet].min() == nz - g["wet_depth_plate"] * nz
