"""The necking workloads against the values the paper prints for them
(tests/golden/necking_paper.txt, each line citing its passage): the material
table, the specimen geometry and spacing, the loading, the stretching steps
and the relaxation count per increment taken from the reported N_s / N_S."""
import os

import pytest

from paper_2309_04010_amd import cases

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "necking_paper.txt")


def _golden():
    vals = {}
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split()
                vals[k] = float(v)
    return vals


@pytest.fixture(scope="module")
def g():
    return _golden()


@pytest.mark.parametrize("name", ["necking2d", "necking3d"])
def test_material_table(g, name):
    m = cases.by_name(name).material
    E, nu = m["E"], m["nu"]
    assert E / (2 * (1 + nu)) == pytest.approx(g["mu"], rel=1e-12)
    assert E / (3 * (1 - 2 * nu)) == pytest.approx(g["K"], rel=1e-12)
    for k in ("sigma0", "sigma_inf", "delta", "H"):
        assert m[k] == pytest.approx(g[k], rel=1e-15), k
    assert m["model"] == cases.J2


def test_bar_geometry_and_loading(g):
    c = cases.necking2d()
    assert c.dp == pytest.approx(g["dp_2d"], rel=1e-4)
    assert c.dp == pytest.approx(g["width"] / 50, rel=1e-15)
    assert abs(c.observable["length"] - g["length"]) <= 0.5 * c.dp
    assert c.observable["v_pull"] == pytest.approx(g["v_2d"], rel=1e-12)
    # the centre section is narrowed by the imperfection
    ys = c.X[1]
    assert (ys.max() - ys.min()) <= g["width"]
    assert c.V.min() == pytest.approx(c.dp ** 2 * (1 - g["imperfection"]), rel=1e-3)


def test_cylinder_geometry_and_loading(g):
    c = cases.necking3d()
    assert c.dp == g["dp_3d"]
    assert c.observable["radius"] == pytest.approx(g["radius"], rel=1e-15)
    assert abs(c.observable["length"] - g["length"]) <= 0.5 * c.dp
    assert c.observable["v_pull"] == pytest.approx(g["v_3d"], rel=1e-12)
    assert c.observable["v_pull"] * g["t_end"] == pytest.approx(g["disp_3d_end"], rel=1e-12)
    assert c.run["eta"] == g["eta_3d"]


@pytest.mark.parametrize("name,key", [("necking2d", "N_s_2d"), ("necking3d", "N_s_3d")])
def test_schedule(g, name, key):
    r = cases.by_name(name).run
    assert r["n_slow"] == g["N_S"]
    assert r["n_slow"] * r["dt_slow"] == pytest.approx(g["t_end"], rel=1e-12)
    # the relaxation count per increment is the reported average, rounded
    assert r["fixed_inner"] == round(g[key] / g["N_S"])
