"""Pins of the necking workloads (Sec. 5.1 and 5.2) and of their observables
on the oracle.

* the material is the necking table: E and nu give back its shear and bulk
  moduli;
* the imperfect 2D bar's area is the closed form of its linear taper (the
  midpoint sum of a piecewise-linear width whose kink falls on a column
  boundary is exact), and its centre width is reduced by the imperfection;
* the cylinder's sites lie inside the tapered radius, and its centre ring
  follows the taper;
* observables: after small-strain stretching and a long relaxation (elastic
  throughout), the reaction forces of the two grips are equal and opposite,
  and the reaction force and the neck's inward displacement match the
  uniaxial closed forms (plane strain in 2D: E/(1 - nu^2) eps W and
  nu/(1 - nu) eps w/2; the cylinder: E eps A and nu eps r).  A wrong sign, a
  missing mass or volume factor, or a wrong component fails them.
"""
import numpy as np
import pytest

from paper_2309_04010_amd import cases


def test_table_moduli():
    m = cases.necking2d(across=10).material
    E, nu = m["E"], m["nu"]
    t = cases.NECK_TABLE
    assert abs(E / (2 * (1 + nu)) - t["mu"]) <= 1e-12 * t["mu"]
    assert abs(E / (3 * (1 - 2 * nu)) - t["K"]) <= 1e-12 * t["K"]
    assert (m["sigma0"], m["sigma_inf"], m["delta"], m["H"]) == (450.0e6, 715.0e6, 16.93, 129.24e6)


def test_imperfect_bar_geometry():
    c = cases.necking2d()
    nx, ny = c.shape
    assert (ny, c.dp) == (50, cases.NECK_WIDTH / 50) and c.n == nx * ny
    L = c.observable["length"]
    grips = 2 * 3 * c.dp
    area = cases.NECK_WIDTH * (L * (1 - 0.018 / 2) + grips)
    assert abs(c.V.sum() - area) <= 1e-12 * area
    # centre columns: width between particle centres reduced by the taper
    col = np.arange(c.n) % nx
    for j in ((nx - 1) // 2, nx // 2):
        y = c.X[1, col == j]
        s = 1 - 0.018 * (1 - abs((j + 0.5) * c.dp - 0.5 * nx * c.dp) / (0.5 * L))
        assert abs((y.max() - y.min()) - s * (cases.NECK_WIDTH - c.dp)) <= 1e-15
    assert c.flags[col < 3].all() and c.flags[col >= nx - 3].all() and not c.flags[(col >= 3) & (col < nx - 3)].any()


def test_cylinder_geometry():
    c = cases.necking3d(dp=1.0e-3)
    L = c.observable["length"]
    x_c = 0.5 * c.shape[0] * c.dp
    s = 1 - 0.018 * np.clip(1 - np.abs(c.X[0] - x_c) / (0.5 * L), 0, 1)
    r = np.sqrt(c.X[1] ** 2 + c.X[2] ** 2)
    assert np.all(r <= cases.NECK_RADIUS * s * (1 + 1e-14))
    assert np.allclose(c.V, c.dp ** 3 * s * s, rtol=1e-14)
    ring = c.observable["w_u"][1] != 0
    assert np.all(r[ring] > (cases.NECK_RADIUS - c.dp) * s[ring])
    # radial weights: unit vectors, averaged
    w = c.observable["w_u"][1:, ring]
    assert np.allclose((w ** 2).sum(axis=0), 1.0 / ring.sum() ** 2)


def _relaxed(oracle_mod, c, n_inc, inner, extra):
    o = oracle_mod.Oracle(c.dim, c.X, c.V, c.h)
    perm = o.perm
    flags = np.ascontiguousarray(c.flags[perm])
    vg = np.ascontiguousarray(c.vgrip[:, perm])
    mat = o.material(**c.material)
    u, v = o.arr(c.dim, c.n), o.arr(c.dim, c.n)
    pl, acc = o.arr(7, c.n), o.arr(c.dim, c.n)
    run = dict(c.run, n_slow=n_inc, fixed_inner=inner,
               dt_slow=c.run["dt_slow"] * c.run["n_slow"] / n_inc)
    o.advance(mat, o.cfg(**run), u, v, plastic=pl, vgrip=vg, flags=flags, acc=acc)
    # hold the grips and relax
    o.advance(mat, o.cfg(**dict(run, n_slow=1, fixed_inner=extra)), u, v, plastic=pl,
              vgrip=np.zeros_like(vg), flags=flags, acc=acc)
    assert pl[6].max() == 0.0            # elastic throughout
    F = (c.observable["w_acc"][:, perm] * acc).sum()
    dr = (c.observable["w_u"][:, perm] * u).sum()
    left = (flags & cases.GRIP).astype(bool) & (o.X[0] < o.X[0].mean())
    F_left = c.material["rho0"] * (o.V[left] * acc[0, left]).sum()
    return F, F_left, dr


def test_bar_observables_elastic(oracle_mod):
    c = cases.necking2d(across=10, n_slow=1, total_stretch=0.5e-4, imperfection=0.0)
    F, F_left, dr = _relaxed(oracle_mod, c, 10, 100, 2000)
    E, nu = c.material["E"], c.material["nu"]
    eps = c.observable["total_stretch"] / (c.observable["length"] + c.dp)
    assert abs(F - F_left) <= 2e-4 * F
    F_an = E / (1 - nu ** 2) * eps * c.observable["width"]
    assert F == pytest.approx(F_an, rel=0.03)
    assert dr == pytest.approx(nu / (1 - nu) * eps * 0.5 * (c.observable["width"] - c.dp), rel=0.03)


def test_cylinder_observables_elastic(oracle_mod):
    c = cases.necking3d(dp=2.0e-3, n_slow=1, total_stretch=0.5e-4, imperfection=0.0)
    F, F_left, dr = _relaxed(oracle_mod, c, 10, 100, 1000)
    E, nu = c.material["E"], c.material["nu"]
    eps = c.observable["total_stretch"] / (c.observable["length"] + c.dp)
    assert abs(F - F_left) <= 2e-4 * F
    end = np.isclose(c.X[0], c.X[0].min())
    A = c.V[end].sum() / c.dp
    assert F == pytest.approx(E * eps * A, rel=0.05)
    ring = c.observable["w_u"][1] != 0
    r_ring = np.sqrt(c.X[1, ring] ** 2 + c.X[2, ring] ** 2).mean()
    assert dr == pytest.approx(nu * eps * r_ring, rel=0.08)
