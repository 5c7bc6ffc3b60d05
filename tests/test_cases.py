"""The seeded synthetic inputs, pinned to the recipe the measurements quote:
sizes, spacing, support, volumes, boundary sets, seeds and the draws of the
batched sweep.  A change to a generator shows here before it moves a
measured number."""
import numpy as np
import pytest

from paper_2309_04010_amd import cases


def _common(c, n, dim, dp):
    assert c.n == n and c.dim == dim and c.X.shape == (dim, n)
    assert c.dp == dp
    assert c.h == pytest.approx(1.3 * dp, rel=1e-15)
    assert np.all(c.V == dp ** dim)
    assert c.flags.dtype == np.uint8 and c.flags.shape == (n,)


def test_bar2d():
    c = cases.bar2d()
    _common(c, 320, 2, 0.25e-3)
    X, idx = cases.lattice((40, 8), 0.25e-3)
    assert np.array_equal(c.X, X)
    left, right = idx[0] < 3, idx[0] >= 37
    assert np.all(c.flags[left | right] & cases.FIXED)
    assert not np.any(c.flags[~(left | right)])
    assert np.all(c.flags[right] & cases.GRIP) and not np.any(c.flags[left] & cases.GRIP)
    assert np.all(c.vgrip[0, right] == 1.0e-3) and not np.any(c.vgrip[:, ~right])
    assert c.run["n_slow"] == 100 and c.run["dt_slow"] == 1.0e-3 and c.run["fixed_inner"] == 0
    assert c.material["E"] == 210.0e9 and c.material["nu"] == 0.3 and c.material["rho0"] == 7850.0


def test_strip2d():
    c = cases.strip2d()
    _common(c, 2000, 2, 12.5e-6)
    _, idx = cases.lattice((200, 10), 12.5e-6)
    top = idx[1] == 9
    assert np.all(c.c_init[top] == 0.4) and not np.any(c.c_init[~top])
    assert np.all(c.flags[top] & cases.CDIR)
    ends = (idx[0] < 3) | (idx[0] >= 197)
    assert np.all(c.flags[ends] & cases.FIXED) and not np.any(c.flags[~ends] & cases.FIXED)
    assert c.run["D"] == 1.0e-10 and c.run["c_bc"] == 0.4 and c.run["n_slow"] == 100
    assert c.vgrip is None


def test_neck3d_jitter_is_seeded_and_bounded():
    c = cases.neck3d()
    _common(c, 40000, 3, 0.53334e-3)
    X0, _ = cases.lattice((100, 20, 20), 0.53334e-3)
    d = np.abs(c.X - X0)
    assert d.max() <= 0.01 * 0.53334e-3 and d.max() > 0.009 * 0.53334e-3
    assert np.array_equal(c.X, cases.neck3d().X)
    assert not np.array_equal(c.X, cases.neck3d(seed=4).X)
    assert c.run["n_slow"] == 100 and c.run["fixed_inner"] == 1000
    assert c.material["model"] == cases.J2


def test_plate3d():
    c = cases.plate3d()
    _common(c, 1_000_000, 3, 31.25e-6)
    _, idx = cases.lattice((500, 500, 4), 31.25e-6)
    side = (idx[0] < 3) | (idx[0] >= 497) | (idx[1] < 3) | (idx[1] >= 497)
    assert np.array_equal((c.flags & cases.FIXED) != 0, side)
    wet = (c.flags & cases.CDIR) != 0
    # the top 2 layers of the central 0.3 L x 0.3 L patch: 150 x 150 x 2
    assert wet.sum() == 150 * 150 * 2 and np.all(idx[2][wet] >= 2)
    assert np.all(c.c_init[wet] == 0.4) and not np.any(c.c_init[~wet])
    # the observable: the two centre columns of each axis, all four layers
    assert len(c.observable["J_index"]) == 16 and c.observable["J_component"] == 2
    assert set(idx[0][c.observable["J_index"]]) == {249, 250}
    assert c.run["n_slow"] == 50 and c.run["fixed_inner"] == 1000


def test_necking_specimens():
    c2 = cases.necking2d()
    assert c2.n == 10700 and c2.dim == 2
    c3 = cases.necking3d()
    assert c3.n == 264224 and c3.dim == 3
    for c in (c2, c3):
        assert c.run["n_slow"] == 10000 and c.material["model"] == cases.J2


def test_strips_sweep_draws():
    ss = cases.strips_sweep()
    assert len(ss) == 64
    n = np.array([s.n for s in ss])
    assert n.sum() == 819780
    assert n.min() >= 1000 - 10 and n.max() <= 50000 + 10
    E = np.array([s.material["E"] for s in ss])
    D = np.array([s.run["D"] for s in ss])
    assert np.all((E >= 50e6) & (E <= 200e6))
    assert np.all((D >= 1e-11) & (D <= 1e-9))
    # the draws are in the order sizes, E, D from one generator of seed 5
    rng = np.random.default_rng(5)
    sizes = np.rint(np.exp(rng.uniform(np.log(1000), np.log(50000), 64))).astype(int)
    assert np.array_equal(E, rng.uniform(50e6, 200e6, 64))
    assert np.array_equal([s.shape[0] for s in ss], [max(int(round(N / 10)), 8) for N in sizes])
    b = cases.batch(ss)
    assert b.n == 819780 and np.array_equal(np.diff(b.offsets), n)
    # a batch carries no step sizes: each side derives its own
    assert "dt_s" not in b.run or not b.run["dt_s"]
