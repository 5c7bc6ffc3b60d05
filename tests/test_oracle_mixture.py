"""Pins of the oracle's mixture momentum (Sec. 2.2.1 eqs. P_equation,
defination_q, totalmomentumupdate; Sec. 3.2 eqs. totalmomentumupdatesph,
solid_velocity_update, fluid_velocity_update), read in the reference
configuration: the momentum flux v^l (x) q enters as the Piola tensor
rho_l0 v^l (x) Q beside P, the inertia is the mixture's (rho0 + rho_l0 c),
and v^l - v^s = q / rho^l = F Q / c.

* rho_l0 = 0 is the dry path, value for value, whatever c and Q are given;
* one mixture solid step and one damping sweep conserve sum m_a v_a with the
  mixture masses (no constrained particles);
* closed forms at the interior particles of a regular lattice, u = 0 and
  uniform content: a linear solid velocity v = G X with a uniform flux Q
  gives dv/dt = -rho_l0 G Q / (rho0 + rho_l0 c) (a transposed G, a lost
  rho_l0 or the dry mass fail it);
* homogeneous deformation F0, v = 0, uniform Q and content linear in X
  (c = c0 + g.X): the relative velocity F0 Q / c alone gives
  dv/dt = rho_l0 (F0 Q)(g.Q) / (c^2 rho_a) (F0^T instead of F0, a division
  by J c, or the opposite sign of the relative velocity fail it);
* the damping sweep relaxes to the mixture-mass-weighted mean velocity;
* the kinetic energy takes the mixture mass.
"""
import numpy as np
import pytest

from paper_2309_04010_amd import cases

RHO0, RHO_L0 = 2000.0, 1000.0


def _mat(o, rho_l0=RHO_L0, model=cases.NH):
    return o.material(model=model, E=100.0e6, nu=0.3, rho0=RHO0, C_swell=0.0, c0=0.0, rho_l0=rho_l0)


def _lattice(oracle_mod, dim, jitter=0.0, seed=2):
    shape = (16, 15) if dim == 2 else (13, 13, 12)
    dp = 1.0e-3
    X, idx = cases.lattice(shape, dp, jitter=jitter, seed=seed)
    o = oracle_mod.Oracle(dim, X, np.full(X.shape[1], dp ** dim), 1.3 * dp)
    inner = np.ones(o.n, bool)
    ids = o.perm
    for k in range(dim):
        i = idx[k][ids]
        # full support for the particle and for each of its neighbours (two
        # layers away at most), so that every B0 involved is the interior one
        inner &= (i >= 5) & (i < shape[k] - 5)
    return o, inner


def _random_state(o, dim, seed):
    rng = np.random.default_rng(seed)
    u = np.ascontiguousarray(1e-5 * rng.normal(size=(dim, o.n)))
    v = np.ascontiguousarray(rng.normal(size=(dim, o.n)))
    c = np.ascontiguousarray(rng.uniform(0.1, 0.5, o.n))
    q = np.ascontiguousarray(1e-3 * rng.normal(size=(dim, o.n)))
    return u, v, c, q


@pytest.mark.parametrize("dim", [2, 3])
def test_dry_limit_is_the_plain_path(oracle_mod, dim):
    o, _ = _lattice(oracle_mod, dim, jitter=0.1)
    u, v, c, q = _random_state(o, dim, 1)
    m0 = _mat(o, rho_l0=0.0)
    v1, v2 = v.copy(), v.copy()
    r1 = o.solid_step(m0, 1e-6, u, v1)
    r2 = o.solid_step(m0, 1e-6, u, v2, c=c, q=q)
    assert np.array_equal(v1, v2) and np.array_equal(r1[2], r2[2]) and np.array_equal(r1[1], r2[1])
    o.damping_sweep(RHO0, 10.0, 1e-6, v1)
    o.damping_sweep(RHO0, 10.0, 1e-6, v2, rho_l0=0.0, c=c)
    assert np.array_equal(v1, v2)
    u1, u2 = u.copy(), u.copy()
    assert o.drift_ke(RHO0, 1e-6, u1, v1) == o.drift_ke(RHO0, 1e-6, u2, v2, rho_l0=0.0, c=c)


@pytest.mark.parametrize("dim", [2, 3])
def test_momentum_conserved(oracle_mod, dim):
    o, _ = _lattice(oracle_mod, dim, jitter=0.15)
    u, v, c, q = _random_state(o, dim, 2)
    m = _mat(o)
    mass = (RHO0 + RHO_L0 * c) * o.V
    v1 = v.copy()
    rc, PB, acc = o.solid_step(m, 1e-3, u, v1, c=c, q=q)
    dp = (mass * (v1 - v)).sum(axis=1)
    assert np.all(np.abs(dp) <= 1e-12 * (mass * np.abs(v1 - v)).sum(axis=1))
    # the flux term is present: the dry step differs
    v2 = v.copy()
    o.solid_step(_mat(o, rho_l0=0.0), 1e-3, u, v2)
    assert np.abs(v2 - v1).max() > 1e-3 * np.abs(v1 - v).max()
    w = v1.copy()
    o.damping_sweep(RHO0, 10.0, 1e-5, w, rho_l0=RHO_L0, c=c)
    assert np.all(np.abs((mass * (w - v1)).sum(axis=1)) <= 1e-12 * (mass * np.abs(v1)).sum(axis=1))


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_velocity_closed_form(oracle_mod, dim):
    o, inner = _lattice(oracle_mod, dim)
    G = np.array([[0.3, -1.2, 0.7], [0.9, 0.2, -0.4], [-0.5, 1.1, 0.6]])[:dim, :dim]
    Xc = o.X - o.X.mean(axis=1, keepdims=True)
    v = np.ascontiguousarray(G @ Xc)
    cbar = 0.3
    c = np.full(o.n, cbar)
    Q = np.array([2.0e-3, -1.0e-3, 1.5e-3])[:dim]
    q = np.ascontiguousarray(np.repeat(Q[:, None], o.n, axis=1))
    rc, PB, acc = o.solid_step(_mat(o), 0.0, o.arr(dim, o.n), v.copy(), c=c, q=q)
    want = -RHO_L0 * (G @ Q) / (RHO0 + RHO_L0 * cbar)
    got = acc[:, inner]
    assert np.allclose(got, want[:, None], rtol=1e-9, atol=1e-9 * np.abs(want).max())
    wrong = -RHO_L0 * (G.T @ Q) / (RHO0 + RHO_L0 * cbar)
    assert np.abs(wrong - want).max() > 0.1 * np.abs(want).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_relative_velocity_closed_form(oracle_mod, dim):
    o, inner = _lattice(oracle_mod, dim)
    F0 = np.eye(dim) + np.array([[0.05, 0.12, -0.03], [-0.07, 0.04, 0.09], [0.02, -0.06, 0.08]])[:dim, :dim]
    Xc = o.X - o.X.mean(axis=1, keepdims=True)
    u = np.ascontiguousarray((F0 - np.eye(dim)) @ Xc)
    g = np.array([4.0, -3.0, 2.0])[:dim]
    c = np.ascontiguousarray(0.3 + g @ Xc)
    Q = np.array([2.0e-3, -1.0e-3, 1.5e-3])[:dim]
    q = np.ascontiguousarray(np.repeat(Q[:, None], o.n, axis=1))
    m = _mat(o)
    rc, PB, acc = o.solid_step(m, 0.0, u, o.arr(dim, o.n), c=c, q=q)
    # the homogeneous stress alone gives no interior force: remove it
    rc, PBd, accd = o.solid_step(_mat(o, rho_l0=0.0), 0.0, u, o.arr(dim, o.n))
    rho = RHO0 + RHO_L0 * c
    f = acc * rho - accd * RHO0
    want = RHO_L0 * np.outer(F0 @ Q, np.ones(o.n)) * (g @ Q) / c ** 2
    scale = np.abs(want[:, inner]).max()
    assert np.abs(f[:, inner] - want[:, inner]).max() <= 1e-3 * scale
    wrong = RHO_L0 * np.outer(F0.T @ Q, np.ones(o.n)) * (g @ Q) / c ** 2
    assert np.abs(wrong[:, inner] - want[:, inner]).max() > 1e-2 * scale


def test_damping_relaxes_to_mixture_mean(oracle_mod):
    o, _ = _lattice(oracle_mod, 2, jitter=0.1)
    rng = np.random.default_rng(5)
    v = np.ascontiguousarray(rng.normal(size=(2, o.n)))
    c = np.ascontiguousarray(rng.uniform(0.0, 0.8, o.n))
    mass = (RHO0 + RHO_L0 * c) * o.V
    mean = (mass * v).sum(axis=1) / mass.sum()
    dry = (o.V * v).sum(axis=1) / o.V.sum()
    assert np.abs(dry - mean).max() > 1e-3 * np.abs(mean).max()   # the masses matter here
    for _ in range(400):
        o.damping_sweep(RHO0, 2.0e3, 1e-3, v, rho_l0=RHO_L0, c=c)
    assert np.abs(v - mean[:, None]).max() <= 1e-8 * np.abs(mean).max()


def test_kinetic_energy_mixture_mass(oracle_mod):
    o, _ = _lattice(oracle_mod, 3, jitter=0.1)
    rng = np.random.default_rng(6)
    v = np.ascontiguousarray(rng.normal(size=(3, o.n)))
    cbar = 0.35
    c = np.full(o.n, cbar)
    ke_dry = o.drift_ke(RHO0, 0.0, o.arr(3, o.n), v)
    ke_mix = o.drift_ke(RHO0, 0.0, o.arr(3, o.n), v, rho_l0=RHO_L0, c=c)
    assert ke_mix == pytest.approx(ke_dry * (RHO0 + RHO_L0 * cbar) / RHO0, rel=1e-14)
