"""Pins of the oracle's two-way coupled diffusion step (Sec. 2.2.2 eqs.
grad_q / fluid_mass_der, Sec. 3.2 eqs. fluid_mass_sph / ralative_velocity_sph
with the updated-Lagrangian kernel gradient F^-1 grad0 W stated there).

* undeformed body, linear flux: the step is the linear diffusion step,
  value for value;
* fluid mass sum_a V_a c_a is conserved for any deformation and either flux
  law (antisymmetric corrected divergence);
* homogeneous deformation F0 (general, non-symmetric, J != 1) with a
  saturation linear in X: the reference flux is J0 F0^-1 (-D w F0^-T alpha)
  at every particle (a transposed F^-1, a missing J or a missing saturation
  factor each fail it), and with the linear flux the content is stationary
  where every neighbour has full support;
* Dirichlet particles hold saturation c_bc, i.e. content c_bc J.
"""
import numpy as np
import pytest

from paper_2309_04010_amd import cases


def _system(oracle_mod, dim, shape=None, jitter=0.15, seed=11, dp=1.0e-3):
    if shape is None:
        shape = (12, 9) if dim == 2 else (8, 7, 6)
    X, idx = cases.lattice(shape, dp, jitter=jitter, seed=seed)
    o = oracle_mod.Oracle(dim, X, np.full(X.shape[1], dp ** dim), 1.3 * dp)
    return o, X, idx


def _smooth_u(o, dim, amp, seed):
    rng = np.random.default_rng(seed)
    L = np.ptp(o.X, axis=1).max()
    k = rng.uniform(0.5, 1.5, (dim, dim))
    ph = rng.uniform(0, 2 * np.pi, (dim, dim))
    u = np.zeros((dim, o.n))
    for i in range(dim):
        for j in range(dim):
            u[i] += amp * L * np.sin(k[i, j] * 2 * np.pi * o.X[j] / L + ph[i, j])
    return np.ascontiguousarray(u)


@pytest.mark.parametrize("dim", [2, 3])
def test_undeformed_linear_is_the_linear_step(oracle_mod, dim):
    o, _, _ = _system(oracle_mod, dim)
    rng = np.random.default_rng(3)
    c = np.ascontiguousarray(rng.uniform(0.1, 0.4, o.n))
    flags = np.zeros(o.n, np.uint8)
    flags[rng.random(o.n) < 0.1] = cases.CDIR
    D, dt = 1e-10, 0.5 * o.h ** 2 / 1e-10
    c1, q1, p1 = c.copy(), o.arr(dim, o.n), o.arr(o.n)
    o.diffusion_step(D, dt, 0.4, 3e6, 0.05, c1, q1, p1, flags)
    c2, q2, p2 = c.copy(), o.arr(dim, o.n), o.arr(o.n)
    o.diffusion_step_coupled(D, dt, 0.4, 3e6, 0.05, 0, o.arr(dim, o.n), c2, q2, p2, flags)
    assert np.array_equal(c1, c2) and np.array_equal(q1, q2) and np.array_equal(p1, p2)


@pytest.mark.parametrize("nonlinear", [0, 1])
@pytest.mark.parametrize("dim", [2, 3])
def test_mass_conserved_under_deformation(oracle_mod, dim, nonlinear):
    o, _, _ = _system(oracle_mod, dim)
    rng = np.random.default_rng(4)
    u = _smooth_u(o, dim, 0.03, 7)
    c = np.ascontiguousarray(rng.uniform(0.1, 0.4, o.n))
    q, p = o.arr(dim, o.n), o.arr(o.n)
    D = 1e-10
    mass0 = (o.V * c).sum()
    for _ in range(4):
        o.diffusion_step_coupled(D, 0.5 * o.h ** 2 / D, 0.0, 3e6, 0.0, nonlinear, u, c, q, p)
    assert abs((o.V * c).sum() - mass0) <= 1e-13 * mass0
    assert np.abs(q).max() > 0


@pytest.mark.parametrize("nonlinear", [0, 1])
@pytest.mark.parametrize("dim", [2, 3])
def test_homogeneous_deformation_closed_form(oracle_mod, dim, nonlinear):
    o, X, idx = _system(oracle_mod, dim, jitter=0.1)
    F0 = np.eye(dim) + np.array([[0.08, 0.21, -0.05], [-0.11, -0.06, 0.13], [0.04, 0.17, 0.09]])[:dim, :dim]
    J0 = np.linalg.det(F0)
    Xc = o.X - o.X.mean(axis=1, keepdims=True)
    u = np.ascontiguousarray((F0 - np.eye(dim)) @ Xc)
    alpha = np.array([30.0, -20.0, 12.0])[:dim]
    a = 0.25 + alpha @ Xc                      # saturation, linear in X
    c = np.ascontiguousarray(J0 * a)           # content per reference volume
    q, p = o.arr(dim, o.n), o.arr(o.n)
    D = 1e-10
    o.diffusion_step_coupled(D, 0.0, 0.0, 3e6, 0.0, nonlinear, u, c, q, p)
    Fi = np.linalg.inv(F0)
    w = a if nonlinear else np.ones(o.n)
    want = J0 * (Fi @ (-D * (Fi.T @ alpha)))[:, None] * w[None, :]
    assert np.allclose(q, want, rtol=1e-10, atol=1e-10 * np.abs(want).max())
    # sanity: the transposed inverse would differ
    wrong = J0 * (Fi @ (-D * (Fi @ alpha)))[:, None] * w[None, :]
    assert np.abs(wrong - want).max() > 1e-3 * np.abs(want).max()
    if not nonlinear:
        o2, X2, idx2 = _system(oracle_mod, 2, shape=(18, 18), jitter=0.0)
        F2 = F0[:2, :2] if dim == 2 else np.eye(2) + np.array([[0.08, 0.21], [-0.11, -0.06]])
        J2 = np.linalg.det(F2)
        Xc2 = o2.X - o2.X.mean(axis=1, keepdims=True)
        u2 = np.ascontiguousarray((F2 - np.eye(2)) @ Xc2)
        c2 = np.ascontiguousarray(J2 * (0.25 + alpha[:2] @ Xc2))
        c20 = c2.copy()
        q2, p2 = o2.arr(2, o2.n), o2.arr(o2.n)
        o2.diffusion_step_coupled(D, 0.5 * o2.h ** 2 / D, 0.0, 0.0, 0.0, 0, u2, c2, q2, p2)
        ids = o2.perm
        inner = np.all([(idx2[k][ids] >= 6) & (idx2[k][ids] < 12) for k in range(2)], axis=0)
        assert np.max(np.abs(c2 - c20)[inner]) <= 1e-12 * np.abs(c20).max()


def test_dirichlet_holds_saturation(oracle_mod):
    o, _, _ = _system(oracle_mod, 2)
    rng = np.random.default_rng(8)
    u = _smooth_u(o, 2, 0.03, 9)
    c = np.ascontiguousarray(rng.uniform(0.1, 0.4, o.n))
    flags = np.zeros(o.n, np.uint8)
    flags[rng.random(o.n) < 0.2] = cases.CDIR
    q, p = o.arr(2, o.n), o.arr(o.n)
    o.diffusion_step_coupled(1e-10, 0.5 * o.h ** 2 / 1e-10, 0.4, 3e6, 0.05, 1, u, c, q, p, flags)
    F = o.deformation_gradient(u).T.reshape(-1, 3, 3)
    J = np.linalg.det(F)
    d = flags == cases.CDIR
    assert np.allclose(c[d], 0.4 * J[d], rtol=1e-14)
    assert np.allclose(p[d], 3e6 * (0.4 - 0.05), rtol=1e-12)
    assert np.allclose(p, 3e6 * (c / J - 0.05), rtol=1e-12, atol=1e-6)
