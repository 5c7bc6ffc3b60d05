"""Pins of the oracle's constitutive update (App. A and B of the paper).

* neo-Hookean stress (eq. kirchoff_stress_equation, eq. stress_trans) equals
  the derivative of the stored energy W_v(J) + W_s(bbar) of eqs.
  (energy_volume), (energy_shear), by central finite differences;
* P(I) = 0, objectivity P(QF) = Q P(F), and the small-strain limit equals the
  linear-elastic reading with the moduli of eq. (relation-modulus);
* swelling (App. B.2, eq. fluid_pressure): a free isotropic stretch under
  pressure p has the closed-form volume ratio J = p/K + sqrt((p/K)^2 + 1);
* Algorithm 1: elastic below yield, closed-form radial return for linear
  hardening, consistency on the yield surface, Newton = bisection.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

from paper_2309_04010_amd import cases

E, NU = 2.0e11, 0.3
MU = E / (2 * (1 + NU))
K = E / (3 * (1 - 2 * NU))


@pytest.fixture(scope="module")
def o(oracle_mod):
    X, _ = cases.lattice((3, 3, 3), 1.0)
    return oracle_mod.Oracle(3, X, np.ones(27), 1.3)


def _energy(F):
    J = np.linalg.det(F)
    bbar = J ** (-2.0 / 3.0) * F @ F.T
    return 0.5 * K * (0.5 * (J * J - 1) - np.log(J)) + 0.5 * MU * (np.trace(bbar) - 3.0)


def _rand_F(seed, amp=0.1):
    rng = np.random.default_rng(seed)
    return np.eye(3) + rng.normal(0, amp, (3, 3))


def test_nh_stress_is_energy_derivative(o):
    mat = o.material(cases.NH, E, NU, 1000.0)
    for seed in range(5):
        F = _rand_F(seed)
        _, P, _ = o.constitutive(mat, F)
        G = np.zeros((3, 3))
        for i in range(3):
            for j in range(3):
                e = 1e-6
                Fp, Fm = F.copy(), F.copy()
                Fp[i, j] += e
                Fm[i, j] -= e
                G[i, j] = (_energy(Fp) - _energy(Fm)) / (2 * e)
        assert np.allclose(P, G, rtol=1e-6, atol=1e-6 * np.abs(G).max())


def test_nh_reference_and_objectivity(o):
    mat = o.material(cases.NH, E, NU, 1000.0)
    _, P0, _ = o.constitutive(mat, np.eye(3))
    assert np.abs(P0).max() < 1e-12 * MU
    F = _rand_F(7)
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    Q = Q @ np.array([[1, 0, 0], [0, np.cos(0.3), -np.sin(0.3)], [0, np.sin(0.3), np.cos(0.3)]])
    _, P, _ = o.constitutive(mat, F)
    _, PQ, _ = o.constitutive(mat, Q @ F)
    assert np.allclose(PQ, Q @ P, rtol=1e-12, atol=1e-12 * np.abs(P).max())


@pytest.mark.parametrize("model", [cases.NH, cases.J2])
def test_small_strain_limit_is_linear_elastic(o, model):
    le = o.material(cases.LE, E, NU, 1000.0)
    mat = o.material(model, E, NU, 1000.0, sigma0=1e12, sigma_inf=1e12, delta=1.0)
    rng = np.random.default_rng(3)
    G = rng.normal(0, 1, (3, 3))
    errs = []
    for eps in [1e-4, 5e-5]:
        _, Pn, _ = o.constitutive(mat, np.eye(3) + eps * G)
        _, Pl, _ = o.constitutive(le, np.eye(3) + eps * G)
        errs.append(np.abs(Pn - Pl).max())
        # linear part matches to first order
        assert np.abs(Pn - Pl).max() < 50 * eps * np.abs(Pl).max()
    assert 3.0 < errs[0] / errs[1] < 5.0  # second-order remainder


def test_linear_elastic_plane_strain_uniaxial(o):
    """Homogeneous plane-strain uniaxial stress: with eps_yy = -nu/(1-nu) eps_xx
    the transverse stress vanishes and P_xx = E/(1-nu^2) eps_xx."""
    le = o.material(cases.LE, E, NU, 1000.0)
    e = 1e-4
    F = np.diag([1 + e, 1 - NU / (1 - NU) * e, 1.0])
    _, P, _ = o.constitutive(le, F)
    assert abs(P[1, 1]) < 1e-12 * abs(P[0, 0])
    assert abs(P[0, 0] - E / (1 - NU ** 2) * e) < 1e-12 * abs(P[0, 0])


@pytest.mark.parametrize("model", [cases.NH, cases.J2, cases.LE])
def test_swelling_free_expansion(o, model):
    p = 0.05 * K
    mat = o.material(model, E, NU, 1000.0, sigma0=1e13, sigma_inf=1e13, delta=1.0)

    def res(lam):
        _, P, _ = o.constitutive(mat, lam * np.eye(3), p=p)
        return P[0, 0]
    lam = brentq(res, 0.9, 1.2, xtol=1e-15)
    if model == cases.LE:
        # small-strain reading: 3K (lam - 1) = J p / lam with J = lam^3
        assert abs(K * 3 * (lam - 1) - lam ** 2 * p) < 1e-9 * p
    else:
        J = p / K + np.sqrt((p / K) ** 2 + 1)
        assert abs(lam ** 3 - J) < 1e-12


def test_j2_elastic_below_yield(o):
    nh = o.material(cases.NH, E, NU, 1000.0)
    j2 = o.material(cases.J2, E, NU, 1000.0, sigma0=1e12, sigma_inf=2e12, delta=10.0)
    F = _rand_F(2, 0.01)
    _, Pn, _ = o.constitutive(nh, F)
    rc, Pj, pl = o.constitutive(j2, F)
    assert rc == 0
    assert np.allclose(Pj, Pn, rtol=1e-12, atol=1e-12 * np.abs(Pn).max())
    assert np.allclose(pl, 0.0, atol=1e-13)


def _dev_tau(F, P):
    tau = P @ F.T
    return tau - np.trace(tau) / 3 * np.eye(3)


def test_j2_linear_hardening_closed_form(o):
    """sigma_inf = sigma0: k(a) = s0 + H a, so the return is the closed form
    dgamma = f_trial / (2 mubar + 2H/3)."""
    s0, H = 4.0e8, 2.0e9
    j2 = o.material(cases.J2, E, NU, 1000.0, sigma0=s0, sigma_inf=s0, delta=5.0, H=H)
    F = np.diag([1.01, 0.997, 0.996])
    J = np.linalg.det(F)
    Fb = J ** (-1 / 3) * F
    b = Fb @ Fb.T
    s = MU * (b - np.trace(b) / 3 * np.eye(3))
    ftr = np.linalg.norm(s) - np.sqrt(2 / 3) * s0
    assert ftr > 0
    mubar = MU * np.trace(b) / 3
    dg = ftr / (2 * mubar + 2 * H / 3)
    rc, P, pl = o.constitutive(j2, F)
    assert rc == 0
    assert abs(pl[6] - np.sqrt(2 / 3) * dg) < 1e-12 * pl[6]
    sn = np.linalg.norm(_dev_tau(F, P))
    assert abs(sn - np.sqrt(2 / 3) * (s0 + H * pl[6])) < 1e-10 * sn


def test_j2_nonlinear_consistency_and_bisection(o):
    s0, sinf, dl = 2.0e8, 4.0e8, 16.0
    j2 = o.material(cases.J2, E, NU, 7850.0, sigma0=s0, sigma_inf=sinf, delta=dl)
    k = lambda a: s0 + (sinf - s0) * (1 - np.exp(-dl * a))  # noqa: E731
    pl = np.zeros(7)
    for step in range(1, 6):
        F = np.diag([1 + 0.004 * step, 1 - 0.002 * step, 1 - 0.002 * step])
        F[0, 1] = 0.001 * step
        J = np.linalg.det(F)
        Fb = J ** (-1 / 3) * F
        Xb = np.eye(3) + np.array([[pl[0], pl[3], pl[5]], [pl[3], pl[1], pl[4]], [pl[5], pl[4], pl[2]]])
        b = Fb @ Xb @ Fb.T
        s = MU * (b - np.trace(b) / 3 * np.eye(3))
        sn = np.linalg.norm(s)
        a0 = pl[6]
        rc, P, pl = o.constitutive(j2, F, pl)
        assert rc == 0
        if sn - np.sqrt(2 / 3) * k(a0) > 0:
            mubar = MU * np.trace(b) / 3
            g = lambda x: sn - np.sqrt(2 / 3) * k(a0 + np.sqrt(2 / 3) * x) - 2 * mubar * x  # noqa: E731
            dg = brentq(g, 0.0, sn / (2 * mubar), xtol=1e-18, rtol=1e-15)
            assert abs(pl[6] - (a0 + np.sqrt(2 / 3) * dg)) <= 1e-11 * pl[6]
            snew = np.linalg.norm(_dev_tau(F, P))
            assert abs(snew - np.sqrt(2 / 3) * k(pl[6])) <= 1e-10 * snew
    assert pl[6] > 0


def test_j2_state_update_is_idempotent(o):
    """After a plastic return at F, the updated state Cbar_p^-1 rebuilds the
    returned elastic strain: evaluating again at the same F from that state is
    an elastic step on the yield surface, so the stress repeats and alpha does
    not grow (App. A.4: the state update closes Algorithm 1).  A transposed or
    mis-signed state update fails this."""
    s0, sinf, dl = 2.0e8, 4.0e8, 16.0
    j2 = o.material(cases.J2, E, NU, 7850.0, sigma0=s0, sigma_inf=sinf, delta=dl)
    rng = np.random.default_rng(4)
    for _ in range(5):
        F = np.eye(3) + rng.normal(0.0, 6e-3, (3, 3))
        rc, P1, pl1 = o.constitutive(j2, F)
        assert rc == 0 and pl1[6] > 0.0          # the first call yields
        rc, P2, pl2 = o.constitutive(j2, F, pl1)
        assert rc == 0
        assert np.abs(P2 - P1).max() <= 1e-9 * np.abs(P1).max()
        assert abs(pl2[6] - pl1[6]) <= 1e-9 * pl1[6]
        assert np.abs(pl2[:6] - pl1[:6]).max() <= 1e-9 * max(np.abs(pl1[:6]).max(), 1e-12)
