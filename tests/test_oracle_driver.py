"""End-to-end pins of the oracle's multi-time-step driver (Sec. 4.2).

* small-strain bar against its analytic elastic solution: grips that follow
  the homogeneous plane-strain uniaxial field (6 layers, so that every free
  particle and all its neighbours have full support) leave that affine field as
  the exact discrete equilibrium; damped relaxation must reach it, with
  P_xx = E/(1 - nu^2) eps and P_yy = 0;
* the kinetic-energy early exit: each slow step stops at the first inner step
  whose E_k is at or below the threshold, and the counts are recorded;
* kinetic energy decays monotonically once the load is applied (damping);
* complex-step derivatives of the oracle equal central finite differences
  (this pins the derivative oracle used for gradient parity), for E, C and D
  on a swelling strip, and for E and the hardening law's sigma0, sigma_inf,
  delta and H through Algorithm 1's return mapping on a J2 bar driven far
  into the plastic range;
* the fast step of Sec. 4.1 (eq. dts-advection at rest) is a stable explicit
  step and within a factor 2 of the stability limit: an undamped elastic
  lattice keeps its energy at dt_s and blows up at 2 dt_s.
"""
import numpy as np
import pytest

from paper_2309_04010_amd import cases


def _setup(oracle_mod, case, complex_step=False):
    o = oracle_mod.Oracle(case.dim, case.X, case.V, case.h, complex_step=complex_step)
    perm = o.perm
    flags = np.ascontiguousarray(case.flags[perm])
    vgrip = None if case.vgrip is None else np.ascontiguousarray(case.vgrip[:, perm].astype(o.dtype))
    return o, flags, vgrip


def test_bar_converges_to_analytic_elastic_solution(oracle_mod):
    nx, ny = 18, 6
    c = cases.bar2d(nx=nx, ny=ny, affine=True, n_slow=1, grip_layers=6)
    o, flags, vgrip = _setup(oracle_mod, c)
    mat = o.material(**c.material)
    cfg = o.cfg(**dict(c.run, fixed_inner=20000))
    u, v = o.arr(2, o.n), o.arr(2, o.n)
    rc, k, ke, conv = o.advance(mat, cfg, u, v, vgrip=vgrip, flags=flags)
    assert rc == 0 and k[0] == 20000
    E, nu = c.material["E"], c.material["nu"]
    eps = c.observable["erate"] * c.run["dt_slow"]
    L, W = nx * c.dp, ny * c.dp
    ua = np.vstack([eps * (o.X[0] - 0.5 * L), -nu / (1 - nu) * eps * (o.X[1] - 0.5 * W)])
    assert np.abs(u - ua).max() <= 1e-6 * np.abs(ua).max()
    H9 = o.displacement_gradient(u)
    _, P9, _ = o.stress(mat, H9)
    sxx = E / (1 - nu * nu) * eps
    assert np.abs(P9[0] - sxx).max() <= 1e-6 * sxx
    assert np.abs(P9[4]).max() <= 1e-6 * sxx


def test_ke_early_exit_and_counts(oracle_mod):
    c = cases.bar2d(n_slow=3)
    o, flags, vgrip = _setup(oracle_mod, c)
    mat = o.material(**c.material)
    cfg = o.cfg(**c.run)
    u, v = o.arr(2, o.n), o.arr(2, o.n)
    rc, k, ke, conv = o.advance(mat, cfg, u, v, vgrip=vgrip, flags=flags)
    assert rc == 0 and np.all(conv == 1)
    assert np.all(ke <= c.run["ke_tol"]) and np.all(k > 10)
    # rerunning with the recorded counts frozen gives the same state, and one
    # step fewer in the first slow step ends above the threshold
    u2, v2 = o.arr(2, o.n), o.arr(2, o.n)
    rc2, k2, ke2, _ = o.advance(mat, cfg, u2, v2, vgrip=vgrip, flags=flags, k_sched=k)
    assert np.array_equal(k2, k) and np.array_equal(u2, u)
    cfg1 = o.cfg(**dict(c.run, n_slow=1))
    u3, v3 = o.arr(2, o.n), o.arr(2, o.n)
    _, _, ke3, _ = o.advance(mat, cfg1, u3, v3, vgrip=vgrip, flags=flags, k_sched=[k[0] - 1])
    assert ke3[0] > c.run["ke_tol"]
    # cap reached: warning code 1 and not converged
    cfg_cap = o.cfg(**dict(c.run, n_slow=1, k_max=5))
    u4, v4 = o.arr(2, o.n), o.arr(2, o.n)
    rc4, k4, _, conv4 = o.advance(mat, cfg_cap, u4, v4, vgrip=vgrip, flags=flags)
    assert rc4 == 1 and k4[0] == 5 and conv4[0] == 0


def test_kinetic_energy_decays_after_load(oracle_mod):
    c = cases.bar2d(n_slow=1)
    o, flags, vgrip = _setup(oracle_mod, c)
    mat = o.material(**c.material)
    u, v = o.arr(2, o.n), o.arr(2, o.n)
    o.load_step(c.run["dt_slow"], u, vgrip, flags)
    K = c.material["E"] / (3 * (1 - 2 * c.material["nu"]))
    dt = 0.6 * c.h / np.sqrt(K / c.material["rho0"])
    kes = []
    for _ in range(3000):
        o.solid_step(mat, dt, u, v, flags=flags)
        o.damping_sweep(c.material["rho0"], c.run["eta"], dt, v, flags)
        kes.append(o.drift_ke(c.material["rho0"], dt, u, v, flags))
    kes = np.array(kes)
    # envelope decays: each block of 300 steps has a lower maximum
    blocks = kes[300:].reshape(9, 300).max(axis=1)
    assert np.all(np.diff(blocks) < 0)
    assert kes[-1] < 1e-3 * kes.max()


def _strip_case():
    return cases.strip2d(nx=24, ny=6, n_slow=2, fixed_inner=30, k_max=0)


@pytest.mark.parametrize("param", ["E", "C_swell", "D"])
def test_complex_step_matches_finite_differences(oracle_mod, param):
    c = _strip_case()

    def run(complex_step, pert):
        o, flags, _ = _setup(oracle_mod, c, complex_step)
        mat_kw = dict(c.material)
        run_kw = dict(c.run)
        K = c.material["E"] / (3 * (1 - 2 * c.material["nu"]))
        run_kw["dt_s"] = 0.6 * c.h / np.sqrt(K / c.material["rho0"])   # frozen
        run_kw["dt_slow"] = 0.5 * c.h ** 2 / c.run["D"]                 # frozen
        if param == "D":
            run_kw["D"] = run_kw["D"] + pert
        else:
            mat_kw[param] = mat_kw[param] + pert
        mat = o.material(**mat_kw)
        cfg = o.cfg(**run_kw)
        u, v = o.arr(2, o.n), o.arr(2, o.n)
        cc = np.ascontiguousarray(c.c_init[o.perm].astype(o.dtype))
        q, p = o.arr(2, o.n), o.arr(o.n)
        rc, k, _, _ = o.advance(mat, cfg, u, v, c=cc, q=q, p=p, flags=flags)
        assert rc in (0, 1)
        return u[1].sum()   # a smooth observable: total transverse displacement
    base = {"E": c.material["E"], "C_swell": c.material["C_swell"], "D": c.run["D"]}[param]
    h = 1e-20 * base
    d_cs = run(True, 1j * h).imag / h
    e = 1e-5 * base
    d_fd = (run(False, e) - run(False, -e)) / (2 * e)
    assert d_cs != 0.0
    assert abs(d_cs - d_fd) <= 1e-5 * abs(d_cs)


def _j2_bar():
    """A small J2 bar (App. A.3 hardening with the necking table's linear term
    H, so that every hardening parameter acts) whose grips jump far enough in
    two load steps that most particles yield."""
    c = cases.neck3d(nx=12, ny=5, nz=5, n_slow=2, fixed_inner=25, total_stretch=1.2e-4)
    c.material["H"] = cases.NECK_TABLE["H"]
    return c


@pytest.mark.parametrize("param", ["E", "sigma0", "sigma_inf", "delta", "H"])
def test_complex_step_j2_matches_finite_differences(oracle_mod, param):
    """d<w, u_final>/d(param) through the J2 return mapping (App. A.4,
    Algorithm 1): the complex-step oracle (its Newton solve for the plastic
    multiplier takes one more step once the real part has converged, so that
    the derivative part converges too) against central differences of the
    real oracle, with the step sizes frozen at their nominal values."""
    c = _j2_bar()
    w = np.random.default_rng(11).normal(0.0, 1.0, (3, c.n))
    o0, _, _ = _setup(oracle_mod, c)
    dt_s, _ = o0.default_steps(o0.material(**c.material))

    def run(complex_step, pert):
        o, flags, vgrip = _setup(oracle_mod, c, complex_step)
        mat_kw = dict(c.material)
        mat_kw[param] = mat_kw[param] + pert
        cfg = o.cfg(**dict(c.run, dt_s=dt_s))
        u, v, pl = o.arr(3, o.n), o.arr(3, o.n), o.arr(7, o.n)
        rc, k, _, _ = o.advance(o.material(**mat_kw), cfg, u, v, plastic=pl, vgrip=vgrip, flags=flags)
        assert rc in (0, 1)
        return (w * u).sum(), pl
    base = c.material[param]
    val, pl = run(False, 0.0)
    alpha = pl[6].real
    # driven into the plastic range: most particles yield, up to ~10% strain
    assert (alpha > 0).mean() > 0.5 and alpha.max() > 0.05
    hcs = 1e-20 * base
    d_cs = run(True, 1j * hcs)[0].imag / hcs
    e = 1e-5 * base
    d_fd = (run(False, e)[0] - run(False, -e)[0]) / (2 * e)
    assert d_cs != 0.0
    assert abs(d_cs - d_fd) <= 1e-5 * abs(d_cs), (d_cs, d_fd)


@pytest.mark.parametrize("name", ["bar2d", "cube3d"])
def test_fast_step_is_stable_and_near_the_limit(oracle_mod, name):
    """Sec. 4.1's fast step at rest, 0.6 h / sqrt(K / rho0): symplectic Euler
    on an undamped free lattice (LE in 2D, NH in 3D) from random velocities
    keeps its kinetic energy bounded at dt_s and diverges at 2 dt_s (a step
    off by a factor 2 either way, e.g. c_s from E instead of K or a missing
    factor, fails one side)."""
    if name == "bar2d":
        c = cases.bar2d(nx=16, ny=8)
        m = dict(c.material)
    else:
        c = cases.neck3d(nx=8, ny=6, nz=6)
        m = dict(c.material, model=cases.NH)
    o = oracle_mod.Oracle(c.dim, c.X, c.V, c.h)
    mat = o.material(**m)
    dt_s, dt_d = o.default_steps(mat)
    assert dt_s > 0.0 and dt_d == 0.0
    flags = np.zeros(o.n, np.uint8)

    def ke_growth(dt):
        v = np.random.default_rng(1).normal(0.0, 1e-3, (c.dim, o.n))
        u = np.zeros((c.dim, o.n))
        o.solid_step(mat, dt, u, v, flags=flags)
        e0 = o.drift_ke(m["rho0"], dt, u, v, flags)
        for _ in range(400):
            o.solid_step(mat, dt, u, v, flags=flags)
            e = o.drift_ke(m["rho0"], dt, u, v, flags)
        return e / e0
    with np.errstate(all="ignore"):
        assert ke_growth(dt_s) < 2.0
        g = ke_growth(2.0 * dt_s)
    assert not np.isfinite(g) or g > 1e6
