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
  (this pins the derivative oracle used for gradient parity).
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
