"""Two-way coupled diffusion step on the GPU against the oracle.

* the step (deformation pass, flux, divergence) on a deformed jittered body,
  2D and 3D, FP64 (1e-10) and FP32 (1e-4), linear and nonlinear flux, with
  Dirichlet particles, over three steps: content c, reference flux Q and
  pressure p;
* undeformed with the linear flux it is the linear step (1e-14);
* a multi-time-step run with coupled slow steps equals the oracle's run;
* the reverse pass refuses the coupled slow kind.
"""
import numpy as np
import pytest

from paper_2309_04010_amd import binding as B
from paper_2309_04010_amd import cases

from .parity_util import TOL, build_pair, dev, host, jittered, rel_err, torch_dtype

pytestmark = pytest.mark.gpu

NH = dict(model=cases.NH, E=1.0e8, nu=0.4, rho0=2000.0, C_swell=3.0e6, c0=0.05)


def _system(oracle_mod, dim, seed):
    shape = (37, 23) if dim == 2 else (13, 9, 7)
    X, V, h = jittered(shape, jitter=0.1, seed=seed)
    return build_pair(oracle_mod, dim, X, V, h)


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


@pytest.mark.parametrize("nonlinear", [0, 1], ids=["linear", "nonlinear"])
@pytest.mark.parametrize("prec", [B.SPH_F64, B.SPH_F32], ids=["f64", "f32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_coupled_step_matches_oracle(oracle_mod, dim, prec, nonlinear):
    print(f"[coupled diffusion] dim={dim} prec={prec} nonlinear={nonlinear}", flush=True)
    rng = np.random.default_rng(50 + dim)
    o, nb = _system(oracle_mod, dim, seed=13)
    mo, mg = o.material(**NH), B.material(**NH)
    u = _smooth_u(o, dim, 0.02, 5 + dim)
    c = np.ascontiguousarray(rng.uniform(0.1, 0.4, o.n))
    flags = np.zeros(o.n, np.uint8)
    flags[rng.random(o.n) < 0.05] = cases.CDIR
    T = torch_dtype(prec)
    st = B.new_state(nb, prec, with_diffusion=True)
    st.u.copy_(dev(u))
    st.c.copy_(dev(c, T))
    st.flags = dev(flags)
    D = 1e-10
    dt = 0.5 * o.h ** 2 / D
    co, qo, po = c.copy(), o.arr(dim, o.n), o.arr(o.n)
    for _ in range(3):
        o.diffusion_step_coupled(D, dt, 0.4, NH["C_swell"], NH["c0"], nonlinear, u, co, qo, po, flags)
        B.sph_diffusion_step_coupled(nb, mg, st, D, dt, 0.4, nonlinear)
    tol = TOL[prec]
    assert rel_err(host(st.c), co) < tol
    assert rel_err(host(st.q), qo) < tol
    assert rel_err(host(st.p), po) < tol
    assert np.abs(qo).max() > 0
    nb.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_undeformed_linear_is_the_linear_step(oracle_mod, dim):
    rng = np.random.default_rng(60 + dim)
    o, nb = _system(oracle_mod, dim, seed=17)
    mg = B.material(**NH)
    c = rng.uniform(0.1, 0.4, o.n)
    flags = np.zeros(o.n, np.uint8)
    flags[rng.random(o.n) < 0.05] = cases.CDIR
    out = []
    for coupled in (False, True):
        st = B.new_state(nb, B.SPH_F64, with_diffusion=True)
        st.c.copy_(dev(c))
        st.flags = dev(flags)
        D = 1e-10
        dt = 0.5 * o.h ** 2 / D
        for _ in range(2):
            if coupled:
                B.sph_diffusion_step_coupled(nb, mg, st, D, dt, 0.4, 0)
            else:
                B.sph_diffusion_step(nb, mg, st, D, dt, 0.4)
        out.append((host(st.c), host(st.q), host(st.p)))
    for a, b in zip(*out):
        assert rel_err(b, a) < 1e-14
    nb.close()


@pytest.mark.parametrize("nonlinear", [0, 1], ids=["linear", "nonlinear"])
def test_coupled_multirate_run_matches_oracle(oracle_mod, nonlinear):
    c = cases.strip2d(nx=40, ny=8, n_slow=3, fixed_inner=30, k_max=0)
    o, nb = build_pair(oracle_mod, 2, c.X, c.V, c.h)
    perm = o.perm
    flags = np.ascontiguousarray(c.flags[perm])
    run = dict(c.run, slow_kind=cases.DIFFUSION_COUPLED)
    st = B.new_state(nb, B.SPH_F64, with_diffusion=True)
    st.flags = dev(flags)
    st.c.copy_(dev(c.c_init[perm]))
    B.sph_advance_multirate(nb, B.material(**c.material), st,
                            B.multirate_cfg(**run, diff_nonlinear=nonlinear))
    uo, vo = o.arr(2, c.n), o.arr(2, c.n)
    co = np.ascontiguousarray(c.c_init[perm])
    qo, po = o.arr(2, c.n), o.arr(c.n)
    rc, k, _, _ = o.advance(o.material(**c.material), o.cfg(**run, nonlinear=nonlinear), uo, vo, c=co,
                            q=qo, p=po, flags=flags)
    assert rc in (0, 1) and np.all(k == run["fixed_inner"])
    assert np.abs(uo).max() > 0
    assert rel_err(host(st.u), uo) < 1e-10
    assert rel_err(host(st.c), co) < 1e-10
    nb.close()


def test_reverse_pass_refuses_coupled(oracle_mod):
    from paper_2309_04010_amd import adjoint as A
    c = cases.strip2d(nx=20, ny=6, n_slow=2, fixed_inner=5, k_max=0)
    pr = A.MultirateProblem(c, B.SPH_F64)
    th = pr.theta0()
    pr.run["slow_kind"] = cases.DIFFUSION_COUPLED
    pr.forward(th)
    w = dev(np.ones((2, c.n)))
    with pytest.raises(B.SphError) as e:
        pr.backward(w)
    assert e.value.code == B.SPH_E_UNSUPPORTED
    pr.close()
