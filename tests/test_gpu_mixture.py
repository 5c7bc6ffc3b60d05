"""GPU parity of the mixture momentum (Sec. 2.2.1, Sec. 3.2; material
rho_l0 > 0) against the oracle.

* one solid stage (2D/3D, FP64/FP32, NH and J2), from random displacement,
  velocity, content (some particles dry) and reference flux, with fixed
  particles: PB (with the fluid's momentum flux), the momentum sum per unit
  mixture mass and the kick;
* the damping sweep with the mixture masses, and drift + kinetic energy;
* multi-time-step runs: the swelling strip with the two-way coupled
  nonlinear diffusion slow step and the mixture momentum in the fast loop,
  FP64 within 1e-10 (fixed counts and the adaptive stop) and FP32 within
  1e-4;
* argument checks: rho_l0 < 0, or a mixture without c and q, is SPH_E_ARG;
  the reverse pass and the whole-run graph refuse a mixture.
"""
import numpy as np
import pytest

from paper_2309_04010_amd import binding as B
from paper_2309_04010_amd import cases

from .parity_util import TOL, build_pair, dev, host, jittered, rel_err, torch_dtype

pytestmark = pytest.mark.gpu

RHO_L0 = 1000.0
MATS = {
    "NH": dict(model=cases.NH, E=1.0e8, nu=0.4, rho0=2000.0, C_swell=3.0e6, c0=0.0, rho_l0=RHO_L0),
    "J2": dict(model=cases.J2, E=2.0e11, nu=0.29, rho0=7850.0, sigma0=2.0e8, sigma_inf=4.0e8,
               delta=16.0, rho_l0=RHO_L0),
}


def _rounded(a, prec):
    return a.astype(np.float32).astype(np.float64) if prec == B.SPH_F32 else a


def _setup(oracle_mod, dim, prec, model, seed):
    shape = (37, 23) if dim == 2 else (13, 9, 7)
    X, V, h = jittered(shape, jitter=0.1, seed=seed)
    o, nb = build_pair(oracle_mod, dim, X, V, h)
    rng = np.random.default_rng(seed)
    amp = 2e-2 if model == "J2" else 5e-3
    u = np.ascontiguousarray(amp * 1e-3 * rng.normal(0, 1, (dim, o.n)) +
                             amp * np.diag(rng.normal(0, 1, dim)) @ o.X)
    v = _rounded(np.ascontiguousarray(rng.normal(0, 1.0, (dim, o.n))), prec)
    c = rng.uniform(0.05, 0.5, o.n)
    c[rng.random(o.n) < 0.1] = 0.0                       # dry particles: no relative velocity
    c = _rounded(np.ascontiguousarray(c), prec)
    # a flux large enough that the fluid's momentum flux is of the order of
    # the stress, so that the comparison sees it
    qs = 1.0e3 if model == "J2" else 30.0
    q = _rounded(np.ascontiguousarray(rng.normal(0, qs, (dim, o.n))), prec)
    p = _rounded(np.ascontiguousarray(rng.uniform(0, 1e6, o.n)), prec) if model == "NH" else None
    flags = np.zeros(o.n, np.uint8)
    flags[rng.random(o.n) < 0.1] = cases.FIXED
    T = torch_dtype(prec)
    st = B.new_state(nb, prec, with_plastic=(model == "J2"), with_diffusion=True, with_acc=True)
    st.u.copy_(dev(u))
    st.v.copy_(dev(v, T))
    st.c.copy_(dev(c, T))
    st.q.copy_(dev(q, T))
    if p is not None:
        st.p.copy_(dev(p, T))
    st.flags = dev(flags)
    return o, nb, st, dict(u=u, v=v, c=c, q=q, p=p, flags=flags)


@pytest.mark.parametrize("prec", [B.SPH_F64, B.SPH_F32], ids=["f64", "f32"])
@pytest.mark.parametrize("model", list(MATS))
@pytest.mark.parametrize("dim", [2, 3])
def test_solid_stage_mixture(oracle_mod, dim, model, prec):
    print(f"[mixture] solid dim={dim} model={model} prec={prec}", flush=True)
    o, nb, st, f = _setup(oracle_mod, dim, prec, model, seed=20 + dim)
    kw = MATS[model]
    mo, mg = o.material(**kw), B.material(**kw)
    pl = np.zeros((7, o.n))
    vo = f["v"].copy()
    dt = 1e-7
    for _ in range(2):
        rc, PBo, acco = o.solid_step(mo, dt, f["u"], vo, plastic=pl if model == "J2" else None,
                                     p=f["p"], flags=f["flags"], c=f["c"], q=f["q"])
        assert rc == 0
        B.sph_solid_relax_step(nb, mg, st, dt)
    tol = TOL[prec]
    assert rel_err(host(st.PB), PBo) < tol
    assert rel_err(host(st.acc), acco) < tol
    assert rel_err(host(st.v) - f["v"], vo - f["v"]) < tol
    # the fluid terms matter in this case
    _, PBd, _ = o.solid_step(o.material(**dict(kw, rho_l0=0.0)), dt, f["u"], f["v"].copy(),
                             plastic=np.zeros((7, o.n)) if model == "J2" else None, p=f["p"],
                             flags=f["flags"])
    assert rel_err(PBd, PBo) > 0.05
    nb.close()


@pytest.mark.parametrize("prec", [B.SPH_F64, B.SPH_F32], ids=["f64", "f32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_damping_and_drift_mixture(oracle_mod, dim, prec):
    print(f"[mixture] damping+drift dim={dim} prec={prec}", flush=True)
    o, nb, st, f = _setup(oracle_mod, dim, prec, "NH", seed=30 + dim)
    kw = MATS["NH"]
    mg = B.material(**kw)
    eta, dt = 50.0, 1e-6
    w = f["v"].copy()
    o.damping_sweep(kw["rho0"], eta, dt, w, f["flags"], rho_l0=RHO_L0, c=f["c"])
    B.sph_damping_sweep(nb, mg, st, eta, dt)
    tol = TOL[prec]
    assert rel_err(host(st.v) - f["v"], w - f["v"]) < tol
    wd = f["v"].copy()
    o.damping_sweep(kw["rho0"], eta, dt, wd, f["flags"])
    assert rel_err(wd - f["v"], w - f["v"]) > 100 * tol       # the masses matter
    import torch
    v2 = host(st.v)
    uo = f["u"].copy()
    keo = o.drift_ke(kw["rho0"], dt, uo, np.ascontiguousarray(v2), f["flags"], rho_l0=RHO_L0, c=f["c"])
    ked = torch.zeros(1, dtype=torch.float64, device="cuda")
    B.sph_drift_ke(nb, mg, st, dt, ke_out=ked)
    assert rel_err(host(st.u) - f["u"], uo - f["u"]) < tol
    assert abs(ked.item() - keo) <= 1e-12 * keo
    nb.close()


def _strip_run(oracle_mod, prec, run_over, rho_l0=RHO_L0):
    c = cases.strip2d(nx=40, ny=8, n_slow=3, fixed_inner=40, k_max=0)
    o, nb = build_pair(oracle_mod, 2, c.X, c.V, c.h)
    perm = o.perm
    flags = np.ascontiguousarray(c.flags[perm])
    run = dict(c.run, slow_kind=cases.DIFFUSION_COUPLED)
    run.update(run_over)
    kw = dict(c.material, rho_l0=rho_l0)
    T = torch_dtype(prec)
    st = B.new_state(nb, prec, with_diffusion=True)
    st.flags = dev(flags)
    c0 = _rounded(np.ascontiguousarray(c.c_init[perm]), prec)
    st.c.copy_(dev(c0, T))
    rc_g, k_g, _, _, _ = B.sph_advance_multirate(nb, B.material(**kw), st,
                                                 B.multirate_cfg(**run, diff_nonlinear=1))
    uo, vo = o.arr(2, c.n), o.arr(2, c.n)
    co = c0.copy()
    qo, po = o.arr(2, c.n), o.arr(c.n)
    rc_o, k_o, _, _ = o.advance(o.material(**kw), o.cfg(**run, nonlinear=1), uo, vo, c=co, q=qo, p=po,
                                flags=flags)
    out = dict(k=(k_o, k_g), u=(uo, host(st.u)), v=(vo, host(st.v)), c=(co, host(st.c)),
               q=(qo, host(st.q)))
    nb.close()
    return out


@pytest.mark.parametrize("prec", [B.SPH_F64, B.SPH_F32], ids=["f64", "f32"])
def test_mixture_multirate_fixed_counts(oracle_mod, prec):
    print(f"[mixture] strip run prec={prec}", flush=True)
    r = _strip_run(oracle_mod, prec, {})
    tol = TOL[prec]
    assert np.array_equal(r["k"][0], r["k"][1])
    assert np.abs(r["u"][0]).max() > 0 and np.abs(r["q"][0]).max() > 0
    for key in ("u", "c", "q"):
        assert rel_err(r[key][1], r[key][0]) < tol, key
    assert rel_err(r["v"][1], r["v"][0]) < (tol if prec == B.SPH_F64 else 1e-3)


def test_mixture_multirate_adaptive_counts(oracle_mod):
    # the kinetic energy, with the mixture masses, decides the inner counts
    r = _strip_run(oracle_mod, B.SPH_F64, dict(fixed_inner=0, k_max=2000))
    assert np.array_equal(r["k"][0], r["k"][1]), r["k"]
    assert np.all(r["k"][0] > 1)
    assert rel_err(r["u"][1], r["u"][0]) < 1e-10
    assert rel_err(r["c"][1], r["c"][0]) < 1e-10


def test_mixture_argument_checks(oracle_mod):
    from paper_2309_04010_amd import adjoint as A
    X, V, h = jittered((12, 9), jitter=0.1, seed=1)
    o, nb = build_pair(oracle_mod, 2, X, V, h)
    st = B.new_state(nb, B.SPH_F64)
    for bad, code in ((dict(MATS["NH"], rho_l0=-1.0), B.SPH_E_ARG), (MATS["NH"], B.SPH_E_ARG)):
        with pytest.raises(B.SphError) as e:
            B.sph_solid_relax_step(nb, B.material(**bad), st, 1e-7)
        assert e.value.code == code
    nb.close()
    c = cases.strip2d(nx=20, ny=6, n_slow=2, fixed_inner=5, k_max=0)
    c.material["rho_l0"] = RHO_L0
    pr = A.MultirateProblem(c, B.SPH_F64)
    th = pr.theta0()
    pr.forward(th)
    with pytest.raises(B.SphError) as e:
        pr.backward(dev(np.ones((2, c.n))))
    assert e.value.code == B.SPH_E_UNSUPPORTED
    with pytest.raises(B.SphError) as e:
        B.sph_advance_multirate_graph(pr.nb, pr._material(th), pr.st, B.multirate_cfg(**pr.run))
    assert e.value.code == B.SPH_E_UNSUPPORTED
    pr.close()
