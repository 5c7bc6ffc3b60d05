"""Two-way coupled diffusion step on the GPU against the oracle.

* the step (deformation pass, flux, divergence) on a deformed jittered body,
  2D and 3D, FP64 (1e-10) and FP32 (1e-4), linear and nonlinear flux, with
  Dirichlet particles, over three steps: content c, reference flux Q and
  pressure p;
* undeformed with the linear flux it is the linear step (1e-14);
* a multi-time-step run with coupled slow steps equals the oracle's run;
* the reverse pass through coupled slow steps gives the complex-step
  oracle's gradients (2D and 3D, linear and nonlinear flux, FP64 and FP32),
  also with slow steps that take no inner step; a batched coupled run's
  reverse is refused;
* the single-step reverse (sph_diffusion_step_coupled_vjp) against
  complex-step derivatives of the oracle's step, in c, u, D and C.
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


@pytest.mark.parametrize("nonlinear", [0, 1], ids=["linear", "nonlinear"])
@pytest.mark.parametrize("prec", [B.SPH_F64, B.SPH_F32], ids=["f64", "f32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_coupled_vjp_is_transpose(oracle_mod, dim, prec, nonlinear):
    """sph_diffusion_step_coupled_vjp against complex-step derivatives of the
    oracle's coupled step, for L = <c_bar, c'> + <p_bar, p'>: the adjoints of
    c and u (through F, J and F^-1) and the D and C gradients (FP64 1e-9,
    FP32 2e-3); a batched neighbourhood is refused."""
    print(f"[coupled diffusion] vjp dim={dim} prec={prec} nonlinear={nonlinear}", flush=True)
    rng = np.random.default_rng(70 + dim)
    X, V, h = jittered((37, 23) if dim == 2 else (13, 9, 7), jitter=0.1, seed=13)
    o, nb = build_pair(oracle_mod, dim, X, V, h)
    oc = oracle_mod.Oracle(dim, X, V, h, complex_step=True)
    assert np.array_equal(oc.perm, o.perm)
    n = o.n
    T = torch_dtype(prec)
    u = _smooth_u(o, dim, 0.02, 5 + dim)
    c0 = rng.uniform(0.1, 0.4, n)
    cb = rng.normal(0.0, 1.0, n)
    pbv = rng.normal(0.0, 1e-6, n)
    if prec == B.SPH_F32:
        c0, cb = (x.astype(np.float32).astype(np.float64) for x in (c0, cb))
    flags = np.zeros(n, np.uint8)
    flags[rng.random(n) < 0.05] = cases.CDIR
    D, c_bc = 1e-10, 0.4
    dt = 0.5 * o.h ** 2 / D
    mat = B.material(**NH)
    st = B.new_state(nb, prec, with_diffusion=True)
    st.u.copy_(dev(u))
    st.c.copy_(dev(c0, T))
    st.flags = dev(flags)
    c_before = st.c.clone()
    B.sph_diffusion_step_coupled(nb, mat, st, D, dt, c_bc, nonlinear)
    adj = B.new_adjoint(nb, prec, with_diffusion=True)
    adj.c.copy_(dev(cb, T))
    adj.p.copy_(dev(pbv))
    B.sph_diffusion_step_coupled_vjp(nb, mat, st, c_before, adj, D, dt, c_bc, nonlinear)
    cbar, ubar, grad = host(adj.c), host(adj.u), host(adj.grad)
    assert np.all(host(adj.p) == 0.0)

    def L(cc=c0, uu=u, Dv=D, C=NH["C_swell"]):
        x = np.ascontiguousarray(cc, dtype=complex).copy()
        q, p = oc.arr(dim, n), oc.arr(n)
        oc.diffusion_step_coupled(Dv, dt, c_bc, C, NH["c0"], nonlinear,
                                  np.ascontiguousarray(uu, dtype=complex), x, q, p, flags)
        return (cb * x).sum() + (pbv * p).sum()

    eps = 1e-30
    tol = 1e-9 if prec == B.SPH_F64 else 2e-3

    def close(got, want, what):
        assert abs(got - want) <= tol * abs(want), (what, got, want)

    dc = rng.normal(0.0, 1.0, n)
    du = rng.normal(0.0, 1e-3 * np.abs(u).max(), (dim, n))
    close((cbar * dc).sum(), L(cc=c0 + 1j * eps * dc).imag / eps, "c")
    want_u = L(uu=u + 1j * eps * du).imag / eps
    assert abs(want_u) > 1e-6 * abs(L().real)            # the step does depend on u
    close((ubar * du).sum(), want_u, "u")
    close(grad[B.GRAD_NAMES.index("D")], L(Dv=D + 1j * eps * D).imag / (eps * D), "D")
    C = NH["C_swell"]
    close(grad[B.GRAD_NAMES.index("C_swell")], L(C=C + 1j * eps * C).imag / (eps * C), "C_swell")
    nb.close()


def _coupled_case(name, nonlinear):
    if name == "strip2d":
        c = cases.strip2d(nx=24, ny=6, n_slow=3, fixed_inner=20, k_max=0)
    else:
        c = cases.plate3d(nx=14, ny=14, n_slow=2, fixed_inner=15)
    c.run["slow_kind"] = cases.DIFFUSION_COUPLED
    c.run["diff_nonlinear"] = nonlinear
    return c


def _oracle_coupled_objective(oracle_mod, c, run, k_sched, w, param, eps_rel=1e-20):
    """d<w, u_final>/d(param) of the coupled run by the complex-step oracle."""
    d, n = c.dim, c.n
    o = oracle_mod.Oracle(d, c.X, c.V, c.h, complex_step=True)
    perm = o.perm
    flags = np.ascontiguousarray(c.flags[perm])
    m, r = dict(c.material), dict(run)
    nonlinear = r.pop("diff_nonlinear")
    base = r["D"] if param == "D" else m[param]
    e = eps_rel * max(abs(base), 1.0)
    if param == "D":
        r["D"] = base + 1j * e
    else:
        m[param] = base + 1j * e
    cfg = o.cfg(**{k: v for k, v in r.items() if k != "D"}, D=r["D"], nonlinear=nonlinear)
    u, v = o.arr(d, n), o.arr(d, n)
    cc = np.ascontiguousarray(c.c_init[perm], dtype=complex)
    q, p = o.arr(d, n), o.arr(n)
    rc, k, _, _ = o.advance(o.material(**m), cfg, u, v, c=cc, q=q, p=p, flags=flags, k_sched=k_sched)
    assert rc in (0, 1) and np.array_equal(k, k_sched)
    return (w * u).sum().imag / e


@pytest.mark.parametrize("prec", [B.SPH_F64, B.SPH_F32], ids=["f64", "f32"])
@pytest.mark.parametrize("nonlinear", [0, 1], ids=["linear", "nonlinear"])
@pytest.mark.parametrize("name", ["strip2d", "plate3d"])
def test_coupled_gradient_matches_oracle(oracle_mod, name, nonlinear, prec):
    """Reverse pass through two-way coupled slow steps: the gradient of
    <w, u_final> with respect to E, D and C against the complex-step oracle
    (FP64 1e-8, FP32 1e-2); the u-dependence of the coupled step (through F,
    J and F^-1) carries the gradient from one slow step to the previous."""
    from paper_2309_04010_amd import adjoint as A
    print(f"[coupled] gradient {name} nonlinear={nonlinear} prec={prec}", flush=True)
    c = _coupled_case(name, nonlinear)
    pr = A.MultirateProblem(c, prec, k_hist=c.run["fixed_inner"])
    pr.forward(pr.theta0())
    pr.freeze()
    w = np.random.default_rng(6).normal(0.0, 1.0, (c.dim, c.n))
    pr.forward(pr.theta0())
    assert np.abs(host(pr.st.u)).max() > 0
    g = host(pr.backward(dev(w)))
    tol = 1e-8 if prec == B.SPH_F64 else 1e-2
    for nm in ("E", "D", "C_swell"):
        want = _oracle_coupled_objective(oracle_mod, c, pr.run, pr.k_sched, w, nm)
        gi = B.GRAD_NAMES.index(nm)
        print(f"  d/d{nm}: gpu {g[gi]:.10e} oracle {want:.10e}", flush=True)
        assert abs(g[gi] - want) <= tol * abs(want), (nm, g[gi], want)
    pr.close()


@pytest.mark.parametrize("k_sched", [(20, 0, 20), (20, 20, 0), (0, 20, 20)], ids=["mid", "last", "first"])
def test_coupled_gradient_with_empty_slow_steps(oracle_mod, k_sched):
    """A slow step with no inner steps: the u_bar of a coupled step reaches
    the drift of the inner step before it either through the increment the
    reverse adds at once (some inner step already reversed) or through the
    last inner step's drift reverse still to come (none reversed yet)."""
    from paper_2309_04010_amd import adjoint as A
    print(f"[coupled] gradient with inner counts {k_sched}", flush=True)
    c = _coupled_case("strip2d", 1)
    pr = A.MultirateProblem(c, B.SPH_F64, k_hist=c.run["fixed_inner"])
    pr.k_sched = np.array(k_sched, dtype=np.int64)
    pr.forward(pr.theta0())
    assert np.array_equal(pr.last["k"], pr.k_sched)
    w = np.random.default_rng(7).normal(0.0, 1.0, (c.dim, c.n))
    g = host(pr.backward(dev(w)))
    for nm in ("E", "D"):
        want = _oracle_coupled_objective(oracle_mod, c, pr.run, pr.k_sched, w, nm)
        gi = B.GRAD_NAMES.index(nm)
        print(f"  d/d{nm}: gpu {g[gi]:.10e} oracle {want:.10e}", flush=True)
        assert abs(g[gi] - want) <= 1e-8 * abs(want), (nm, g[gi], want)
    pr.close()


def test_batched_coupled_reverse_is_refused(oracle_mod):
    bt = cases.batch([cases.strip2d(nx=n, ny=6, n_slow=1, fixed_inner=5, k_max=0) for n in (10, 14)])
    nb = B.sph_build_neighbors_batched(dev(bt.X), dev(bt.V), bt.h, dev(bt.spec))
    st = B.new_state(nb, B.SPH_F64, with_diffusion=True)
    perm = nb.host("perm").astype(np.int64)
    st.flags = dev(bt.flags[perm])
    st.c.copy_(dev(bt.c_init[perm]))
    import torch
    grad = torch.zeros((2, B.SPH_NGRAD), dtype=torch.float64, device="cuda")
    batch = B.SphBatch(bt.E, bt.D, grad=grad)
    cfg = B.multirate_cfg(**dict(bt.run, slow_kind=cases.DIFFUSION_COUPLED), batch=batch)
    tape = B.SphTape(nb, B.SPH_F64, 1, 5, with_diffusion=True)
    adj = B.new_adjoint(nb, B.SPH_F64, with_diffusion=True)
    B.sph_advance_multirate(nb, B.material(**bt.material), st, cfg, tape=tape)
    with pytest.raises(B.SphError) as e:
        B.sph_advance_multirate_backward(nb, B.material(**bt.material), st, cfg, tape, adj)
    assert e.value.code == B.SPH_E_UNSUPPORTED
    nb.close()
