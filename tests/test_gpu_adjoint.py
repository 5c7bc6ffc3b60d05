"""Reverse mode on the GPU against the oracle's complex-step derivatives.

The oracle built with complex `real` gives exact directional derivatives of
the same discrete algorithm (Im f(x + i e) / e; pinned against central
differences in the oracle's own tests).  Each reverse-mode function of the
library is checked as the transpose of the forward map it reverses:
<w, J dx> from the oracle must equal <J^T w, dx> from the GPU, for random w
and dx, separately for every input group (state arrays and parameters).

Tolerances: FP64 1e-9 relative (rounding of two different evaluation orders
of the same derivative); FP32 2e-3 for the point and single-step checks (the
derivative is evaluated at FP32-rounded states; its terms carry ~1e-6
relative error that cancellation in the contractions amplifies) and 1e-3 for
whole runs against the FP64 oracle (the FP32 forward trajectory itself is
only within 1e-4 of the FP64 one; the gradients of the plate's whole
checkpointed run stay within 1e-5).
"""
import numpy as np
import pytest
import torch

from paper_2309_04010_amd import adjoint as A
from paper_2309_04010_amd import binding as B
from paper_2309_04010_amd import cases

from .parity_util import dev, host, jittered, torch_dtype

pytestmark = pytest.mark.gpu

TOL_POINT = {B.SPH_F64: 1e-9, B.SPH_F32: 2e-3}
TOL_RUN = {B.SPH_F64: 1e-8, B.SPH_F32: 1e-3}
PRECS = [B.SPH_F64, B.SPH_F32]
PIDS = ["f64", "f32"]


def _close(got, want, tol, what):
    scale = max(abs(want), 1e-300)
    assert abs(got - want) <= tol * scale, f"{what}: gpu {got!r} oracle {want!r} rel {abs(got - want) / scale:.3e}"


def _cs_oracle(oracle_mod, dim=3):
    X, V, h = jittered((3, 3, 3) if dim == 3 else (3, 3), jitter=0.0)
    return oracle_mod.Oracle(dim, X, V, h, complex_step=True)


# ---------------------------------------------------------------------------
# constitutive update: forward point parity and reverse vs complex step
MATS = {
    "LE": (dict(model=B.SPH_MODEL_LE, E=210e9, nu=0.3, rho0=7850.0), 1e-3),
    "NH": (dict(model=B.SPH_MODEL_NH, E=100e6, nu=0.4, rho0=2000.0), 5e-2),
    "J2": (cases.neck3d(nx=4, ny=3, nz=3).material, 5e-3),
}


def _point_inputs(model, n, scale, seed):
    rng = np.random.default_rng(seed)
    H = rng.normal(0.0, 1.0, (9, n)) * scale
    pl = np.zeros((7, n))
    if model == B.SPH_MODEL_J2:
        H[:, ::4] *= 0.04          # every fourth particle stays elastic
        pl[:6] = rng.normal(0.0, 1e-3, (6, n))
        pl[6] = rng.uniform(0.0, 0.05, n)
    p = rng.normal(0.0, 1e6, n)
    Pbar = rng.normal(0.0, 1.0, (9, n))
    plb = rng.normal(0.0, 1e11, (7, n)) if model == B.SPH_MODEL_J2 else np.zeros((7, n))
    return H, pl, p, Pbar, plb


@pytest.mark.parametrize("prec", PRECS, ids=PIDS)
@pytest.mark.parametrize("mname", list(MATS))
def test_constitutive_vjp_matches_complex_step(oracle_mod, mname, prec):
    kw, scale = MATS[mname]
    n = 24
    print(f"[adjoint] constitutive vjp {mname} prec={prec}", flush=True)
    H, pl, p, Pbar, plb = _point_inputs(kw["model"], n, scale, seed=11)
    T = torch_dtype(prec)
    if prec == B.SPH_F32:   # compare at the inputs the GPU actually sees
        H, pl, p, Pbar = (x.astype(np.float32).astype(np.float64) for x in (H, pl, p, Pbar))
    mat = B.material(**kw)
    j2 = kw["model"] == B.SPH_MODEL_J2
    plb_d = dev(plb, T)
    Hb, pb, thb = B.sph_constitutive_vjp(mat, prec, dev(H, T), dev(Pbar, T),
                                         plastic=dev(pl, T) if j2 else None,
                                         plastic_bar=plb_d if j2 else None, p=dev(p, T))
    Hb, pb, thb, plbar = host(Hb), host(pb), host(thb), host(plb_d)
    # forward point parity on the same inputs
    P = host(B.sph_constitutive(mat, prec, dev(H, T), plastic=dev(pl, T) if j2 else None, p=dev(p, T)))
    o = _cs_oracle(oracle_mod)
    eps = 1e-30
    pnames = ["E", "sigma0", "sigma_inf", "delta", "H"]
    for a in range(n):
        def L(Hc=H[:, a], plc=pl[:, a], pc=p[a], **mk):
            m = dict(kw)
            m.update(mk)
            rc, Pm, pln = o.constitutive(o.material(**m), H=Hc, plastic7=plc, p=pc)
            assert rc == 0
            return (Pbar[:, a] * Pm.reshape(9)).sum() + (plb[:, a] * pln).sum(), Pm
        _, P_or = L()
        ptol = 1e-10 if prec == B.SPH_F64 else 1e-4
        assert np.abs(P[:, a] - P_or.reshape(9).real).max() <= ptol * np.abs(P_or).max()
        tol = TOL_POINT[prec]
        gH = np.array([L(Hc=H[:, a] + 1j * eps * np.eye(9)[j])[0].imag / eps for j in range(9)])
        assert np.abs(Hb[:, a] - gH).max() <= tol * np.abs(gH).max(), (a, Hb[:, a], gH)
        gp = L(pc=p[a] + 1j * eps)[0].imag / eps
        _close(pb[a], gp, tol, f"pbar[{a}]")
        for j, nm in enumerate(pnames):
            base = kw.get(nm, 0.0)
            if not j2 and j > 0:
                assert thb[j, a] == 0.0
                continue
            e = eps * max(abs(base), 1.0)
            g = L(**{nm: base + 1j * e})[0].imag / e
            if g == 0.0:
                assert abs(thb[j, a]) <= 1e-12 * max(abs(thb[0, a]) * abs(kw["E"]), 1.0)
            else:
                _close(thb[j, a], g, tol, f"theta {nm}[{a}]")
        if j2:
            gY = np.array([L(plc=pl[:, a] + 1j * eps * np.eye(7)[j])[0].imag / eps for j in range(7)])
            assert np.abs(plbar[:, a] - gY).max() <= tol * np.abs(gY).max(), (a, plbar[:, a], gY)


# ---------------------------------------------------------------------------
# single steps: dot-product tests against the oracle's tangents
def _step_case(name):
    if name == "bar2d-LE":
        c = cases.bar2d(nx=14, ny=6)
        return c, 1e-3 * c.dp, False
    if name == "strip2d-NH":
        c = cases.strip2d(nx=16, ny=6)
        return c, 2e-2 * c.dp, True
    if name == "neck3d-J2":
        c = cases.neck3d(nx=9, ny=5, nz=5)
        return c, 5e-3 * c.dp, False
    if name == "plate3d-NH":
        c = cases.plate3d(nx=10, ny=9, nz=4)
        return c, 2e-2 * c.dp, True
    raise KeyError(name)


STEP_CASES = ["bar2d-LE", "strip2d-NH", "neck3d-J2", "plate3d-NH"]


def _dt(c):
    m = c.material
    K = m["E"] / (3 * (1 - 2 * m["nu"]))
    return 0.6 * c.h / np.sqrt(K / m["rho0"])


@pytest.mark.parametrize("prec", PRECS, ids=PIDS)
@pytest.mark.parametrize("name", STEP_CASES)
def test_solid_step_vjp_is_transpose(oracle_mod, name, prec):
    print(f"[adjoint] solid step vjp {name} prec={prec}", flush=True)
    c, uscale, with_p = _step_case(name)
    d, n = c.dim, c.n
    T = torch_dtype(prec)
    o = oracle_mod.Oracle(d, c.X, c.V, c.h)
    oc = oracle_mod.Oracle(d, c.X, c.V, c.h, complex_step=True)
    nb = B.sph_build_neighbors(dev(c.X), dev(c.V), c.h)
    perm = o.perm
    flags = np.ascontiguousarray(c.flags[perm])
    rng = np.random.default_rng(7)
    j2 = c.material["model"] == B.SPH_MODEL_J2
    # a stretched state with noise (J2: beyond first yield near the ends)
    u = np.vstack([(8.0 if j2 else 1.0) * uscale / c.dp * (o.X[0] - o.X[0].mean())] +
                  [np.zeros(n)] * (d - 1)) + rng.normal(0.0, uscale, (d, n))
    pl = np.zeros((7, n))
    if j2:
        pl[:6] = rng.normal(0.0, 1e-4, (6, n))
        pl[6] = rng.uniform(0.0, 0.01, n)
    p = rng.normal(0.0, 1e5, n) if with_p else np.zeros(n)
    w = rng.normal(0.0, 1.0, (d, n))
    yb = rng.normal(0.0, 1e9, (7, n)) if j2 else np.zeros((7, n))
    if prec == B.SPH_F32:
        pl, p, w = (x.astype(np.float32).astype(np.float64) for x in (pl, p, w))
    dt = _dt(c)
    st = B.new_state(nb, prec, with_plastic=j2, with_diffusion=with_p)
    st.u.copy_(dev(u))
    st.flags = dev(flags)
    if j2:
        st.plastic.copy_(dev(pl, T))
    if with_p:
        st.p.copy_(dev(p, T))
    adj = B.new_adjoint(nb, prec, with_plastic=j2, with_p=True)
    adj.v.copy_(dev(w, T))
    if j2:
        adj.plastic.copy_(dev(yb, T))
    mat = B.material(**c.material)
    B.sph_solid_relax_step_vjp(nb, mat, st, adj, dt)
    ub, pb, grad = host(adj.u), host(adj.p), host(adj.grad)
    plb = host(adj.plastic) if j2 else None
    # the step must leave the forward state alone
    assert np.array_equal(host(st.u), u)

    def L(uc=u, plc=pl, pc=p, **mk):
        m = dict(c.material)
        m.update(mk)
        v = oc.arr(d, n)
        pll = np.ascontiguousarray(plc, dtype=complex).copy() if j2 else None
        rc, _, _ = oc.solid_step(oc.material(**m), dt, np.ascontiguousarray(uc, dtype=complex), v,
                                 plastic=pll, p=np.ascontiguousarray(pc, dtype=complex) if with_p else None,
                                 flags=flags)
        assert rc == 0
        val = (w * v).sum()
        if j2:
            val += (yb * pll).sum()
        return val

    eps = 1e-30
    tol = TOL_POINT[prec]
    du = rng.normal(0.0, 1.0, (d, n))
    _close((ub * du).sum(), L(uc=u + 1j * eps * du).imag / eps, tol, "u")
    if j2:
        dy = rng.normal(0.0, 1.0, (7, n))
        _close((plb * dy).sum(), L(plc=pl + 1j * eps * dy).imag / eps, tol, "plastic")
    if with_p:
        dp_ = rng.normal(0.0, 1.0, n)
        _close((pb * dp_).sum(), L(pc=p + 1j * eps * dp_).imag / eps, tol, "p")
    E = c.material["E"]
    _close(grad[B.SPH_GRAD_E], L(E=E + 1j * eps * E).imag / (eps * E), tol, "E")
    if j2:
        for gi, nm in [(B.SPH_GRAD_S0, "sigma0"), (B.SPH_GRAD_SINF, "sigma_inf"),
                       (B.SPH_GRAD_DELTA, "delta"), (B.SPH_GRAD_H, "H")]:
            base = c.material[nm]
            e = eps * max(abs(base), 1.0)
            want = L(**{nm: base + 1j * e}).imag / e
            if want == 0.0:
                assert grad[gi] == 0.0
            else:
                _close(grad[gi], want, tol, nm)
    nb.close()


@pytest.mark.parametrize("prec", PRECS, ids=PIDS)
@pytest.mark.parametrize("name", ["strip2d-NH", "plate3d-NH", "neck3d-J2"])
def test_damping_vjp_is_transpose(oracle_mod, name, prec):
    print(f"[adjoint] damping vjp {name} prec={prec}", flush=True)
    c, _, _ = _step_case(name)
    d, n = c.dim, c.n
    T = torch_dtype(prec)
    o = oracle_mod.Oracle(d, c.X, c.V, c.h)
    nb = B.sph_build_neighbors(dev(c.X), dev(c.V), c.h)
    flags = np.ascontiguousarray(c.flags[o.perm])
    rng = np.random.default_rng(3)
    wbar = rng.normal(0.0, 1.0, (d, n))
    dv = rng.normal(0.0, 1.0, (d, n))
    if prec == B.SPH_F32:
        wbar = wbar.astype(np.float32).astype(np.float64)
    dt, eta, rho0 = _dt(c), 50.0 * c.run["eta"], c.material["rho0"]
    st = B.new_state(nb, prec)
    st.flags = dev(flags)
    adj = B.new_adjoint(nb, prec)
    adj.v.copy_(dev(wbar, T))
    B.sph_damping_sweep_vjp(nb, B.material(**c.material), st, adj, eta, dt)
    Sdv = dv.copy()
    o.damping_sweep(rho0, eta, dt, Sdv, flags)
    assert np.abs(Sdv - dv).max() > 1e-3 * np.abs(dv).max()   # the sweep does something
    _close((host(adj.v) * dv).sum(), (wbar * Sdv).sum(), 1e-12 if prec == B.SPH_F64 else 1e-5, "sweep^T")
    nb.close()


@pytest.mark.parametrize("prec", PRECS, ids=PIDS)
@pytest.mark.parametrize("name", ["strip2d-NH", "plate3d-NH"])
def test_diffusion_vjp_is_transpose(oracle_mod, name, prec):
    print(f"[adjoint] diffusion vjp {name} prec={prec}", flush=True)
    c, _, _ = _step_case(name)
    d, n = c.dim, c.n
    T = torch_dtype(prec)
    o = oracle_mod.Oracle(d, c.X, c.V, c.h, complex_step=True)
    nb = B.sph_build_neighbors(dev(c.X), dev(c.V), c.h)
    flags = np.ascontiguousarray(c.flags[o.perm])
    rng = np.random.default_rng(5)
    c0 = rng.uniform(0.0, 0.4, n)
    cb = rng.normal(0.0, 1.0, n)
    pbv = rng.normal(0.0, 1e-6, n)
    if prec == B.SPH_F32:
        c0, cb = (x.astype(np.float32).astype(np.float64) for x in (c0, cb))
    Dc, dt_d = c.run["D"], 0.5 * c.h ** 2 / c.run["D"]
    mk = c.material
    st = B.new_state(nb, prec, with_diffusion=True)
    st.flags = dev(flags)
    st.c.copy_(dev(c0, T))
    c_before = st.c.clone()
    mat = B.material(**mk)
    B.sph_diffusion_step(nb, mat, st, Dc, dt_d, c.run["c_bc"])
    adj = B.new_adjoint(nb, prec, with_diffusion=True)
    adj.c.copy_(dev(cb, T))
    adj.p.copy_(dev(pbv))
    B.sph_diffusion_step_vjp(nb, mat, st, c_before, adj, Dc, dt_d, c.run["c_bc"])
    cbar, grad = host(adj.c), host(adj.grad)
    assert np.all(host(adj.p) == 0.0)

    def L(cc=c0, D=Dc, C=mk["C_swell"]):
        x = np.ascontiguousarray(cc, dtype=complex).copy()
        q, p = o.arr(d, n), o.arr(n)
        o.diffusion_step(D, dt_d, c.run["c_bc"], C, mk["c0"], x, q, p, flags)
        return (cb * x).sum() + (pbv * p).sum()

    eps = 1e-30
    tol = TOL_POINT[prec]
    dc = rng.normal(0.0, 1.0, n)
    _close((cbar * dc).sum(), L(cc=c0 + 1j * eps * dc).imag / eps, tol, "c")
    _close(grad[B.SPH_GRAD_D], L(D=Dc + 1j * eps * Dc).imag / (eps * Dc), tol, "D")
    C = mk["C_swell"]
    _close(grad[B.SPH_GRAD_C], L(C=C + 1j * eps * C).imag / (eps * C), tol, "C_swell")
    nb.close()


# ---------------------------------------------------------------------------
# whole multi-time-step runs: gradient of <w, u_final> against the oracle
def _run_case(name):
    if name == "strip2d":
        return cases.strip2d(nx=24, ny=6, n_slow=2, fixed_inner=30, k_max=0), ["E", "D", "C_swell"]
    if name == "neck3d":
        c = cases.neck3d(nx=12, ny=5, nz=5, n_slow=2, fixed_inner=25, total_stretch=1.2e-4)
        return c, ["E", "sigma0", "sigma_inf", "delta", "H"]
    if name == "bar2d":
        return cases.bar2d(nx=16, ny=6, n_slow=3), ["E"]
    if name == "plate3d-40x40x4":
        return cases.plate3d(nx=40, ny=40, n_slow=2, fixed_inner=20), ["E", "D", "C_swell"]
    raise KeyError(name)


def _oracle_objective(oracle_mod, c, run, k_sched, w, param=None, eps_rel=1e-20):
    """<w, u_final> from the complex-step oracle with one parameter perturbed
    by i eps; returns d<w,u>/d(param)."""
    d, n = c.dim, c.n
    o = oracle_mod.Oracle(d, c.X, c.V, c.h, complex_step=True)
    perm = o.perm
    flags = np.ascontiguousarray(c.flags[perm])
    m, r = dict(c.material), dict(run)
    base = (r["D"] if param == "D" else m[param])
    e = eps_rel * max(abs(base), 1.0)
    if param == "D":
        r["D"] = base + 1j * e
    else:
        m[param] = base + 1j * e
    mat = o.material(**m)
    cfg = o.cfg(**{k: v for k, v in r.items() if k != "D"}, D=r["D"])
    u, v = o.arr(d, n), o.arr(d, n)
    pl = o.arr(7, n) if m["model"] == B.SPH_MODEL_J2 else None
    diff = r["slow_kind"] == B.SPH_SLOW_DIFFUSION
    cc = np.ascontiguousarray(c.c_init[perm], dtype=complex) if diff else None
    q, p = (o.arr(d, n), o.arr(n)) if diff else (None, None)
    vg = np.ascontiguousarray(c.vgrip[:, perm], dtype=complex) if c.vgrip is not None else None
    rc, k, _, _ = o.advance(mat, cfg, u, v, plastic=pl, c=cc, q=q, p=p, vgrip=vg, flags=flags,
                            k_sched=k_sched)
    assert rc in (0, 1) and np.array_equal(k, k_sched)
    return (w * u).sum().imag / e


@pytest.mark.parametrize("prec", PRECS, ids=PIDS)
@pytest.mark.parametrize("name", ["bar2d", "strip2d", "neck3d", "plate3d-40x40x4"])
def test_multirate_gradient_matches_oracle(oracle_mod, name, prec):
    print(f"[adjoint] multirate gradient {name} prec={prec}", flush=True)
    c, params = _run_case(name)
    kh = c.run["fixed_inner"] if c.run["fixed_inner"] > 0 else 20000
    pr = A.MultirateProblem(c, prec, k_hist=kh)
    pr.forward(pr.theta0())
    pr.freeze()
    rng = np.random.default_rng(2)
    w = rng.normal(0.0, 1.0, (c.dim, c.n))
    pr.forward(pr.theta0())
    g = host(pr.backward(dev(w)))
    for nm in params:
        want = _oracle_objective(oracle_mod, c, pr.run, pr.k_sched, w, nm)
        gi = B.GRAD_NAMES.index(nm)
        print(f"  d/d{nm}: gpu {g[gi]:.10e} oracle {want:.10e}", flush=True)
        _close(g[gi], want, TOL_RUN[prec], nm)
    pr.close()


def test_backward_is_deterministic_and_recomputes(oracle_mod):
    """Two reverse passes of one taped run agree bitwise: the second re-runs
    the last slow step from its checkpoint instead of reading the recorded
    inner states, so this also checks the recompute path; the state is
    restored to the final one."""
    c = cases.strip2d(nx=24, ny=6, n_slow=3, fixed_inner=20, k_max=0)
    pr = A.MultirateProblem(c, B.SPH_F64, k_hist=20)
    u_end = pr.forward(pr.theta0()).clone()
    assert pr.tape.hist_slow == 2
    w = dev(np.random.default_rng(1).normal(0.0, 1.0, (2, c.n)))
    g1 = pr.backward(w)
    assert pr.tape.hist_slow == 0
    assert torch.equal(pr.st.u, u_end)
    g2 = pr.backward(w)
    assert torch.equal(g1, g2)
    pr.close()


@pytest.mark.parametrize("prec", PRECS, ids=PIDS)
@pytest.mark.parametrize("name", ["strip2d", "neck3d", "bar2d"])
def test_segmented_reverse_equals_whole(oracle_mod, name, prec):
    """Slow steps reversed in segments of k_hist inner steps (two-level
    checkpointing, a ragged last segment) give the gradient, the adjoint state
    and the restored final state of the reverse pass over whole slow steps,
    bitwise: the same kernels see the same recorded states.  One inner
    checkpoint too few is refused before anything runs."""
    print(f"[adjoint] segmented reverse {name} prec={prec}", flush=True)
    c, _ = _run_case(name)
    kh = c.run["fixed_inner"] if c.run["fixed_inner"] > 0 else 20000
    pr = A.MultirateProblem(c, prec, k_hist=kh)
    th = pr.theta0()
    pr.forward(th)
    pr.freeze()
    kmax = int(pr.k_sched.max())
    K = 7 if kmax <= 60 else kmax // 5 + 3
    ns = -(-kmax // K)
    assert ns >= 3 and kmax % K != 0, (kmax, K)
    w = dev(np.random.default_rng(4).normal(0.0, 1.0, (c.dim, c.n)))
    u_end = pr.forward(th).clone()
    g_whole = pr.backward(w, recompute=True)
    au, av = pr.adj.u.clone(), pr.adj.v.clone()
    whole = pr.tape
    pr.tape = B.SphTape(pr.nb, prec, c.run["n_slow"], K, with_plastic=pr.j2,
                        with_diffusion=pr.diff, seg_cap=ns - 1)
    pr.forward(th)
    assert torch.equal(pr.st.u, u_end)
    g_seg = pr.backward(w)
    assert torch.equal(g_seg, g_whole)
    assert torch.equal(pr.adj.u, au) and torch.equal(pr.adj.v, av)
    assert torch.equal(pr.st.u, u_end)
    assert pr.tape.hist_slow == -1
    pr.tape = B.SphTape(pr.nb, prec, c.run["n_slow"], K, with_plastic=pr.j2,
                        with_diffusion=pr.diff, seg_cap=ns - 2)
    pr.forward(th)
    with pytest.raises(B.SphError) as e:
        pr.backward(w)
    assert e.value.code == B.SPH_E_CAPACITY
    assert torch.equal(pr.st.u, u_end)
    pr.tape = whole
    pr.close()


def test_finite_differences_plate_subset(oracle_mod):
    """d(mean centre deflection)/d(E, D, C) on the 40 x 40 x 4 plate: the
    reverse pass against central differences of the GPU FP64 forward run with
    the same frozen schedule."""
    c, params = _run_case("plate3d-40x40x4")
    pr = A.MultirateProblem(c, B.SPH_F64)
    th0 = pr.theta0()
    pr.forward(th0)
    pr.freeze()
    idx = pr.perm.argsort()[c.observable["J_index"]]   # sorted positions of the centre columns
    comp = c.observable["J_component"]
    w = np.zeros((3, c.n))
    w[comp, idx] = 1.0 / len(idx)

    def J(th):
        return float((host(pr.forward(th)) * w).sum())

    pr.forward(th0)
    g = host(pr.backward(dev(w)))
    assert J(th0) != 0.0
    for nm in params:
        i = B.GRAD_NAMES.index(nm)
        h = 1e-5 * th0[i]
        tp, tm = th0.copy(), th0.copy()
        tp[i] += h
        tm[i] -= h
        fd = (J(tp) - J(tm)) / (2 * h)
        print(f"  dJ/d{nm}: adjoint {g[i]:.8e} fd {fd:.8e}", flush=True)
        _close(g[i], fd, 1e-5, nm)
    pr.close()


def test_autograd_function(oracle_mod):
    """torch.autograd through the solve equals the direct reverse pass."""
    c = cases.strip2d(nx=20, ny=6, n_slow=2, fixed_inner=15, k_max=0)
    pr = A.MultirateProblem(c, B.SPH_F64)
    theta = torch.tensor(pr.theta0(), dtype=torch.float64, requires_grad=True)
    u = A.solve(theta, pr)
    idx = torch.as_tensor(pr.perm.argsort()[c.observable["J_index"]])
    J = u[1, idx.cuda()].mean()
    J.backward()
    w = torch.zeros_like(u)
    w[1, idx.cuda()] = 1.0 / len(idx)
    pr.forward(pr.theta0())
    g = pr.backward(w).cpu()
    assert torch.allclose(theta.grad, g, rtol=1e-13, atol=0.0)
    assert theta.grad[B.SPH_GRAD_E] != 0.0 and theta.grad[B.SPH_GRAD_D] != 0.0
    pr.close()


def test_autograd_function_two_solves_before_backward(oracle_mod):
    """Two solves on one problem at different theta, then the first
    objective's backward: the gradient is the first run's (the reverse pass
    re-records that run when a later one replaced its tape)."""
    c = cases.strip2d(nx=20, ny=6, n_slow=2, fixed_inner=15, k_max=0)
    pr = A.MultirateProblem(c, B.SPH_F64)
    th0 = pr.theta0()
    th1 = th0.copy()
    th1[B.SPH_GRAD_E] *= 1.7
    th1[B.SPH_GRAD_D] *= 0.5
    idx = torch.as_tensor(pr.perm.argsort()[c.observable["J_index"]]).cuda()
    t0 = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    t1 = torch.tensor(th1, dtype=torch.float64, requires_grad=True)
    J0 = A.solve(t0, pr)[1, idx].mean()
    J1 = A.solve(t1, pr)[1, idx].mean()
    J0.backward()
    J1.backward()
    w = torch.zeros((2, c.n), dtype=torch.float64, device="cuda")
    w[1, idx] = 1.0 / len(idx)
    want = []
    for th in (th0, th1):
        pr.forward(th)
        want.append(pr.backward(w).cpu())
    assert not torch.allclose(want[0], want[1])
    assert torch.allclose(t0.grad, want[0], rtol=1e-13, atol=0.0)
    assert torch.allclose(t1.grad, want[1], rtol=1e-13, atol=0.0)
    pr.close()
