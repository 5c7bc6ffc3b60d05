"""Parity at the benchmark's full size: the 500 x 500 x 4 plate (1,000,000
particles, 60,256,216 directed pairs), with the launch shapes the benchmark
tunes and uses.

The state is made non-trivial on the GPU (a diffusion step and some inner
steps), copied to the host, and one application of each step is then
compared, element by element, with the oracle applied to the same input:
the solid stage (stress, P B0, momentum, kick), the damping sweep, its
transpose (as a dot product with the oracle's sweep), drift + kinetic
energy, the diffusion step, a solid stage with the mixture momentum and the
two-way coupled diffusion step.  Tolerances: FP64 1e-10, FP32 1e-4 (1e-5
for the transposed sweep's dot product).
"""
import numpy as np
import pytest
import torch

from paper_2309_04010_amd import binding as B
from paper_2309_04010_amd import cases

from .parity_util import TOL, dev, host, rel_err, torch_dtype

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def plate(oracle_mod):
    c = cases.plate3d()
    print(f"[fullsize] building the {c.n}-particle plate on both sides", flush=True)
    o = oracle_mod.Oracle(3, c.X, c.V, c.h)
    nb = B.sph_build_neighbors(dev(c.X), dev(c.V), c.h)
    yield c, o, nb
    nb.close()


@pytest.mark.parametrize("prec", [B.SPH_F32, B.SPH_F64], ids=["f32", "f64"])
def test_full_size_steps(plate, prec):
    c, o, nb = plate
    T = torch_dtype(prec)
    perm = o.perm
    flags = np.ascontiguousarray(c.flags[perm])
    m = c.material
    mg, mo = B.material(**m), o.material(**m)
    K = m["E"] / (3 * (1 - 2 * m["nu"]))
    dt = 0.6 * c.h / np.sqrt(K / m["rho0"])
    eta = c.run["eta"]
    st = B.new_state(nb, prec, with_diffusion=True, with_acc=True)
    st.flags = dev(flags)
    st.c.copy_(dev(c.c_init[perm], T))
    B.sph_autotune(nb, mg, st, eta, dt, with_adjoint=True)
    # a non-trivial state: diffusion, then some inner steps
    cfg = B.multirate_cfg(**dict(c.run, n_slow=1, fixed_inner=60))
    B.sph_advance_multirate(nb, mg, st, cfg)
    u, v = host(st.u), host(st.v)
    cc, p = host(st.c), host(st.p)
    assert np.abs(u).max() > 0 and np.abs(v).max() > 0
    tol = TOL[prec]

    # solid stage
    print(f"[fullsize] solid stage prec={prec}", flush=True)
    vo = v.copy()
    rc, PBo, acco = o.solid_step(mo, dt, np.ascontiguousarray(u), vo, p=np.ascontiguousarray(p),
                                 flags=flags)
    assert rc == 0
    B.sph_solid_relax_step(nb, mg, st, dt)
    assert rel_err(host(st.PB), PBo) < tol
    assert rel_err(host(st.acc), acco) < tol
    assert rel_err(host(st.v) - v, vo - v) < tol

    # damping sweep from the kicked velocity
    print(f"[fullsize] damping sweep prec={prec}", flush=True)
    v1 = host(st.v)
    w = v1.copy()
    o.damping_sweep(m["rho0"], eta, dt, w, flags)
    B.sph_damping_sweep(nb, mg, st, eta, dt)
    assert rel_err(host(st.v) - v1, w - v1) < tol

    # transposed sweep: <wbar, S dv> = <S^T wbar, dv>
    rng = np.random.default_rng(0)
    wbar = rng.normal(0.0, 1.0, (3, c.n))
    if prec == B.SPH_F32:
        wbar = wbar.astype(np.float32).astype(np.float64)
    dv = rng.normal(0.0, 1.0, (3, c.n))
    adj = B.new_adjoint(nb, prec)
    adj.v.copy_(dev(wbar, T))
    B.sph_damping_sweep_vjp(nb, mg, st, adj, eta, dt)
    Sdv = dv.copy()
    o.damping_sweep(m["rho0"], eta, dt, Sdv, flags)
    lhs, rhs = (host(adj.v) * dv).sum(), (wbar * Sdv).sum()
    assert abs(lhs - rhs) <= (1e-12 if prec == B.SPH_F64 else 1e-5) * abs(rhs)

    # drift and kinetic energy
    print(f"[fullsize] drift prec={prec}", flush=True)
    v2 = host(st.v)
    uo = u.copy()
    keo = o.drift_ke(m["rho0"], dt, uo, np.ascontiguousarray(v2), flags)
    ked = torch.zeros(1, dtype=torch.float64, device="cuda")
    B.sph_drift_ke(nb, mg, st, dt, ke_out=ked)
    assert rel_err(host(st.u) - u, uo - u) < tol
    assert abs(ked.item() - keo) <= 1e-12 * keo

    # diffusion step from the current saturation
    print(f"[fullsize] diffusion prec={prec}", flush=True)
    co = cc.copy()
    qo, po = o.arr(3, c.n), o.arr(c.n)
    Dc, dtd = c.run["D"], 0.5 * c.h ** 2 / c.run["D"]
    o.diffusion_step(Dc, dtd, c.run["c_bc"], m["C_swell"], m["c0"], co, qo, po, flags)
    B.sph_diffusion_step(nb, mg, st, Dc, dtd, c.run["c_bc"])
    assert rel_err(host(st.c) - cc, co - cc) < tol
    assert rel_err(host(st.p), po) < tol

    # one solid stage with the mixture momentum (fluid density 1000), from the
    # state and the flux the diffusion step has just left
    print(f"[fullsize] mixture solid stage prec={prec}", flush=True)
    mm = dict(m, rho_l0=1000.0)
    u4, v4, c4, q4, p4 = host(st.u), host(st.v), host(st.c), host(st.q), host(st.p)
    vo = v4.copy()
    rc, PBo, acco = o.solid_step(o.material(**mm), dt, np.ascontiguousarray(u4), vo, p=p4, flags=flags,
                                 c=c4, q=q4)
    assert rc == 0
    B.sph_solid_relax_step(nb, B.material(**mm), st, dt)
    assert rel_err(host(st.PB), PBo) < tol
    assert rel_err(host(st.acc), acco) < tol
    assert rel_err(host(st.v) - v4, vo - v4) < tol

    # two-way coupled diffusion (nonlinear flux) from the deformed state
    print(f"[fullsize] coupled diffusion prec={prec}", flush=True)
    u3, c3 = host(st.u), host(st.c)
    co = c3.copy()
    qo, po = o.arr(3, c.n), o.arr(c.n)
    o.diffusion_step_coupled(Dc, dtd, c.run["c_bc"], m["C_swell"], m["c0"], 1,
                             np.ascontiguousarray(u3), co, qo, po, flags)
    B.sph_diffusion_step_coupled(nb, mg, st, Dc, dtd, c.run["c_bc"], nonlinear=1)
    assert rel_err(host(st.c) - c3, co - c3) < tol
    assert rel_err(host(st.p), po) < tol
