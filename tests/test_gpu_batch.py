"""Batched specimens: one particle set holding several strips with their own
E, D and step sizes, run forward and in reverse in single launches.

* each specimen of an FP64 batched run equals the oracle run of that
  specimen alone (1e-10), and FP32 is within 1e-4; also with the two-way
  coupled nonlinear slow step and the mixture momentum;
* with each specimen at its own coordinates (overlapping in space), a
  batched specimen equals its own GPU run bitwise: same cells, order,
  neighbours and schedule;
* per-specimen gradients of <w, u_final> equal the complex-step oracle's for
  each specimen alone;
* the whole forward + reverse run recorded as one hipGraph equals the eager
  calls bitwise, also when relaunched with new per-specimen E and D;
* specimen ids that are not contiguous ascending runs are refused.
"""
import numpy as np
import pytest
import torch

from paper_2309_04010_amd import binding as B
from paper_2309_04010_amd import cases

from .parity_util import dev, host, rel_err, torch_dtype

pytestmark = pytest.mark.gpu


def _small_batch(n_slow=2, fixed_inner=20, stack=True):
    rng = np.random.default_rng(8)
    cs = []
    for nx in (9, 14, 22, 11):
        E = float(rng.uniform(50e6, 200e6))
        D = float(np.exp(rng.uniform(np.log(1e-11), np.log(1e-9))))
        cs.append(cases.strip2d(nx=nx, ny=6, E=E, D=D, n_slow=n_slow, fixed_inner=fixed_inner,
                                k_max=0, eta=5.0))
    return cases.batch(cs, stack=stack)


class _Run:
    """Device set-up of a batch: neighbourhood, specimen ids, state, tape."""

    def __init__(self, bt, prec, grad=True):
        self.bt, self.prec = bt, prec
        T = torch_dtype(prec)
        self.nb = B.sph_build_neighbors_batched(dev(bt.X), dev(bt.V), bt.h, dev(bt.spec))
        self.perm = self.nb.host("perm").astype(np.int64)
        self.st = B.new_state(self.nb, prec, with_diffusion=True)
        self.st.flags = dev(bt.flags[self.perm])
        self.c0 = dev(bt.c_init[self.perm], T)
        self.grad = torch.zeros((len(bt.cases), B.SPH_NGRAD), dtype=torch.float64, device="cuda")
        # step sizes left to the library: each specimen's sph_default_steps
        self.batch = B.SphBatch(bt.E, bt.D, grad=self.grad)
        r = dict(bt.run)
        self.cfg = B.multirate_cfg(**r, batch=self.batch)
        self.mat = B.material(**bt.material)
        self.tape = B.SphTape(self.nb, prec, r["n_slow"], r["fixed_inner"], with_diffusion=True)
        self.adj = B.new_adjoint(self.nb, prec, with_diffusion=True)

    def reset(self):
        st = self.st
        st.u.zero_()
        st.v.zero_()
        st.c.copy_(self.c0)
        st.q.zero_()
        st.p.zero_()

    def set_w(self, w_sorted):
        self.adj.zero_()
        self.adj.u.copy_(w_sorted)
        self.grad.zero_()

    def u_input_order(self):
        u = host(self.st.u)
        out = np.empty_like(u)
        out[:, self.perm] = u
        return out


def _oracle_strip(oracle_mod, c, E, D, complex_step=False, pert=None, slow_kind=None,
                  nonlinear=0, rho_l0=0.0):
    """The oracle run of one specimen alone; it derives its own step sizes
    (Sec. 4.1) from E and D, independently of the library."""
    o = oracle_mod.Oracle(2, c.X, c.V, c.h, complex_step=complex_step)
    perm = o.perm
    flags = np.ascontiguousarray(c.flags[perm])
    m = dict(c.material, E=E, rho_l0=rho_l0)
    r = dict(c.run, D=D, dt_s=0.0, dt_slow=0.0)
    if slow_kind is not None:
        r["slow_kind"] = slow_kind
    if pert:
        (nm, val), = pert.items()
        if nm == "D":
            r["D"] = val
        else:
            m[nm] = val
    cfg = o.cfg(**{k: v for k, v in r.items() if k != "D"}, D=r["D"], nonlinear=nonlinear)
    u, v = o.arr(2, c.n), o.arr(2, c.n)
    cc = np.ascontiguousarray(c.c_init[perm], dtype=o.dtype)
    q, p = o.arr(2, c.n), o.arr(c.n)
    rc, k, _, _ = o.advance(o.material(**m), cfg, u, v, c=cc, q=q, p=p, flags=flags)
    assert rc in (0, 1)
    uin = np.empty_like(u)
    uin[:, perm] = u
    return uin


@pytest.mark.parametrize("prec", [B.SPH_F64, B.SPH_F32], ids=["f64", "f32"])
def test_batched_forward_equals_each_specimen_alone(oracle_mod, prec):
    bt = _small_batch()
    print(f"[batch] forward parity, {len(bt.cases)} strips, n={bt.n}, prec={prec}", flush=True)
    R = _Run(bt, prec)
    R.reset()
    rc, k, _, _, _ = B.sph_advance_multirate(R.nb, R.mat, R.st, R.cfg)
    assert np.all(k == bt.run["fixed_inner"])
    u = R.u_input_order()
    tol = 1e-10 if prec == B.SPH_F64 else 1e-4
    for i, c in enumerate(bt.cases):
        want = _oracle_strip(oracle_mod, c, bt.E[i], bt.D[i])
        got = u[:, bt.offsets[i]:bt.offsets[i + 1]]
        assert np.abs(want).max() > 0
        assert rel_err(got, want) < tol, (i, rel_err(got, want))
    R.nb.close()


def test_batched_coupled_mixture_equals_each_specimen_alone(oracle_mod):
    """The two-way coupled nonlinear slow step and the mixture momentum in a
    batched run: per-specimen D and step sizes reach the coupled kernels, the
    mixture masses and the kinetic energy."""
    bt = _small_batch()
    print(f"[batch] coupled + mixture, {len(bt.cases)} strips, n={bt.n}", flush=True)
    R = _Run(bt, B.SPH_F64)
    R.reset()
    r = dict(bt.run, slow_kind=cases.DIFFUSION_COUPLED)
    cfg = B.multirate_cfg(**r, batch=R.batch, diff_nonlinear=1)
    mat = B.material(**dict(bt.material, rho_l0=1000.0))
    rc, k, _, _, _ = B.sph_advance_multirate(R.nb, mat, R.st, cfg)
    assert np.all(k == bt.run["fixed_inner"])
    u = R.u_input_order()
    for i, c in enumerate(bt.cases):
        want = _oracle_strip(oracle_mod, c, bt.E[i], bt.D[i],
                             slow_kind=cases.DIFFUSION_COUPLED, nonlinear=1, rho_l0=1000.0)
        got = u[:, bt.offsets[i]:bt.offsets[i + 1]]
        assert np.abs(want).max() > 0
        assert rel_err(got, want) < 1e-10, (i, rel_err(got, want))
    R.nb.close()


def test_batched_gradients_equal_each_specimen_alone(oracle_mod):
    bt = _small_batch()
    R = _Run(bt, B.SPH_F64)
    rng = np.random.default_rng(4)
    w_in = rng.normal(0.0, 1.0, (2, bt.n))
    R.reset()
    B.sph_advance_multirate(R.nb, R.mat, R.st, R.cfg, tape=R.tape)
    R.set_w(dev(w_in[:, R.perm]))
    B.sph_advance_multirate_backward(R.nb, R.mat, R.st, R.cfg, R.tape, R.adj)
    g = host(R.grad)
    eps = 1e-20
    for i, c in enumerate(bt.cases):
        wi = w_in[:, bt.offsets[i]:bt.offsets[i + 1]]
        args = (bt.E[i], bt.D[i])
        for nm, gi, base in [("E", B.SPH_GRAD_E, bt.E[i]), ("D", B.SPH_GRAD_D, bt.D[i]),
                             ("C_swell", B.SPH_GRAD_C, bt.material["C_swell"])]:
            h = eps * base
            if nm == "E":
                u = _oracle_strip(oracle_mod, c, base + 1j * h, *args[1:], complex_step=True)
            else:
                u = _oracle_strip(oracle_mod, c, *args, complex_step=True, pert={nm: base + 1j * h})
            want = (wi * u).sum().imag / h
            print(f"  strip {i} d/d{nm}: gpu {g[i, gi]:.10e} oracle {want:.10e}", flush=True)
            assert abs(g[i, gi] - want) <= 1e-8 * abs(want), (i, nm)
    R.nb.close()


@pytest.mark.parametrize("prec", [B.SPH_F32, B.SPH_F64], ids=["f32", "f64"])
def test_whole_run_graph_equals_eager_bitwise(oracle_mod, prec):
    bt = _small_batch(n_slow=3, fixed_inner=15)
    R = _Run(bt, prec)
    w = dev(np.random.default_rng(6).normal(0.0, 1.0, (2, bt.n))[:, R.perm])
    T = torch_dtype(prec)

    def eager():
        R.reset()
        B.sph_advance_multirate(R.nb, R.mat, R.st, R.cfg, tape=R.tape)
        R.set_w(w)
        B.sph_advance_multirate_backward(R.nb, R.mat, R.st, R.cfg, R.tape, R.adj)
        return R.st.u.clone(), R.grad.clone(), R.adj.u.clone()

    def graph():
        R.reset()
        R.set_w(w)
        B.sph_advance_multirate_graph(R.nb, R.mat, R.st, R.cfg, R.tape, R.adj)
        return R.st.u.clone(), R.grad.clone(), R.adj.u.clone()

    ue, ge, ae = eager()
    for _ in range(2):        # first launch records, the second replays the cached graph
        ug, gg, ag = graph()
        assert torch.equal(ue, ug) and torch.equal(ge, gg) and torch.equal(ae, ag)
    # new per-specimen values: the cached graph is relaunched with new tables
    R.batch.E[:] = R.batch.E[::-1].copy()
    R.batch.D[:] = R.batch.D * 1.5
    ue2, ge2, _ = eager()
    ug2, gg2, _ = graph()
    assert not torch.equal(ue2, ue)
    assert torch.equal(ue2, ug2) and torch.equal(ge2, gg2)
    assert R.st.u.dtype == torch.float64 and R.st.v.dtype == T
    R.nb.close()


@pytest.mark.parametrize("k_hist,seg_cap", [(12, 0), (5, 2)], ids=["whole", "segments"])
def test_single_specimen_whole_run_graph(oracle_mod, k_hist, seg_cap):
    """Without a batch: one recorded forward + reverse equals the eager pair,
    also with the slow steps reversed in segments (5 + 5 + 2 inner steps)."""
    from paper_2309_04010_amd import adjoint as A
    c = cases.strip2d(nx=20, ny=6, n_slow=3, fixed_inner=12, k_max=0)
    pr = A.MultirateProblem(c, B.SPH_F64, k_hist=k_hist, seg_cap=seg_cap)
    th = pr.theta0()
    w = dev(np.random.default_rng(3).normal(0.0, 1.0, (2, c.n)))
    pr.forward(th)
    ge = pr.backward(w)
    ue = pr.st.u.clone()
    pr.reset()
    a = pr.adj.zero_()
    a.u.copy_(w)
    B.sph_advance_multirate_graph(pr.nb, pr._material(th), pr.st, pr._cfg(th), pr.tape, a)
    assert torch.equal(pr.st.u, ue)
    assert torch.equal(a.grad, ge)
    pr.close()


@pytest.mark.parametrize("prec", [B.SPH_F64, B.SPH_F32], ids=["f64", "f32"])
def test_overlapping_specimens_equal_their_own_runs_bitwise(oracle_mod, prec):
    from paper_2309_04010_amd import adjoint as A
    bt = _small_batch(stack=False)
    R = _Run(bt, prec)
    R.reset()
    B.sph_advance_multirate(R.nb, R.mat, R.st, R.cfg)
    u = R.st.u.clone()
    for i, c in enumerate(bt.cases):
        pr = A.MultirateProblem(c, prec)
        pr.forward(pr.theta0(), record=False)
        q0, q1 = bt.offsets[i], bt.offsets[i + 1]
        assert torch.equal(u[:, q0:q1], pr.st.u), i
        pr.close()
    R.nb.close()


def test_batched_build_rejects_bad_specimen_ids(oracle_mod):
    bt = _small_batch()
    bad = bt.spec.copy()
    bad[3] = 1                             # not a contiguous ascending run
    with pytest.raises(B.SphError) as e:
        B.sph_build_neighbors_batched(dev(bt.X), dev(bt.V), bt.h, dev(bad))
    assert e.value.code == B.SPH_E_ARG
    bad = bt.spec + 1                      # does not start at 0
    with pytest.raises(B.SphError):
        B.sph_build_neighbors_batched(dev(bt.X), dev(bt.V), bt.h, dev(bad))
    nb = B.sph_build_neighbors_batched(dev(bt.X), dev(bt.V), bt.h, dev(bt.spec))
    assert nb.info.n == bt.n
    nb.close()
