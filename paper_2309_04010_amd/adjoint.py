"""Gradients of the multi-time-step solve for parameter identification.

`MultirateProblem` holds one specimen on the device (neighbourhood, initial
state, flags, loading) with its schedule frozen: the inner step dt_s and the
slow step dt_slow are fixed from the nominal parameters (a gradient with
respect to E or D then differentiates the discrete map the run executes, not
the step-size rule), and after `freeze()` the inner counts are fixed too.
`forward(theta)` runs `sph_advance_multirate` with a tape, `backward(u_bar)`
runs `sph_advance_multirate_backward` and returns d(objective)/d(theta) for
theta = (E, D, C_swell, sigma0, sigma_inf, delta, H).

`solve(theta, problem)` wraps both as a torch.autograd.Function, so any
objective written in torch on the final displacement (a tip displacement, a
mean deflection) back-propagates into theta.  Everything numeric runs in
libsph.so; this module only moves arguments.
"""
from __future__ import annotations

import numpy as np

from . import binding as B

PARAMS = B.GRAD_NAMES  # order of theta


class MultirateProblem:
    def __init__(self, case, prec, k_hist=None, chunk=64, use_graph=0, seg_cap=0,
                 tape_mem_frac=None):
        """k_hist: inner steps whose states the tape holds at once (default:
        the whole slow step); seg_cap: inner checkpoints for longer slow steps
        (reversed in segments).  tape_mem_frac: instead, fit the tape for slow
        steps of k_hist inner steps into this fraction of the device memory
        left free (SphTape.plan)."""
        import torch
        self.case = case
        self.prec = prec
        self.T = torch.float32 if prec == B.SPH_F32 else torch.float64
        dev = lambda a, dt=None: (torch.as_tensor(np.ascontiguousarray(a)).to(dt or torch.float64)  # noqa: E731
                                  .contiguous().cuda())
        self.nb = B.sph_build_neighbors(dev(case.X), dev(case.V), case.h)
        self.perm = self.nb.host("perm").astype(np.int64)
        self.j2 = case.material["model"] == B.SPH_MODEL_J2
        self.diff = case.run["slow_kind"] != B.SPH_SLOW_LOAD
        self.st = B.new_state(self.nb, prec, with_plastic=self.j2, with_diffusion=self.diff)
        self.st.flags = torch.as_tensor(np.ascontiguousarray(case.flags[self.perm])).cuda()
        if case.vgrip is not None:
            self.st.vgrip = dev(case.vgrip[:, self.perm], self.T)
        self.c_init = dev(case.c_init[self.perm], self.T) if self.diff else None
        r = dict(case.run)
        # the schedule is frozen at the library's own step sizes (Sec. 4.1)
        # for the nominal parameters
        dt_s, dt_d = B.sph_default_steps(case.h, B.material(**case.material), r.get("D", 0.0))
        r["dt_s"] = r.get("dt_s") or dt_s
        if self.diff and not r.get("dt_slow"):
            r["dt_slow"] = dt_d
        self.run = r
        self.chunk, self.use_graph = chunk, use_graph
        self.k_sched = None
        n_slow = r["n_slow"]
        if k_hist is None:
            k_hist = r["fixed_inner"] if r.get("fixed_inner", 0) > 0 else r.get("k_max", 0)
        self.adj = B.new_adjoint(self.nb, prec, with_plastic=self.j2, with_diffusion=self.diff)
        if tape_mem_frac is not None:
            free = torch.cuda.mem_get_info()[0]
            k_hist, seg_cap = B.SphTape.plan(self.nb.n, self.nb.dim, prec, k_hist,
                                             tape_mem_frac * free, with_plastic=self.j2)
        self.tape = B.SphTape(self.nb, prec, n_slow, int(k_hist), with_plastic=self.j2,
                              with_diffusion=self.diff, seg_cap=seg_cap)
        self._fwd_id = 0
        self._tape_id = -1
        self.last = None

    # -- parameters ----------------------------------------------------------
    def theta0(self):
        m = self.case.material
        return np.array([m["E"], self.run.get("D", 0.0), m.get("C_swell", 0.0), m.get("sigma0", 0.0),
                         m.get("sigma_inf", 0.0), m.get("delta", 0.0), m.get("H", 0.0)])

    def _material(self, th):
        m = dict(self.case.material)
        m.update(E=th[0], C_swell=th[2], sigma0=th[3], sigma_inf=th[4], delta=th[5], H=th[6])
        return B.material(**m)

    def _cfg(self, th, k_sched=None):
        r = dict(self.run)
        r["D"] = th[1]
        ks = self.k_sched if k_sched is None else k_sched
        return B.multirate_cfg(**r, chunk=self.chunk, use_graph=self.use_graph, k_sched=ks)

    # -- runs --------------------------------------------------------------------
    def reset(self):
        st = self.st
        st.u.zero_()
        st.v.zero_()
        st.PB.zero_()
        if st.plastic is not None:
            st.plastic.zero_()
        if self.diff:
            st.c.copy_(self.c_init)
            st.q.zero_()
            st.p.zero_()

    def forward(self, theta, record=True, k_sched=None):
        """Run from the initial state with parameters theta (and, if given,
        these inner counts instead of the problem's); returns the final u (a
        view of the state: clone it to keep it)."""
        th = np.asarray(theta, dtype=np.float64)
        self.reset()
        cfg = self._cfg(th, k_sched)
        rc, k, ke, conv, rep = B.sph_advance_multirate(self.nb, self._material(th), self.st, cfg,
                                                       tape=self.tape if record else None)
        self._fwd_id += 1
        if record:
            self._tape_id = self._fwd_id
        self.last = dict(rc=rc, k=k.copy(), ke=ke.copy(), conv=conv.copy(), theta=th.copy(),
                         k_sched=None if k_sched is None else np.array(k_sched))
        return self.st.u

    def freeze(self):
        """Fix the inner counts to those of the last forward run."""
        self.k_sched = self.last["k"].copy()

    def backward(self, u_bar, v_bar=None, recompute=False):
        """d(objective)/d(theta) given the objective's derivative with respect
        to the final u (and v).  Requires the last forward run to be taped.
        recompute: re-run every slow step from its checkpoint, also the last
        one, whose inner states the forward run kept (the cost of a slow step
        in a long checkpointed run)."""
        if self._tape_id != self._fwd_id:
            raise RuntimeError("the last forward run was not recorded")
        if recompute:
            self.tape.forget_inner_states()
        th = self.last["theta"]
        a = self.adj.zero_()
        a.u.copy_(u_bar)
        if v_bar is not None:
            a.v.copy_(v_bar)
        B.sph_advance_multirate_backward(self.nb, self._material(th), self.st,
                                         self._cfg(th, self.last["k_sched"]), self.tape, a)
        return a.grad.clone()

    def _ensure_taped(self, fwd_id, theta, k):
        """Make the tape hold forward run `fwd_id` (theta, inner counts k):
        when a later run has replaced it, the same run is recorded again (the
        forward pass is deterministic, so it is the same run)."""
        if self._tape_id == fwd_id:
            return
        self.forward(theta, record=True, k_sched=k)

    def close(self):
        self.nb.close()


def _function():
    import torch

    class MultirateSolve(torch.autograd.Function):
        """u_final = solve(theta): forward and reverse multi-time-step runs."""

        @staticmethod
        def forward(ctx, theta, problem):
            ctx.problem = problem
            ctx.theta_meta = (theta.dtype, theta.device)
            u = problem.forward(theta.detach().double().cpu().numpy()).clone()
            # which run this is: the reverse pass must differentiate this run,
            # even if the problem has run again (another theta) since
            ctx.fwd = (problem._fwd_id, problem.last["theta"].copy(), problem.last["k"].copy())
            return u

        @staticmethod
        def backward(ctx, u_bar):
            ctx.problem._ensure_taped(*ctx.fwd)
            g = ctx.problem.backward(u_bar.contiguous().double())
            dt, dv = ctx.theta_meta
            return g.to(device=dv, dtype=dt), None

    return MultirateSolve


_FN = None


def solve(theta, problem):
    """Final displacement [dim, n] (cell-sorted order) as a differentiable
    function of theta (a float64 tensor of the 7 parameters in PARAMS order)."""
    global _FN
    if _FN is None:
        _FN = _function()
    return _FN.apply(theta, problem)
