"""Tensile necking runs (Sec. 5.1 and 5.2) on the multi-time-step path.

The specimen is stretched by displacement control in N_S load increments.
After each increment the inner loop relaxes it: stress, momentum, damping
sweep and drift.  Every `record_every` increments the run records three
quantities:
* the imposed stretch;
* the reaction force on the right grip, i.e. minus the summed internal
  force m_a a_a of its particles at the last relaxation step;
* the inward displacement of the neck.

At the end it reports the iteration counts as the paper's efficiency tables
do: N_S load increments, N_s relaxation steps and N_d damping sweeps (one
per relaxation step).

Every step runs in libsph.so.  The two observables are dot products of
device arrays with weights from the case description, evaluated with torch
between calls.
"""
from __future__ import annotations

import time

import numpy as np

from . import binding as B


class NeckingRun:
    """One necking specimen (`cases.necking2d` / `cases.necking3d`) on the GPU."""

    def __init__(self, case, prec=B.SPH_F64, record_every=100, use_graph=True, autotune=True):
        import torch
        self.case, self.prec = case, prec
        self.record_every = int(record_every)
        self.use_graph = bool(use_graph)
        if self.record_every < 1:
            raise ValueError("record_every must be positive")
        dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()  # noqa: E731
        self.nb = B.sph_build_neighbors(dev(case.X), dev(case.V), case.h)
        self.perm = self.nb.host("perm").astype(np.int64)
        T = torch.float32 if prec == B.SPH_F32 else torch.float64
        st = B.new_state(self.nb, prec, with_plastic=True, with_acc=True)
        st.flags = dev(case.flags[self.perm])
        st.vgrip = dev(case.vgrip[:, self.perm]).to(T).contiguous()
        self.st = st
        self.mat = B.material(**case.material)
        if autotune:
            dt_s, _ = B.sph_default_steps(case.h, self.mat)
            self.tuning = B.sph_autotune(self.nb, self.mat, st, case.run["eta"], dt_s,
                                         with_adjoint=False).as_dict()
        self.w_acc = dev(case.observable["w_acc"][:, self.perm])
        self.w_u = dev(case.observable["w_u"][:, self.perm])
        self.done = 0

    def observables(self):
        """(reaction force on the right grip, inward neck displacement)."""
        F = float((self.w_acc * self.st.acc.double()).sum().item())
        dr = float((self.w_u * self.st.u).sum().item())
        return F, dr

    def run(self, n_slow=None, progress=None):
        """Run `n_slow` load increments (default: the case's N_S) from the
        current state; returns the history and the iteration counts."""
        import torch
        run = dict(self.case.run)
        total = run["n_slow"] if n_slow is None else int(n_slow)
        inner = int(run["fixed_inner"])
        v_pull = self.case.observable["v_pull"]
        hist = dict(increment=[], stretch=[], reaction=[], radius=[])
        N_s = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        left = total
        while left > 0:
            m = min(self.record_every, left)
            cfg = B.multirate_cfg(**dict(run, n_slow=m), chunk=inner if inner > 0 else 64,
                                  use_graph=int(self.use_graph))
            rc, k, ke, conv, rep = B.sph_advance_multirate(self.nb, self.mat, self.st, cfg)
            N_s += int(k.sum())
            left -= m
            self.done += m
            F, dr = self.observables()
            hist["increment"].append(self.done)
            hist["stretch"].append(2.0 * v_pull * run["dt_slow"] * self.done)
            hist["reaction"].append(F)
            hist["radius"].append(dr)
            if progress:
                progress(self.done, F, dr)
        torch.cuda.synchronize()
        seconds = time.perf_counter() - t0
        pairs = int(self.nb.info.n_pairs)
        rc, bits = B.sph_status(self.nb)
        return dict(N_p=int(self.nb.info.n), N_S=total, N_s=N_s, N_d=N_s, seconds=seconds,
                    pairs=pairs, interactions_per_s=pairs * N_s / seconds if seconds > 0 else None,
                    status_bits=bits, history={k: np.asarray(v) for k, v in hist.items()})

    def close(self):
        if self.nb is not None:
            self.nb.close()
            self.nb = None
