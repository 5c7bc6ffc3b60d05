"""Throughput of the multi-time-step TL-SPH hot path on one MI355X.

Workload (default): the 3D membrane plate, 500 x 500 x 4 = 1,000,000
particles (60,256,216 directed neighbour pairs), neo-Hookean solid with the
fluid-pressure coupling, diffusion slow steps, whose gradient runs through
50 checkpointed slow steps x 1000 inner steps.  One bench "step" is one slow
step of that checkpointed adjoint: the diffusion update and 1000 inner steps
of {deformation gradient + stress, pair momentum + kick, implicit pairwise
damping sweep (4 colour passes on the plate), drift + kinetic energy}
forward, then the reverse pass of that slow step, which first re-runs it
from its checkpoint to record H = F - I of every inner step (a long run keeps
only the checkpoints) and then runs the 1000 transposed inner steps and the
transposed diffusion step, giving the gradient of the mean centre deflection
with respect to E, D and C.  FP32 bulk arithmetic with FP64 displacements
and reductions.  The neighbour build (once per configuration,
total-Lagrangian) is setup and is not timed.

Metric: inner-step particle-interactions/s = directed pairs x forward inner
steps / wall time of forward + re-run + reverse, inputs resident in HBM.
Also reported: the same step without the re-run (the inner states kept from
the forward run), the whole 50 x 1000 checkpointed run in FP32 (timed as one
run), the FP32 forward alone, the plain FP64 forward (the baseline of the
speedup), the FP32 state and gradient errors against an FP64 run of the same
step, the roofline of the dominant kernel class (live HIP-event timing of its
launches in the timed region, the calibrated counter traffic, a measured
copy bandwidth), the damping sweep's and the whole inner step's fractions of
the HBM and FP32 roofs, the per-kernel breakdown, the CPU oracle timed on a
bounded sample (one thread, and all host cores), and, outside the timed
region: the slow-step variants (one-way and two-way coupled diffusion), the
cost of the mixture momentum, the necking runs of Sec. 5.1/5.2 with their
iteration counts (N_S, N_s, N_d) and curves, the batched sweep of 64
strips, the 3D J2 bar (100 loading slow steps x 1000 inner steps; FP32 with
eager launches and as a hipGraph, and FP64), and the 2D bar and the swelling
strip over their whole adaptive schedules (eager and as a hipGraph).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--inner M] [--no-cpu]
                  [--no-fp64] [--no-sweep] [--no-coupled] [--necking none|sample|full]
                  [--necking-compare] [--nx N] [--copy-calibration] [--full-adjoint]
                  [--no-full-adjoint] [--no-small] [--neck3d-slow N]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def algorithmic_bytes(kernel, dim, prec_bytes, model_j2=False, n_colors=8):
    """Minimum HBM bytes per particle per launch: each per-particle array the
    kernel must read or write, once (neighbour lists and re-reads of
    neighbours' data are not algorithmic)."""
    T = prec_bytes
    d, dd = dim, dim * dim
    if kernel == "stress":
        b = 8 * d + 8 * d + T + T * dd + T + T * dd      # u, X, V, B0, p | PB
        if model_j2:
            b += 2 * 7 * T
        return b
    if kernel == "momentum":
        return 8 * d + T + T * dd + 2 * T * d + 1         # X, V, PB, v(rw), flags
    if kernel in ("damping", "adj_damping"):
        # per SWEEP (all colour passes): v read and written once and the
        # inverse mass read once; the pair schedule and its coefficients are
        # per-pair data, not algorithmic (the pair geometry is fixed)
        return 2 * T * d + T
    if kernel == "drift_ke":
        return 2 * 8 * d + T * d + 8 + 1                  # u(rw), v, V, flags
    if kernel == "diff_grad":
        return 8 * d + T + T * dd + T + T * d             # X, V, B0, c | q
    if kernel == "diff_div":
        return 8 * d + T + T * dd + T * d + 2 * T + 1 + T  # X, V, B0, q, c(rw), flags | p
    if kernel == "adj_stress":
        # X, V, B0, H_k (the forward's record), w, flags, p | G_bar, p_bar(rw, f64)
        b = 8 * d + T + T * dd + T * dd + T * d + 1 + T + T * dd + 16
        if model_j2:
            b += 7 * T + 2 * 7 * T
        return b
    if kernel == "adj_gather":
        return 8 * d + T + T * dd + 16 * d + 2 * T * d + 1   # X, V, G_bar, u_bar(rw), w(rw), flags
    return 0.0


def flops_per_pair(kernel, dim):
    """Useful floating-point operations per directed pair (FMA = 2); the
    per-particle epilogues (constitutive update and its transpose) are not
    counted."""
    d = dim
    geo = 3 * d + 6            # dx, r^2, sqrt, q, (1-q/2)^3 and scaling
    if kernel == "stress":
        return geo + d + 2 * d * d + 2 * d   # du, outer-product accumulation
    if kernel == "momentum":
        return geo + d * d + 2 * d * d + 2 * d
    if kernel == "adj_stress":
        # e = w grad; V_b a_a - V_a a_b; its outer-product sum with e
        return geo + d + 3 * d + 2 * d * d
    if kernel == "adj_gather":
        # V_b scaling; G_bar_b d; its weighted sum; sum_b V_b grad W
        return geo + 1 + 2 * d * d + 2 * d + 2 * d
    return 0


def roofline_of(kern, prof, dim, n, n_pairs, n_colors, workload_key, passes=1):
    """Roofline of one kernel class from its timed launches: the HBM roof
    (algorithmic bytes per launch) or, when the class's algorithmic intensity
    (flops per byte) exceeds the ridge of the two peaks, the FP32 vector roof
    (useful flops per launch).  The damping classes are taken per sweep of
    `passes` colour passes."""
    launches, kms = prof[kern]
    if kern in ("damping", "adj_damping"):
        launches = launches / passes
    avg_s = kms / 1000.0 / max(launches, 1)
    alg_bytes = algorithmic_bytes(kern, dim, 4, n_colors=n_colors) * n
    flops = flops_per_pair(kern, dim) * n_pairs
    ridge = FP32_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    common = dict(kernel=kern, traffic=measured_traffic(kern, workload_key), avg_launch_us=avg_s * 1e6,
                  launches=launches, alg_bytes_per_launch=alg_bytes, alg_flops_per_launch=flops,
                  intensity_flop_per_byte=flops / alg_bytes if alg_bytes else None)
    if flops and flops / alg_bytes > ridge:
        ach = flops / avg_s / 1e12
        return dict(bound="alu", achieved=ach, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=ach / FP32_PEAK_TFLOPS, **common)
    ach = alg_bytes / avg_s / 1e9
    return dict(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                **common)


def kernel_source_hash():
    """Hash of the HIP sources: counter-based traffic is only reported while
    the kernels are the ones the counters were taken on."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2309_04010_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), or None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash() or t.get("workload") != workload:
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def setup(case, prec, torch, B):
    import numpy as np
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()  # noqa: E731
    nb = B.sph_build_neighbors(dev(case.X), dev(case.V), case.h)
    perm = nb.host("perm").astype(np.int64)
    st = B.new_state(nb, prec, with_diffusion=case.c_init is not None,
                     with_plastic=case.material["model"] == 2)
    st.flags = dev(case.flags[perm])
    if case.c_init is not None:
        T = torch.float32 if prec == B.SPH_F32 else torch.float64
        st.c.copy_(dev(case.c_init[perm]).to(T))
    if case.vgrip is not None:
        T = torch.float32 if prec == B.SPH_F32 else torch.float64
        st.vgrip = dev(case.vgrip[:, perm]).to(T).contiguous()
    return nb, st


def run_gpu(case, prec, steps, warmup, inner, torch, B, profile=True, use_graph=0):
    nb, st = setup(case, prec, torch, B)
    mat = B.material(**case.material)
    run = dict(case.run)
    run.update(n_slow=1, fixed_inner=inner)
    B.sph_autotune(nb, mat, st, run["eta"], B.sph_default_steps(case.h, mat)[0], with_adjoint=False)
    cfg = B.multirate_cfg(**run, chunk=min(inner, 250), use_graph=use_graph)
    for _ in range(warmup):
        B.sph_advance_multirate(nb, mat, st, cfg)
    torch.cuda.synchronize()
    if profile:
        B.sph_profile_enable(nb, True)
    t0 = time.perf_counter()
    total_inner = 0
    for _ in range(steps):
        rc, k, ke, conv, rep = B.sph_advance_multirate(nb, mat, st, cfg)
        total_inner += int(k.sum())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = B.sph_profile_read(nb) if profile else {}
    B.sph_profile_enable(nb, False)
    rc, bits = B.sph_status(nb)
    info = dict(n=nb.info.n, pairs=nb.info.n_pairs, dim=nb.info.dim, n_colors=nb.info.n_colors,
                total_inner=total_inner, seconds=t1 - t0, status=bits,
                u_finite=bool(torch.isfinite(st.u).all().item()))
    nb.close()
    return info, prof


def _oracle_sample(case, openmp, seconds_budget):
    import numpy as np
    import oracle
    o = oracle.Oracle(case.dim, case.X, case.V, case.h, openmp=openmp)
    perm = o.perm
    flags = np.ascontiguousarray(case.flags[perm])
    mat = o.material(**case.material)
    d, n = case.dim, o.n
    u, v = o.arr(d, n), o.arr(d, n)
    c = np.ascontiguousarray(case.c_init[perm]) if case.c_init is not None else None
    q, p = o.arr(d, n), o.arr(n)
    dt, dtd = o.default_steps(mat, case.run["D"])
    rho0 = case.material["rho0"]
    t0 = time.perf_counter()
    if c is not None:
        o.diffusion_step(case.run["D"], dtd, case.run["c_bc"], case.material.get("C_swell", 0.0),
                         case.material.get("c0", 0.0), c, q, p, flags)
    steps = 0
    while True:
        o.solid_step(mat, dt, u, v, p=p, flags=flags)
        o.damping_sweep(rho0, case.run["eta"], dt, v, flags)
        o.drift_ke(rho0, dt, u, v, flags)
        steps += 1
        if time.perf_counter() - t0 >= seconds_budget:
            break
    t1 = time.perf_counter()
    return o.n_pairs * steps / (t1 - t0), steps, t1 - t0, n


def cpu_baseline(case, seconds_budget=15.0, all_cores_budget=10.0):
    """The oracle as it stands, single-threaded, on the same workload: build
    (untimed), one diffusion step, then inner steps until the budget is
    spent (at least one).  Beside it, the oracle's OpenMP build on all host
    cores (per-particle loops and the anchors of one damping colour in
    parallel; the same values)."""
    val, steps, sec, n = _oracle_sample(case, False, seconds_budget)
    out = dict(value=val, unit="interactions/s", cores=1, kind="oracle",
               sample=f"{case.name} full size ({n} particles): one diffusion step + {steps} inner "
                      f"steps, single thread, {sec:.1f} s (build not timed)")
    try:
        ncores = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
        val2, steps2, sec2, _ = _oracle_sample(case, True, all_cores_budget)
        out["all_cores"] = dict(value=val2, unit="interactions/s", cores=ncores, kind="oracle (OpenMP build)",
                                sample=f"one diffusion step + {steps2} inner steps, {ncores} threads, "
                                       f"{sec2:.1f} s")
    except OSError as e:      # no OpenMP runtime on the host: the single-thread figure stands
        out["all_cores"] = dict(error=str(e))
    return out


def run_adjoint(case, prec, steps, warmup, inner, torch, B, A, profile=True, taped_steps=2):
    """One slow step of the checkpointed adjoint, `steps` times: forward
    (checkpoint + taped inner states), then the reverse pass with the slow
    step re-run from its checkpoint (recompute), as every slow step of a long
    checkpointed run costs.  After the timed region, `taped_steps` more
    forward + reverse steps without the re-run.  Returns timing, the final u
    of the last forward run and the gradient."""
    import numpy as np
    import dataclasses
    run = dict(case.run)
    run.update(n_slow=1, fixed_inner=inner)
    c = dataclasses.replace(case, run=run)
    # the recorded inner states of a slow step take (dim^2) values per
    # particle per inner step: where they do not fit, the reverse pass goes
    # in segments (two-level checkpointing)
    torch.cuda.empty_cache()
    pr = A.MultirateProblem(c, prec, k_hist=inner, chunk=min(inner, 250), tape_mem_frac=0.8)
    segments = pr.tape.seg_cap + 1
    if segments > 1:
        taped_steps = 0
    th = pr.theta0()
    tuning = B.sph_autotune(pr.nb, pr._material(th), pr.st, run["eta"], pr.run["dt_s"],
                            with_adjoint=True).as_dict()
    idx = pr.perm.argsort()[case.observable["J_index"]]
    w = torch.zeros((case.dim, case.n), dtype=torch.float64, device="cuda")
    w[case.observable["J_component"], torch.as_tensor(idx).cuda()] = 1.0 / len(idx)
    for _ in range(warmup):
        pr.forward(th)
        pr.backward(w, recompute=True)
    torch.cuda.synchronize()
    breakdown, dominant = {}, None
    if profile:
        # one more (untimed) forward + reverse without the re-run, with events
        # around every launch: the per-kernel breakdown of one inner step
        # forward and in reverse, and the dominant kernel class by total time
        B.sph_profile_classes(pr.nb, None)
        B.sph_profile_enable(pr.nb, True)
        pr.forward(th)
        pr.backward(w)
        breakdown = B.sph_profile_read(pr.nb)
        B.sph_profile_enable(pr.nb, False)
        dominant = max(breakdown, key=lambda k: breakdown[k][1])
        # the timed region records events around the dominant class only
        # (each event adds queue time between kernels)
        B.sph_profile_classes(pr.nb, [dominant])
        B.sph_profile_enable(pr.nb, True)
    t0 = time.perf_counter()
    t_fwd = 0.0
    total_inner = 0
    g = None
    for _ in range(steps):
        ta = time.perf_counter()
        pr.forward(th)
        torch.cuda.synchronize()
        t_fwd += time.perf_counter() - ta
        total_inner += int(pr.last["k"].sum())
        g = pr.backward(w, recompute=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = B.sph_profile_read(pr.nb) if profile else {}
    B.sph_profile_enable(pr.nb, False)
    B.sph_profile_classes(pr.nb, None)
    # the same step with the inner states kept from the forward run (no
    # re-run): the forward + reverse cost of one inner step
    t_taped = 0.0
    if taped_steps:
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(taped_steps):
            pr.forward(th)
            pr.backward(w)
        torch.cuda.synchronize()
        t_taped = (time.perf_counter() - ta) / taped_steps
    rc, bits = B.sph_status(pr.nb)
    u = pr.st.u.detach().double().cpu().numpy()
    info = dict(n=pr.nb.info.n, pairs=pr.nb.info.n_pairs, dim=pr.nb.info.dim,
                n_colors=pr.nb.info.n_colors, total_inner=total_inner, seconds=t1 - t0,
                seconds_forward=t_fwd, seconds_taped_step=t_taped,
                damping_passes=int(sum(1 for k in range(8) if pr.nb.info.color_off[k + 1] >
                                       pr.nb.info.color_off[k])),
                status=bits, grad=g.cpu().numpy(),
                J=float((pr.st.u * w).sum().item()), u=u,
                u_finite=bool(np.isfinite(u).all()), tuning=tuning, breakdown=breakdown,
                dominant=dominant, tape_k_hist=pr.tape.k_hist_cap, tape_segments=segments)
    pr.close()
    del pr
    torch.cuda.empty_cache()
    return info, prof


def run_coupled(case, torch, B, reps=10):
    """The slow step's variants on the same deformed FP32 state: the
    reference-configuration step, and the two-way coupled step with the
    linear and the nonlinear flux.  Per variant: average wall time of one
    slow step over `reps` back-to-back calls, and the per-class kernel times
    of one further profiled call."""
    import numpy as np
    nb, st = setup(case, B.SPH_F32, torch, B)
    mat = B.material(**case.material)
    run = dict(case.run)
    run.update(n_slow=1, fixed_inner=200)
    B.sph_advance_multirate(nb, mat, st, B.multirate_cfg(**run, chunk=200, use_graph=0))
    Dc, dtd, cbc = run["D"], B.sph_default_steps(case.h, mat, run["D"])[1], run["c_bc"]
    c_keep = st.c.clone()
    variants = {
        "reference": lambda: B.sph_diffusion_step(nb, mat, st, Dc, dtd, cbc),
        "coupled_linear": lambda: B.sph_diffusion_step_coupled(nb, mat, st, Dc, dtd, cbc, 0),
        "coupled_nonlinear": lambda: B.sph_diffusion_step_coupled(nb, mat, st, Dc, dtd, cbc, 1),
    }
    out = {}
    for name, call in variants.items():
        st.c.copy_(c_keep)
        call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            call()
        torch.cuda.synchronize()
        us = 1e6 * (time.perf_counter() - t0) / reps
        B.sph_profile_enable(nb, True)
        call()
        prof = B.sph_profile_read(nb)
        B.sph_profile_enable(nb, False)
        out[name] = dict(us_per_slow_step=us,
                         kernels_us={k: 1000.0 * ms for k, (c, ms) in prof.items() if c})
    out["c_finite"] = bool(torch.isfinite(st.c).all().item())
    out["note"] = ("one slow step on the relaxed plate (200 inner steps), FP32; "
                   "diff_grad of the coupled step includes its deformation pass")
    nb.close()
    return out


def run_necking(name, prec, n_slow, torch, B, record_every=100):
    """A necking run (Sec. 5.1 / 5.2) of `n_slow` of the case's load
    increments on the GPU: iteration counts as in the paper's efficiency
    tables, wall time, and the reaction-force / neck-displacement curve."""
    import numpy as np
    from paper_2309_04010_amd import cases
    from paper_2309_04010_amd.necking import NeckingRun
    c = cases.by_name(name)
    r = NeckingRun(c, prec, record_every=record_every)
    def progress(done, F, dr):
        if done % 2000 == 0:
            print(f"[bench] {name}: {done} load increments, reaction {F:.4g}, neck {dr:.4g}", flush=True)

    try:
        res = r.run(n_slow=n_slow, progress=progress)
    finally:
        r.close()
    h = res["history"]
    dt_s = B.sph_default_steps(c.h, B.material(**c.material))[0]
    t_end = c.run["dt_slow"] * c.run["n_slow"]
    ipk = int(np.argmax(h["reaction"]))
    stride = max(1, len(h["increment"]) // 20)
    return dict(
        workload=f"{name}: {res['N_p']} particles, {res['pairs']} directed pairs, J2 (necking table), "
                 f"{c.run['fixed_inner']} relaxation steps per load increment, "
                 f"{'FP64' if prec == B.SPH_F64 else 'FP32 bulk / FP64 displacement'}",
        N_p=res["N_p"], N_S=res["N_S"], N_s=res["N_s"], N_d=res["N_d"],
        N_S_paper_run=c.run["n_slow"], fraction_of_paper_run=res["N_S"] / c.run["n_slow"],
        straightforward_N_s=t_end / dt_s,
        seconds=res["seconds"], us_per_inner_step=1e6 * res["seconds"] / max(res["N_s"], 1),
        interactions_per_s=res["interactions_per_s"], status_bits=res["status_bits"],
        reaction_unit="N per metre of depth" if c.dim == 2 else "N",
        peak_reaction=float(h["reaction"][ipk]), stretch_at_peak=float(h["stretch"][ipk]),
        final_stretch=float(h["stretch"][-1]), final_reaction=float(h["reaction"][-1]),
        final_neck_displacement=float(h["radius"][-1]),
        curve_stretch_reaction_neck=[[float(h["stretch"][i]), float(h["reaction"][i]), float(h["radius"][i])]
                                     for i in range(stride - 1, len(h["increment"]), stride)])


def run_mixture(case, torch, B, inner=200):
    """Forward cost of the mixture momentum on the same workload (FP32): one
    two-way coupled (nonlinear) diffusion slow step and `inner` fast steps,
    dry (rho_l0 = 0) and with the fluid's momentum and mass (rho_l0 = 1000);
    per inner step: wall time of the run (after a warm-up run) and the
    per-class kernel times of one profiled run."""
    import numpy as np
    out = {}
    for name, rho_l0 in (("dry", 0.0), ("mixture", 1000.0)):
        nb, st = setup(case, B.SPH_F32, torch, B)
        mat = B.material(**dict(case.material, rho_l0=rho_l0))
        run = dict(case.run, n_slow=1, fixed_inner=inner, slow_kind=B.SPH_SLOW_DIFFUSION_COUPLED)
        cfg = B.multirate_cfg(**run, chunk=inner, use_graph=0, diff_nonlinear=1)
        c_keep = st.c.clone()
        B.sph_advance_multirate(nb, mat, st, cfg)
        torch.cuda.synchronize()
        st.c.copy_(c_keep)
        t0 = time.perf_counter()
        B.sph_advance_multirate(nb, mat, st, cfg)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        B.sph_profile_enable(nb, True)
        B.sph_advance_multirate(nb, mat, st, cfg)
        prof = B.sph_profile_read(nb)
        B.sph_profile_enable(nb, False)
        out[name] = dict(us_per_inner_step=1e6 * sec / inner,
                         kernels_us={k: 1000.0 * ms / c for k, (c, ms) in prof.items() if c},
                         u_finite=bool(torch.isfinite(st.u).all().item()))
        nb.close()
    out["note"] = ("FP32, eager launches; kernels_us: average per launch (damping: per colour pass; "
                   "diff_*: the slow step's)")
    return out


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of `nbytes` (torch's copy kernel), timed
    with events: the practical HBM ceiling beside the published peak."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1000.0 / reps
    del a, b
    return dict(GBps=2.0 * nbytes / s / 1e9, bytes=nbytes, note="read + write of a 1 GiB copy")


def run_full_adjoint(case, torch, B, A, n_slow=50, inner=1000, with_fp64=False):
    """The whole checkpointed adjoint run of the plate: `n_slow` diffusion
    slow steps x `inner` inner steps forward (one checkpoint per slow step,
    the inner states of the last one), then the reverse pass, which re-runs
    each earlier slow step from its checkpoint to record its inner states.
    FP32, and with `with_fp64` FP64 for the gradient's error."""
    import dataclasses
    out = {}
    precs = ((B.SPH_F32, "f32"), (B.SPH_F64, "f64")) if with_fp64 else ((B.SPH_F32, "f32"),)
    for prec, tag in precs:
        run = dict(case.run)
        run.update(n_slow=n_slow, fixed_inner=inner)
        c = dataclasses.replace(case, run=run)
        pr = A.MultirateProblem(c, prec, k_hist=inner, chunk=min(inner, 250))
        th = pr.theta0()
        B.sph_autotune(pr.nb, pr._material(th), pr.st, run["eta"], pr.run["dt_s"], with_adjoint=True)
        idx = pr.perm.argsort()[case.observable["J_index"]]
        w = torch.zeros((case.dim, case.n), dtype=torch.float64, device="cuda")
        w[case.observable["J_component"], torch.as_tensor(idx).cuda()] = 1.0 / len(idx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pr.forward(th)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        print(f"[bench] full adjoint {tag}: forward {t1 - t0:.1f} s", flush=True)
        J = float((pr.st.u * w).sum().item())
        g = pr.backward(w).cpu().numpy()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        print(f"[bench] full adjoint {tag}: reverse {t2 - t1:.1f} s", flush=True)
        total_inner = int(pr.last["k"].sum())
        out[tag] = dict(seconds_forward=t1 - t0, seconds_reverse=t2 - t1, inner_steps=total_inner,
                        interactions_per_s=pr.nb.info.n_pairs * total_inner / (t2 - t0), J=J,
                        grad={B.GRAD_NAMES[i]: float(g[i]) for i in (B.SPH_GRAD_E, B.SPH_GRAD_D,
                                                                      B.SPH_GRAD_C)},
                        grad_finite=bool(all(abs(x) < float("inf") for x in g)))
        pr.close()
    if with_fp64:
        out["grad_rel_err_f32"] = {k: abs(out["f32"]["grad"][k] - out["f64"]["grad"][k]) /
                                   abs(out["f64"]["grad"][k]) for k in out["f64"]["grad"]}
        out["J_rel_err_f32"] = abs(out["f32"]["J"] - out["f64"]["J"]) / abs(out["f64"]["J"])
    out["workload"] = (f"plate3d {case.shape[0]}x{case.shape[1]}x{case.shape[2]}, {n_slow} diffusion slow steps x "
                       f"{inner} inner steps, forward with checkpoints, then the reverse pass "
                       f"(d mean centre deflection / d(E, D, C))")
    return out


def run_small_configs(torch, B):
    """The 2D bar (plain FP64) and the swelling strip (FP32, and FP64 as its
    reference) over their whole schedules of 100 slow steps, the inner
    counts chosen by the kinetic-energy stop test."""
    import numpy as np
    from paper_2309_04010_amd import cases
    out = {}
    runs = (("bar2d", cases.bar2d(), B.SPH_F64), ("strip2d_f32", cases.strip2d(), B.SPH_F32),
            ("strip2d_f64", cases.strip2d(), B.SPH_F64))
    u_end = {}
    for tag, c, prec in runs:
        res = {}
        for g in (0, 1):
            nb, st = setup(c, prec, torch, B)
            cfg = B.multirate_cfg(**c.run, chunk=250, use_graph=g)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, k, ke, conv, rep = B.sph_advance_multirate(nb, B.material(**c.material), st, cfg)
            torch.cuda.synchronize()
            res[g] = (time.perf_counter() - t0, k, conv, st.u.double().cpu().numpy())
            n, pairs = nb.info.n, nb.info.n_pairs
            nb.close()
        sec, k, conv, u_end[tag] = res[0]
        gsec = res[1][0]
        out[tag] = dict(particles=n, pairs=pairs, N_S=int(len(k)), N_s=int(k.sum()),
                        k_min=int(k.min()), k_max=int(k.max()), converged=int(conv.sum()), seconds=sec,
                        interactions_per_s=pairs * float(k.sum()) / sec, seconds_graph=gsec,
                        interactions_per_s_graph=pairs * float(k.sum()) / gsec,
                        graph_equals_eager=bool(np.array_equal(res[1][1], k) and
                                                np.array_equal(res[1][3], u_end[tag])))
    out["strip2d_f32_u_rel_err"] = float(np.abs(u_end["strip2d_f32"] - u_end["strip2d_f64"]).max() /
                                         np.abs(u_end["strip2d_f64"]).max())
    out["note"] = ("bar2d: 40x8, LE, 100 loading slow steps; strip2d: 200x10, NH + swelling, 100 diffusion "
                   "slow steps; inner counts by the kinetic-energy stop test (N_s inner steps in all); "
                   "seconds: eager launches, seconds_graph: the inner steps replayed as a hipGraph (its "
                   "capture included)")
    return out


def run_sweep(torch, B, launches=2):
    """The batched parameter sweep: 64 strips of log-uniform size (1e3-5e4
    particles), each with its own E and D, 10 diffusion slow steps x 200
    inner steps, forward and reverse recorded as one hipGraph and launched
    whole; per-specimen gradients of the mid-span top deflection."""
    import numpy as np
    from paper_2309_04010_amd import cases
    bt = cases.batch(cases.strips_sweep(64))
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()  # noqa: E731
    t0 = time.perf_counter()
    nb = B.sph_build_neighbors_batched(dev(bt.X), dev(bt.V), bt.h, dev(bt.spec))
    t_build = time.perf_counter() - t0
    perm = nb.host("perm").astype(np.int64)
    prec = B.SPH_F32
    st = B.new_state(nb, prec, with_diffusion=True)
    st.flags = dev(bt.flags[perm])
    c0 = dev(bt.c_init[perm]).float()
    grad = torch.zeros((len(bt.cases), B.SPH_NGRAD), dtype=torch.float64, device="cuda")
    batch = B.SphBatch(bt.E, bt.D, grad=grad)      # per-specimen steps: the library's
    run = dict(bt.run)
    cfg = B.multirate_cfg(**run, batch=batch)
    mat = B.material(**bt.material)
    tape = B.SphTape(nb, prec, run["n_slow"], run["fixed_inner"], with_diffusion=True)
    adj = B.new_adjoint(nb, prec, with_diffusion=True)
    # objective: mid-span top deflection of every strip
    w = torch.zeros((2, bt.n), dtype=torch.float64, device="cuda")
    inv = np.argsort(perm)
    for i, c in enumerate(bt.cases):
        j = bt.offsets[i] + c.observable["J_index"]
        w[1, torch.as_tensor(inv[j]).cuda()] = 1.0 / len(j)
    dt_min = min(B.sph_default_steps(bt.h, B.material(**dict(bt.material, E=E)))[0] for E in bt.E)
    B.sph_autotune(nb, mat, st, run["eta"], dt_min, with_adjoint=True)

    def launch():
        st.u.zero_()
        st.v.zero_()
        st.c.copy_(c0)
        adj.zero_()
        adj.u.copy_(w)
        grad.zero_()
        return B.sph_advance_multirate_graph(nb, mat, st, cfg, tape, adj)

    t0 = time.perf_counter()
    launch()                                  # records and instantiates the graph
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(launches):
        k = launch()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / launches
    P = nb.info.n_pairs
    inner = int(np.sum(k))
    g = grad.cpu().numpy()
    out = dict(workload=f"64 strips, {bt.n} particles in total ({int(np.diff(bt.offsets).min())}.."
                        f"{int(np.diff(bt.offsets).max())} per strip), {P} directed pairs, "
                        f"{run['n_slow']} slow x {run['fixed_inner']} inner steps, forward + reverse, FP32",
               value=P * inner / t, unit="interactions/s (forward inner steps / forward+reverse time)",
               seconds_per_launch=t, seconds_first_launch_incl_recording=t_first,
               build_seconds=t_build,
               dJ_dE_first3=g[:3, B.SPH_GRAD_E].tolist(), dJ_dD_first3=g[:3, B.SPH_GRAD_D].tolist(),
               grad_finite=bool(np.isfinite(g).all()))
    nb.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--inner", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--nx", type=int, default=500)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-coupled", action="store_true")
    ap.add_argument("--necking", choices=["none", "sample", "full"], default="sample",
                    help="necking runs: sample = the full 2D run and the first 1000 load increments "
                         "of the 3D one; full = both full runs")
    ap.add_argument("--no-neck3d", action="store_true", help="skip the neck3d, bar2d and strip2d runs")
    ap.add_argument("--no-small", action="store_true", help="skip the bar2d and strip2d runs")
    ap.add_argument("--neck3d-slow", type=int, default=100,
                    help="loading slow steps of the neck3d runs (1000 inner steps each)")
    ap.add_argument("--full-adjoint", action="store_true",
                    help="run the whole checkpointed adjoint (50 slow x 1000 inner steps) in FP64 as "
                         "well as in FP32 (the FP32 run is in the default bench)")
    ap.add_argument("--no-full-adjoint", action="store_true",
                    help="skip the whole checkpointed adjoint run")
    ap.add_argument("--necking-compare", action="store_true",
                    help="run each necking case in FP32 and in FP64 and report how far the FP32 "
                         "curves deviate")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2309_04010_amd import adjoint as A
    from paper_2309_04010_amd import binding as B
    from paper_2309_04010_amd import cases

    torch.cuda.set_device(0)
    case = cases.plate3d(nx=args.nx, ny=args.nx)
    print(f"[bench] workload {case.name} n={case.n} inner={args.inner} steps={args.steps}", flush=True)
    adj32, prof32 = run_adjoint(case, B.SPH_F32, args.steps, args.warmup, args.inner, torch, B, A)
    print(f"[bench] fp32 forward+adjoint done: {adj32['seconds']:.3f} s", flush=True)
    P = adj32["pairs"]
    value = P * adj32["total_inner"] / adj32["seconds"]
    ms_per_step = 1000.0 * adj32["seconds"] / args.steps
    fwd32 = dict(value=P * adj32["total_inner"] / adj32["seconds_forward"],
                 ms_per_step=1000.0 * adj32["seconds_forward"] / args.steps)
    taped = None
    if adj32["seconds_taped_step"] > 0:
        taped = dict(value=P * args.inner / adj32["seconds_taped_step"],
                     ms_per_step=1000.0 * adj32["seconds_taped_step"],
                     note="forward + reverse of one slow step with the inner states kept from the "
                          "forward run (no re-run); measured after the timed region")

    fp64 = None
    accuracy = None
    if not args.no_fp64:
        info64, _ = run_gpu(case, B.SPH_F64, max(1, args.steps - 1), args.warmup, args.inner,
                            torch, B, profile=False)
        print(f"[bench] fp64 plain done: {info64['seconds']:.3f} s", flush=True)
        v64 = P * info64["total_inner"] / info64["seconds"]
        fp64 = dict(value=v64, ms_per_step=1000.0 * info64["seconds"] / max(1, args.steps - 1),
                    status=info64["status"])
        # accuracy of the FP32 step (state and gradient) against the same step in FP64
        adj64, _ = run_adjoint(case, B.SPH_F64, 1, 0, args.inner, torch, B, A, profile=False)
        print("[bench] fp64 forward+adjoint reference done", flush=True)
        ue = float(np.abs(adj32["u"] - adj64["u"]).max() / np.abs(adj64["u"]).max())
        gr = {B.GRAD_NAMES[i]: dict(fp32=float(adj32["grad"][i]), fp64=float(adj64["grad"][i]),
                                    rel_err=float(abs(adj32["grad"][i] - adj64["grad"][i]) /
                                                  abs(adj64["grad"][i])))
              for i in (B.SPH_GRAD_E, B.SPH_GRAD_D, B.SPH_GRAD_C)}
        accuracy = dict(reference="the same step on the FP64 GPU path (itself within 1e-10 of the "
                                  "FP64 oracle in the parity tests)",
                        u_rel_err=ue, J_fp32=adj32["J"], J_fp64=adj64["J"], grad=gr,
                        fp64_tape_segments=adj64["tape_segments"])

    # dominant kernel class (by total time in the profiled untimed step),
    # timed with HIP events around its launches in the timed region
    kern = adj32["dominant"]
    nper = adj32["n"]
    seg_note = ("" if adj32["tape_segments"] == 1 else
                f" in {adj32['tape_segments']} segments of {adj32['tape_k_hist']} inner steps")
    workload_key = f"plate3d-{args.nx}x{args.nx}x4-fp32"
    copy_bw = copy_bandwidth(torch)
    npass = adj32["damping_passes"]
    roofline = roofline_of(kern, prof32, adj32["dim"], nper, P, adj32["n_colors"], workload_key,
                           passes=npass)
    roofline.update(copy_GBps=copy_bw["GBps"])
    if roofline["bound"] == "hbm":
        roofline["frac_of_copy"] = roofline["achieved"] / copy_bw["GBps"]
    # the damping sweep beside it, from the profiled step (HBM view, per
    # sweep: v read and written once, the inverse mass read once)
    damping_view = None
    if kern != "damping" and adj32["breakdown"].get("damping", (0, 0))[0]:
        damping_view = roofline_of("damping", adj32["breakdown"], adj32["dim"], nper, P,
                                   adj32["n_colors"], workload_key, passes=npass)
        damping_view["frac_of_copy"] = damping_view["achieved"] / copy_bw["GBps"]
        damping_view["passes_per_sweep"] = npass
        damping_view["per"] = "sweep (all colour passes)"
        damping_view["measured"] = "the profiled step outside the timed region"
    # the whole inner step, forward + reverse, against the algorithmic totals
    # of the path: 883 B per particle (276 forward, 2.2x that in reverse) and
    # 321 flop per directed pair (107 forward, 2x that in reverse)
    whole_step = None
    if taped:
        t_inner = adj32["seconds_taped_step"] / args.inner
        hbm = 883.0 * nper / t_inner / 1e9
        alu = 321.0 * P / t_inner / 1e12
        whole_step = dict(us_per_inner_step=1e6 * t_inner, bytes_per_particle=883, flops_per_pair=321,
                          hbm_GBps=hbm, hbm_frac=hbm / HBM_PEAK_GBS, fp32_TFLOPs=alu,
                          fp32_frac=alu / FP32_PEAK_TFLOPS,
                          note="forward + reverse inner step (taped step / inner steps) against the "
                               "algorithmic bytes and flops of the path")
    kernels = {}
    for k, (c, ms) in adj32["breakdown"].items():
        if not c:
            continue
        kernels[k] = dict(launches=c, avg_us=1000.0 * ms / c, total_ms=ms)
        ab = algorithmic_bytes(k, adj32["dim"], 4) * nper
        if ab and k in ("damping", "adj_damping"):
            kernels[k]["avg_us_per_sweep"] = 1000.0 * ms / (c / npass)
            kernels[k]["alg_GBps"] = ab / (ms / 1000.0 / (c / npass)) / 1e9
        elif ab:
            kernels[k]["alg_GBps"] = ab / (ms / 1000.0 / c) / 1e9
        fl = flops_per_pair(k, adj32["dim"]) * P
        if fl:
            kernels[k]["alu_TFLOPs"] = fl / (ms / 1000.0 / c) / 1e12

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    coupled = None
    if not args.no_coupled:
        coupled = run_coupled(case, torch, B)
        print("[bench] slow-step variants done", flush=True)

    mixture = None
    if not args.no_coupled:
        mixture = run_mixture(case, torch, B)
        print("[bench] mixture momentum done", flush=True)

    necking = None
    if args.necking != "none":
        necking = {}
        for name, n3 in (("necking2d", None), ("necking3d", None if args.necking == "full" else 1000)):
            necking[name] = run_necking(name, B.SPH_F64 if name == "necking2d" else B.SPH_F32, n3,
                                        torch, B)
            print(f"[bench] {name} done: {necking[name]['seconds']:.1f} s", flush=True)
            if args.necking_compare:
                other = B.SPH_F32 if name == "necking2d" else B.SPH_F64
                r2 = run_necking(name, other, n3, torch, B)
                print(f"[bench] {name} in the other precision done: {r2['seconds']:.1f} s", flush=True)
                r32, r64 = (r2, necking[name]) if other == B.SPH_F32 else (necking[name], r2)
                c32 = np.array(r32["curve_stretch_reaction_neck"])
                c64 = np.array(r64["curve_stretch_reaction_neck"])
                necking[name]["fp32_vs_fp64"] = dict(
                    seconds_fp32=r32["seconds"], seconds_fp64=r64["seconds"],
                    reaction_max_rel_dev=float(np.abs(c32[:, 1] - c64[:, 1]).max() / np.abs(c64[:, 1]).max()),
                    neck_max_rel_dev=float(np.abs(c32[:, 2] - c64[:, 2]).max() / np.abs(c64[:, 2]).max()),
                    peak_reaction_fp32=r32["peak_reaction"], peak_reaction_fp64=r64["peak_reaction"],
                    final_neck_fp32=r32["final_neck_displacement"],
                    final_neck_fp64=r64["final_neck_displacement"])

    full_adjoint = None
    if not args.no_full_adjoint:
        full_adjoint = run_full_adjoint(case, torch, B, A, inner=args.inner, with_fp64=args.full_adjoint)
        print("[bench] whole checkpointed adjoint done", flush=True)

    small = None if (args.no_neck3d or args.no_small) else run_small_configs(torch, B)
    if small:
        print("[bench] bar2d / strip2d done", flush=True)

    # the 3D J2 bar (100 x 20 x 20): its whole schedule, 100 loading slow steps
    # x 1000 inner steps, forward, in FP32 and in plain FP64
    neck = None
    if not args.no_neck3d:
        nc = cases.neck3d()
        neck = {"workload": f"neck3d 100x20x20 ({nc.n} particles), J2, {args.neck3d_slow} loading slow "
                            f"steps x 1000 inner steps, forward"}
        for prec, tag in ((B.SPH_F32, "f32"), (B.SPH_F64, "f64")):
            info, _ = run_gpu(nc, prec, args.neck3d_slow, 1, 1000, torch, B, profile=False)
            neck[tag] = dict(seconds=info["seconds"], inner_steps=info["total_inner"], pairs=info["pairs"],
                             interactions_per_s=info["pairs"] * info["total_inner"] / info["seconds"],
                             status=info["status"], u_finite=info["u_finite"])
            print(f"[bench] neck3d {tag} done: {info['seconds']:.1f} s", flush=True)
        neck["f32_over_f64"] = neck["f32"]["interactions_per_s"] / neck["f64"]["interactions_per_s"]
        info, _ = run_gpu(nc, B.SPH_F32, args.neck3d_slow, 1, 1000, torch, B, profile=False, use_graph=1)
        neck["f32_graph"] = dict(seconds=info["seconds"], inner_steps=info["total_inner"],
                                 interactions_per_s=info["pairs"] * info["total_inner"] / info["seconds"],
                                 status=info["status"], u_finite=info["u_finite"])
        print(f"[bench] neck3d f32 graph done: {info['seconds']:.1f} s", flush=True)

    sweep = None
    if not args.no_sweep:
        sweep = run_sweep(torch, B)
        print(f"[bench] batched sweep done: {sweep['seconds_per_launch']:.3f} s per launch", flush=True)

    cpu = None if args.no_cpu else cpu_baseline(case)
    out = {
        "metric": "inner-step particle-interactions/s FP32+adjoint vs FP64 plain; %HBM roofline",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"plate3d {args.nx}x{args.nx}x4 membrane ({adj32['n']} particles, {P} directed "
                        f"pairs), neo-Hookean + fluid pressure, checkpointed adjoint; per step one "
                        f"slow step of it: a diffusion slow step + {args.inner} inner steps forward, "
                        f"then its reverse pass (the slow step re-run from its checkpoint with "
                        f"H = F - I recorded{seg_note}, {args.inner} transposed inner steps, the "
                        f"transposed diffusion "
                        f"step) for d(mean centre deflection)/d(E, D, C); FP32 bulk / FP64 "
                        f"displacement",
            "headline": "per slow step of the 50 x 1000 checkpointed adjoint, re-run included; "
                        "full_adjoint times the whole run",
            "adjoint": True,
            "tape_segments": adj32["tape_segments"],
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "roofline_damping": damping_view,
        "whole_step": whole_step,
        "taped_step": taped,
        "kernels": kernels,
        "kernels_measured": "one profiled step after the warmup, outside the timed region (HIP events "
                            "around every launch, around every sweep for the damping classes, whose "
                            "passes share the sweep's time); the timed region times the roofline "
                            "kernel class only",
        "fp32_forward_only": fwd32,
        "fp64_plain": fp64,
        "speedup_vs_fp64_plain": (value / fp64["value"]) if fp64 else None,
        "accuracy": accuracy,
        "batched_sweep": sweep,
        "slow_step_variants": coupled,
        "mixture_momentum": mixture,
        "necking": necking,
        "full_adjoint": full_adjoint,
        "neck3d": neck,
        "bar2d_strip2d": small,
        "gradient": {B.GRAD_NAMES[i]: float(adj32["grad"][i])
                     for i in (B.SPH_GRAD_E, B.SPH_GRAD_D, B.SPH_GRAD_C)},
        "cpu_baseline": cpu,
        "launch_shapes": adj32["tuning"],
        "status_bits": adj32["status"],
        "u_finite": adj32["u_finite"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
