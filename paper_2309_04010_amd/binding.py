"""Thin ctypes binding of libsph.so (include/sph.h), same names as the C ABI.

Argument marshalling only: every step of the computation runs in the HIP
kernels of libsph.so.  PyTorch supplies device memory (tensors) and the stream
(torch's current stream).  If the library is missing, or no GPU is visible,
calls raise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph.so")

SPH_OK, SPH_E_ARG, SPH_E_CAPACITY, SPH_E_DEVICE, SPH_E_NUMERIC, SPH_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
SPH_W_NOT_CONVERGED = 1
SPH_F32, SPH_F64 = 0, 1
SPH_MODEL_LE, SPH_MODEL_NH, SPH_MODEL_J2 = 0, 1, 2
SPH_SLOW_LOAD, SPH_SLOW_DIFFUSION, SPH_SLOW_DIFFUSION_COUPLED = 0, 1, 2
SPH_FLAG_FIXED, SPH_FLAG_CDIR, SPH_FLAG_GRIP = 1, 2, 4

EXPORTED = [
    "sph_build_neighbors", "sph_nbr_destroy", "sph_nbr_query", "sph_solid_relax_step",
    "sph_damping_sweep", "sph_drift_ke", "sph_load_step", "sph_diffusion_step", "sph_diffusion_step_coupled",
    "sph_advance_multirate", "sph_status", "sph_profile_enable", "sph_profile_classes", "sph_profile_read",
    "sph_last_error", "sph_solid_relax_step_vjp", "sph_damping_sweep_vjp", "sph_drift_vjp",
    "sph_diffusion_step_vjp", "sph_diffusion_step_coupled_vjp", "sph_advance_multirate_backward",
    "sph_constitutive",
    "sph_constitutive_vjp", "sph_build_neighbors_batched", "sph_advance_multirate_graph",
    "sph_autotune", "sph_set_tuning", "sph_get_tuning", "sph_default_steps", "sph_drift_ke_noalloc",
    "sph_workspace_size", "sph_set_workspace",
]
SPH_KERNEL_NAMES = ["stress", "momentum", "damping", "drift_ke", "diff_grad", "diff_div", "load",
                    "adj_stress", "adj_gather", "adj_damping"]
SPH_GRAD_E, SPH_GRAD_D, SPH_GRAD_C, SPH_GRAD_S0, SPH_GRAD_SINF, SPH_GRAD_DELTA, SPH_GRAD_H = range(7)
SPH_NGRAD = 7
GRAD_NAMES = ["E", "D", "C_swell", "sigma0", "sigma_inf", "delta", "H"]


class SphError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sph error {code}: {msg}")
        self.code = code


vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double


class NbrInfo(C.Structure):
    _fields_ = [("dim", i32), ("n_colors", i32), ("n", i64), ("n_pairs", i64), ("n_upairs", i64),
                ("n_cells", i64), ("ncell", i64 * 3), ("n_anchors", i64), ("max_deg", i64),
                ("max_level", i64), ("color_off", i64 * 9), ("origin", dbl * 3), ("h", dbl),
                ("inv_rc", dbl), ("key", vp), ("perm", vp), ("cell_start", vp), ("nbr_off", vp),
                ("nbr_idx", vp), ("X", vp), ("V", vp), ("B0", vp), ("sched_a", vp), ("sched_b", vp),
                ("sched_level", vp), ("anchor_key", vp), ("anchor_off", vp), ("anchor_nlev", vp)]


class Material(C.Structure):
    _fields_ = [("model", i32), ("pad_", i32), ("E", dbl), ("nu", dbl), ("rho0", dbl),
                ("sigma0", dbl), ("sigma_inf", dbl), ("delta", dbl), ("H", dbl),
                ("C_swell", dbl), ("c0", dbl), ("rho_l0", dbl)]


class State(C.Structure):
    _fields_ = [("prec", i32), ("pad_", i32), ("u", vp), ("v", vp), ("PB", vp), ("plastic", vp),
                ("c", vp), ("q", vp), ("p", vp), ("acc", vp), ("vgrip", vp), ("flags", vp)]


class MultirateCfg(C.Structure):
    _fields_ = [("n_slow", i32), ("slow_kind", i32), ("dt_slow", dbl), ("dt_s", dbl), ("eta", dbl),
                ("k_max", i64), ("fixed_inner", i64), ("ke_tol", dbl), ("D", dbl), ("c_bc", dbl),
                ("chunk", i32), ("use_graph", i32), ("k_sched", vp), ("batch", vp),
                ("diff_nonlinear", i32), ("pad2_", i32)]


class Batch(C.Structure):
    _fields_ = [("n_spec", i32), ("pad_", i32), ("E", vp), ("D", vp), ("dt_s", vp), ("dt_slow", vp),
                ("grad", vp)]


class Tape(C.Structure):
    _fields_ = [("n_slow_cap", i32), ("pad_", i32), ("k_hist_cap", i64), ("ck_u", vp), ("ck_v", vp),
                ("ck_plastic", vp), ("ck_c", vp), ("hist_H", vp), ("hist_plastic", vp), ("k_rec", vp),
                ("n_rec", i32), ("hist_slow", i32), ("dt_s", dbl), ("dt_slow", dbl),
                ("seg_cap", i64), ("seg_u", vp), ("seg_v", vp), ("seg_plastic", vp)]


class Adjoint(C.Structure):
    _fields_ = [("prec", i32), ("pad_", i32), ("u", vp), ("v", vp), ("plastic", vp), ("c", vp),
                ("p", vp), ("work", vp), ("grad", vp)]


class Tuning(C.Structure):
    _fields_ = [("lpp_stress", i32), ("lpp_momentum", i32), ("lpp_adj_stress", i32), ("lpp_adj_gather", i32),
                ("damp_lanes", i32 * 8), ("damp_idle", i32 * 8), ("ms_solid", dbl), ("ms_adjoint", dbl),
                ("ms_damping_sweep", dbl)]

    def as_dict(self):
        return dict(lpp_stress=self.lpp_stress, lpp_momentum=self.lpp_momentum,
                    lpp_adj_stress=self.lpp_adj_stress, lpp_adj_gather=self.lpp_adj_gather,
                    damp_lanes=list(self.damp_lanes), damp_idle=list(self.damp_idle),
                    ms_solid=self.ms_solid, ms_adjoint=self.ms_adjoint,
                    ms_damping_sweep=self.ms_damping_sweep)


class Report(C.Structure):
    _fields_ = [("k", vp), ("ke", vp), ("converged", vp), ("dt_s", dbl), ("dt_slow", dbl),
                ("k_max", i64), ("total_inner", i64)]


_lib = None


def lib():
    """Load libsph.so (built in-tree by build.py); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SphError(SPH_E_DEVICE, f"{LIB_PATH} is missing: run paper_2309_04010_amd/build.py")
    L = C.CDLL(LIB_PATH)
    L.sph_build_neighbors.argtypes = [C.c_int, i64, vp, vp, dbl, vp, C.POINTER(vp)]
    L.sph_nbr_destroy.argtypes = [vp]
    L.sph_nbr_query.argtypes = [vp, C.POINTER(NbrInfo)]
    L.sph_workspace_size.argtypes = [vp, C.POINTER(i64)]
    L.sph_set_workspace.argtypes = [vp, vp, i64, vp]
    L.sph_solid_relax_step.argtypes = [vp, C.POINTER(Material), C.POINTER(State), dbl, vp]
    L.sph_damping_sweep.argtypes = [vp, C.POINTER(Material), C.POINTER(State), dbl, dbl, vp]
    L.sph_drift_ke.argtypes = [vp, C.POINTER(Material), C.POINTER(State), dbl, vp, vp]
    L.sph_drift_ke_noalloc.argtypes = [vp, C.POINTER(Material), C.POINTER(State), dbl, vp, vp]
    L.sph_load_step.argtypes = [vp, C.POINTER(State), dbl, vp]
    L.sph_diffusion_step.argtypes = [vp, C.POINTER(Material), C.POINTER(State), dbl, dbl, dbl, vp]
    L.sph_diffusion_step_coupled.argtypes = [vp, C.POINTER(Material), C.POINTER(State), dbl, dbl, dbl,
                                             i32, vp]
    L.sph_advance_multirate.argtypes = [vp, C.POINTER(Material), C.POINTER(State),
                                        C.POINTER(MultirateCfg), C.POINTER(Report), C.POINTER(Tape), vp]
    L.sph_advance_multirate_backward.argtypes = [vp, C.POINTER(Material), C.POINTER(State),
                                                 C.POINTER(MultirateCfg), C.POINTER(Tape),
                                                 C.POINTER(Adjoint), vp]
    L.sph_solid_relax_step_vjp.argtypes = [vp, C.POINTER(Material), C.POINTER(State),
                                           C.POINTER(Adjoint), dbl, vp]
    L.sph_damping_sweep_vjp.argtypes = [vp, C.POINTER(Material), C.POINTER(State), C.POINTER(Adjoint),
                                        dbl, dbl, vp]
    L.sph_drift_vjp.argtypes = [vp, C.POINTER(State), C.POINTER(Adjoint), dbl, vp]
    L.sph_diffusion_step_vjp.argtypes = [vp, C.POINTER(Material), C.POINTER(State), vp,
                                         C.POINTER(Adjoint), dbl, dbl, dbl, vp]
    L.sph_diffusion_step_coupled_vjp.argtypes = [vp, C.POINTER(Material), C.POINTER(State), vp,
                                                 C.POINTER(Adjoint), dbl, dbl, dbl, i32, vp]
    L.sph_constitutive.argtypes = [C.POINTER(Material), C.c_int, i64, vp, vp, vp, vp, vp]
    L.sph_constitutive_vjp.argtypes = [C.POINTER(Material), C.c_int, i64, vp, vp, vp, vp, vp, vp, vp,
                                       vp, vp]
    L.sph_build_neighbors_batched.argtypes = [C.c_int, i64, vp, vp, dbl, i32, vp, vp, C.POINTER(vp)]
    L.sph_advance_multirate_graph.argtypes = [vp, C.POINTER(Material), C.POINTER(State),
                                              C.POINTER(MultirateCfg), C.POINTER(Report), C.POINTER(Tape),
                                              C.POINTER(Adjoint), vp]
    L.sph_autotune.argtypes = [vp, C.POINTER(Material), C.POINTER(State), dbl, dbl, C.c_int,
                               C.POINTER(Tuning), vp]
    L.sph_set_tuning.argtypes = [vp, C.c_int, C.POINTER(Tuning)]
    L.sph_get_tuning.argtypes = [vp, C.c_int, C.POINTER(Tuning)]
    L.sph_default_steps.argtypes = [dbl, C.POINTER(Material), dbl, C.POINTER(dbl), C.POINTER(dbl)]
    L.sph_status.argtypes = [vp, vp, C.POINTER(i32)]
    L.sph_profile_enable.argtypes = [vp, C.c_int]
    L.sph_profile_classes.argtypes = [vp, C.c_uint32]
    L.sph_profile_read.argtypes = [vp, C.c_int, C.POINTER(i64), C.POINTER(dbl)]
    L.sph_last_error.restype = C.c_char_p
    for name in EXPORTED:
        getattr(L, name).restype = C.c_int if name != "sph_last_error" else C.c_char_p
    _lib = L
    return L


def _check(rc, allow_warning=False):
    if rc == SPH_OK or (allow_warning and rc == SPH_W_NOT_CONVERGED):
        return rc
    raise SphError(rc, lib().sph_last_error().decode())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, dtype, shape, name):
    import torch
    if t is None:
        return
    if not t.is_cuda:
        raise SphError(SPH_E_ARG, f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise SphError(SPH_E_ARG, f"{name}: want {dtype} {tuple(shape)} contiguous, got "
                                  f"{t.dtype} {tuple(t.shape)}")
    del torch


# --- device -> host copies of handle-owned arrays (plumbing) ----------------
_hip = None


def _hip_lib():
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [vp, vp, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
    return _hip


def copy_out(ptr, count, dtype):
    out = np.empty(int(count), dtype=dtype)
    if count:
        rc = _hip_lib().hipMemcpy(out.ctypes.data_as(vp), C.c_void_p(ptr), out.nbytes, 2)
        if rc != 0:
            raise SphError(SPH_E_DEVICE, f"hipMemcpy failed ({rc})")
    return out


class Neighbors:
    """Owner of an sph_nbr handle (fixed TL neighbourhood + damping schedule)."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep
        self.info = NbrInfo()
        _check(lib().sph_nbr_query(self._h, C.byref(self.info)))
        self.dim = self.info.dim
        self.n = self.info.n

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().sph_nbr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def host(self, name):
        """Copy one handle-owned array to a numpy array (for checks)."""
        i = self.info
        d, n = i.dim, i.n
        spec = {
            "key": (i.key, n, np.uint32), "perm": (i.perm, n, np.uint32),
            "cell_start": (i.cell_start, i.n_cells + 1, np.uint32),
            "nbr_off": (i.nbr_off, n + 1, np.int64), "nbr_idx": (i.nbr_idx, i.n_pairs, np.uint32),
            "X": (i.X, d * n, np.float64), "V": (i.V, n, np.float64),
            "B0": (i.B0, d * d * n, np.float64),
            "sched_a": (i.sched_a, i.n_upairs, np.uint32), "sched_b": (i.sched_b, i.n_upairs, np.uint32),
            "sched_level": (i.sched_level, i.n_upairs, np.uint32),
            "anchor_key": (i.anchor_key, i.n_anchors, np.uint32),
            "anchor_off": (i.anchor_off, i.n_anchors + 1, np.int64),
            "anchor_nlev": (i.anchor_nlev, i.n_anchors, np.uint32),
        }[name]
        arr = copy_out(*spec)
        if name == "X":
            arr = arr.reshape(d, n)
        elif name == "B0":
            arr = arr.reshape(d * d, n)
        return arr


def sph_build_neighbors(X, V, h, stream=None):
    """X: cuda float64 [dim, n]; V: cuda float64 [n] (input order)."""
    import torch
    dim, n = X.shape
    _need(X, torch.float64, (dim, n), "X")
    _need(V, torch.float64, (n,), "V")
    out = C.c_void_p()
    _check(lib().sph_build_neighbors(int(dim), int(n), _dptr(X), _dptr(V), float(h), _stream(stream),
                                     C.byref(out)))
    return Neighbors(out, (X, V))


def material(model, E, nu, rho0, sigma0=0.0, sigma_inf=0.0, delta=0.0, H=0.0, C_swell=0.0, c0=0.0,
             rho_l0=0.0):
    return Material(int(model), 0, float(E), float(nu), float(rho0), float(sigma0), float(sigma_inf),
                    float(delta), float(H), float(C_swell), float(c0), float(rho_l0))


@dataclass
class SphState:
    """Caller-owned device state (torch tensors), cell-sorted order."""
    prec: int
    u: object
    v: object
    PB: object
    plastic: object = None
    c: object = None
    q: object = None
    p: object = None
    acc: object = None
    vgrip: object = None
    flags: object = None
    _c: State = field(default=None, repr=False)

    def validate(self, nbr):
        import torch
        d, n = nbr.dim, nbr.n
        T = torch.float32 if self.prec == SPH_F32 else torch.float64
        _need(self.u, torch.float64, (d, n), "u")
        _need(self.v, T, (d, n), "v")
        _need(self.PB, T, (d * d, n), "PB")
        _need(self.plastic, T, (7, n), "plastic")
        _need(self.c, T, (n,), "c")
        _need(self.q, T, (d, n), "q")
        _need(self.p, T, (n,), "p")
        _need(self.acc, T, (d, n), "acc")
        _need(self.vgrip, T, (d, n), "vgrip")
        _need(self.flags, torch.uint8, (n,), "flags")

    def cstruct(self, nbr):
        self.validate(nbr)
        return State(int(self.prec), 0, _dptr(self.u), _dptr(self.v), _dptr(self.PB), _dptr(self.plastic),
                     _dptr(self.c), _dptr(self.q), _dptr(self.p), _dptr(self.acc), _dptr(self.vgrip),
                     _dptr(self.flags))


def new_state(nbr, prec, with_plastic=False, with_diffusion=False, with_acc=False, device="cuda"):
    import torch
    d, n = nbr.dim, nbr.n
    T = torch.float32 if prec == SPH_F32 else torch.float64
    z = lambda *s, dt=T: torch.zeros(s, dtype=dt, device=device)  # noqa: E731
    st = SphState(prec, z(d, n, dt=torch.float64), z(d, n), z(d * d, n))
    if with_plastic:
        st.plastic = z(7, n)   # Cbar_p^-1 - I and alpha: virgin state is zero
    if with_diffusion:
        st.c, st.q, st.p = z(n), z(d, n), z(n)
    if with_acc:
        st.acc = z(d, n)
    return st


def sph_default_steps(h, mat, D=0.0):
    """(dt_s, dt_d): the library's step sizes of Sec. 4.1 (host computation)."""
    a, b = dbl(0.0), dbl(0.0)
    _check(lib().sph_default_steps(float(h), C.byref(mat), float(D), C.byref(a), C.byref(b)))
    return a.value, b.value


def sph_solid_relax_step(nbr, mat, st, dt_s, stream=None):
    cs = st.cstruct(nbr)
    _check(lib().sph_solid_relax_step(nbr.handle, C.byref(mat), C.byref(cs), float(dt_s), _stream(stream)))


def sph_damping_sweep(nbr, mat, st, eta, dt_s, stream=None):
    cs = st.cstruct(nbr)
    _check(lib().sph_damping_sweep(nbr.handle, C.byref(mat), C.byref(cs), float(eta), float(dt_s),
                                   _stream(stream)))


def sph_drift_ke(nbr, mat, st, dt_s, ke_out=None, stream=None):
    cs = st.cstruct(nbr)
    _check(lib().sph_drift_ke(nbr.handle, C.byref(mat), C.byref(cs), float(dt_s), _dptr(ke_out),
                              _stream(stream)))


def sph_drift_ke_noalloc(nbr, mat, st, dt_s, ke_out=None, stream=None):
    cs = st.cstruct(nbr)
    _check(lib().sph_drift_ke_noalloc(nbr.handle, C.byref(mat), C.byref(cs), float(dt_s),
                                      _dptr(ke_out), _stream(stream)))


def sph_workspace_size(nbr):
    """Bytes of the per-step scratch of the handle (its workspace)."""
    b = i64(0)
    _check(lib().sph_workspace_size(nbr.handle, C.byref(b)))
    return int(b.value)


def sph_set_workspace(nbr, ws=None, stream=None):
    """Make the handle use the device tensor `ws` (any dtype, contiguous,
    256-byte aligned, at least sph_workspace_size bytes) as its per-step
    scratch, or its own block again with ws=None.  The caller keeps `ws`
    alive while the handle uses it."""
    if ws is None:
        _check(lib().sph_set_workspace(nbr.handle, None, 0, _stream(stream)))
        nbr._ws = None
        return
    if not ws.is_cuda or not ws.is_contiguous():
        raise SphError(SPH_E_ARG, "ws must be a contiguous device tensor")
    nbytes = ws.numel() * ws.element_size()
    _check(lib().sph_set_workspace(nbr.handle, _dptr(ws), int(nbytes), _stream(stream)))
    nbr._ws = ws


def sph_load_step(nbr, st, dt_l, stream=None):
    cs = st.cstruct(nbr)
    _check(lib().sph_load_step(nbr.handle, C.byref(cs), float(dt_l), _stream(stream)))


def sph_diffusion_step_coupled(nbr, mat, st, D, dt_d, c_bc, nonlinear=0, stream=None):
    cs = st.cstruct(nbr)
    _check(lib().sph_diffusion_step_coupled(nbr.handle, C.byref(mat), C.byref(cs), float(D), float(dt_d),
                                            float(c_bc), int(nonlinear), _stream(stream)))


def sph_diffusion_step(nbr, mat, st, D, dt_d, c_bc, stream=None):
    cs = st.cstruct(nbr)
    _check(lib().sph_diffusion_step(nbr.handle, C.byref(mat), C.byref(cs), float(D), float(dt_d),
                                    float(c_bc), _stream(stream)))


def sph_status(nbr, stream=None):
    bits = i32(0)
    rc = lib().sph_status(nbr.handle, _stream(stream), C.byref(bits))
    return rc, bits.value


def multirate_cfg(n_slow, slow_kind, dt_slow=0.0, dt_s=0.0, eta=0.0, k_max=0, fixed_inner=0,
                  ke_tol=0.0, D=0.0, c_bc=0.0, chunk=64, use_graph=0, k_sched=None, batch=None,
                  diff_nonlinear=0):
    cfg = MultirateCfg(int(n_slow), int(slow_kind), float(dt_slow), float(dt_s), float(eta), int(k_max),
                       int(fixed_inner), float(ke_tol), float(D), float(c_bc), int(chunk), int(use_graph),
                       None, None, int(diff_nonlinear), 0)
    if k_sched is not None:
        ks = np.ascontiguousarray(k_sched, dtype=np.int64)
        cfg._ks = ks
        cfg.k_sched = ks.ctypes.data_as(vp)
    if batch is not None:
        cfg._batch = batch
        cfg.batch = C.cast(C.pointer(batch.cstruct()), vp)
    return cfg


class SphBatch:
    """Per-specimen values of a batched run (sph_batch): host arrays of n_spec
    doubles for E, D, dt_s, dt_slow (dt_s / dt_slow None or entries <= 0: the
    library's per-specimen sph_default_steps); `grad` a device [n_spec,
    SPH_NGRAD] tensor."""

    def __init__(self, E, D, dt_s=None, dt_slow=None, grad=None):
        self.E = np.ascontiguousarray(E, dtype=np.float64)
        n = self.E.size
        self.D = np.ascontiguousarray(D, dtype=np.float64)
        self.dt_s = np.ascontiguousarray(np.zeros(n) if dt_s is None else dt_s, dtype=np.float64)
        self.dt_slow = np.ascontiguousarray(np.zeros(n) if dt_slow is None else dt_slow, dtype=np.float64)
        assert self.D.size == n and self.dt_s.size == n and self.dt_slow.size == n
        self.grad = grad
        self._c = None

    def cstruct(self):
        import torch
        if self.grad is not None:
            _need(self.grad, torch.float64, (self.E.size, SPH_NGRAD), "batch.grad")
        self._c = Batch(int(self.E.size), 0, self.E.ctypes.data_as(vp), self.D.ctypes.data_as(vp),
                        self.dt_s.ctypes.data_as(vp), self.dt_slow.ctypes.data_as(vp), _dptr(self.grad))
        return self._c


def sph_build_neighbors_batched(X, V, h, spec_id, stream=None):
    """X: cuda float64 [dim, n]; V: cuda float64 [n]; spec_id: cuda int32 [n]
    (contiguous ascending runs 0..n_spec-1), all in input order."""
    import torch
    dim, n = X.shape
    _need(X, torch.float64, (dim, n), "X")
    _need(V, torch.float64, (n,), "V")
    _need(spec_id, torch.int32, (n,), "spec_id")
    n_spec = int(spec_id.max().item()) + 1
    out = C.c_void_p()
    _check(lib().sph_build_neighbors_batched(int(dim), int(n), _dptr(X), _dptr(V), float(h), n_spec,
                                             _dptr(spec_id), _stream(stream), C.byref(out)))
    return Neighbors(out, (X, V, spec_id))


def sph_advance_multirate_graph(nbr, mat, st, cfg, tape=None, adj=None, stream=None):
    """Forward (+ reverse when adj is given) as one recorded graph; returns k."""
    cs = st.cstruct(nbr)
    ns = cfg.n_slow
    k = np.zeros(max(ns, 1), np.int64)
    rep_ = Report(k.ctypes.data_as(vp), None, None, 0.0, 0.0, 0, 0)
    tp = None if tape is None else C.byref(tape.cstruct(nbr, st))
    ad = None if adj is None else C.byref(adj.cstruct(nbr))
    _check(lib().sph_advance_multirate_graph(nbr.handle, C.byref(mat), C.byref(cs), C.byref(cfg),
                                             C.byref(rep_), tp, ad, _stream(stream)))
    if tape is not None:
        tape.sync_out()
    return k[:ns]


def sph_advance_multirate(nbr, mat, st, cfg, tape=None, stream=None):
    """Returns (rc, k[n_slow], ke[n_slow], converged[n_slow], report)."""
    cs = st.cstruct(nbr)
    ns = cfg.n_slow
    k = np.zeros(max(ns, 1), np.int64)
    ke = np.zeros(max(ns, 1))
    conv = np.zeros(max(ns, 1), np.int32)
    rep = Report(k.ctypes.data_as(vp), ke.ctypes.data_as(vp), conv.ctypes.data_as(vp), 0.0, 0.0, 0, 0)
    tp = None if tape is None else C.byref(tape.cstruct(nbr, st))
    rc = _check(lib().sph_advance_multirate(nbr.handle, C.byref(mat), C.byref(cs), C.byref(cfg),
                                            C.byref(rep), tp, _stream(stream)), allow_warning=True)
    if tape is not None:
        tape.sync_out()
    return rc, k[:ns], ke[:ns], conv[:ns], rep


# --- reverse mode -------------------------------------------------------------
class SphTape:
    """Device checkpoints of a forward multi-time-step run (sph_tape).
    k_hist: inner steps whose states the tape holds at once; seg_cap: inner
    checkpoints for slow steps longer than that (reversed in segments of
    k_hist inner steps, up to (seg_cap + 1) * k_hist)."""

    def __init__(self, nbr, prec, n_slow, k_hist, with_plastic=False, with_diffusion=False,
                 device="cuda", seg_cap=0):
        import torch
        d, n = nbr.dim, nbr.n
        T = torch.float32 if prec == SPH_F32 else torch.float64
        z = lambda *s, dt=T: torch.zeros(s, dtype=dt, device=device)  # noqa: E731
        self.prec = prec
        self.n_slow_cap = int(n_slow)
        self.k_hist_cap = int(k_hist)
        self.ck_u = z(n_slow + 1, d, n, dt=torch.float64)
        self.ck_v = z(n_slow + 1, d, n)
        self.ck_plastic = z(n_slow + 1, 7, n) if with_plastic else None
        self.ck_c = z(n_slow + 1, n) if with_diffusion else None
        self.hist_H = z(max(k_hist, 1), d * d, n)
        self.hist_plastic = z(max(k_hist, 1), 7, n) if with_plastic else None
        self.seg_cap = int(seg_cap)
        self.seg_u = z(seg_cap, d, n, dt=torch.float64) if seg_cap > 0 else None
        self.seg_v = z(seg_cap, d, n) if seg_cap > 0 else None
        self.seg_plastic = z(seg_cap, 7, n) if seg_cap > 0 and with_plastic else None
        self.k_rec = np.zeros(max(n_slow, 1), np.int64)
        self._c = Tape(self.n_slow_cap, 0, self.k_hist_cap, _dptr(self.ck_u), _dptr(self.ck_v),
                       _dptr(self.ck_plastic), _dptr(self.ck_c), _dptr(self.hist_H),
                       _dptr(self.hist_plastic), self.k_rec.ctypes.data_as(vp), 0, -1, 0.0, 0.0,
                       self.seg_cap, _dptr(self.seg_u), _dptr(self.seg_v), _dptr(self.seg_plastic))

    @staticmethod
    def plan(n, dim, prec, k_inner, budget_bytes, with_plastic=False):
        """(k_hist, seg_cap) for slow steps of k_inner inner steps with the
        recorded inner states within budget_bytes: the whole slow step when it
        fits, else the fewest segments whose states and inner checkpoints do."""
        T = 4 if prec == SPH_F32 else 8
        per_step = (dim * dim + (7 if with_plastic else 0)) * n * T
        per_seg = (dim * 8 + dim * T + (7 * T if with_plastic else 0)) * n
        k_inner = max(int(k_inner), 1)
        for ns in range(1, k_inner + 1):
            k_hist = -(-k_inner // ns)
            if k_hist * per_step + (ns - 1) * per_seg <= budget_bytes:
                return k_hist, ns - 1
        raise SphError(SPH_E_CAPACITY, "no segmentation of the tape fits the budget")

    def cstruct(self, nbr, st):
        if st.prec != self.prec:
            raise SphError(SPH_E_ARG, "tape and state precisions differ")
        return self._c

    def sync_out(self):
        self.n_rec = self._c.n_rec
        self.hist_slow = self._c.hist_slow
        self.dt_s = self._c.dt_s
        self.dt_slow = self._c.dt_slow

    def forget_inner_states(self):
        """Mark hist_H as holding no slow step's inner states (hist_slow = -1):
        the next reverse pass re-runs every slow step from its checkpoint, as
        a checkpointed run whose inner states were not kept does."""
        self._c.hist_slow = -1
        self.hist_slow = -1


@dataclass
class SphAdjoint:
    """Adjoint state (sph_adjoint): device tensors, same layout as SphState."""
    prec: int
    u: object
    v: object
    work: object
    grad: object
    plastic: object = None
    c: object = None
    p: object = None

    def cstruct(self, nbr):
        import torch
        d, n = nbr.dim, nbr.n
        T = torch.float32 if self.prec == SPH_F32 else torch.float64
        _need(self.u, torch.float64, (d, n), "adj.u")
        _need(self.v, T, (d, n), "adj.v")
        _need(self.work, T, (d * d, n), "adj.work")
        _need(self.grad, torch.float64, (SPH_NGRAD,), "adj.grad")
        _need(self.plastic, T, (7, n), "adj.plastic")
        _need(self.c, T, (n,), "adj.c")
        _need(self.p, torch.float64, (n,), "adj.p")
        return Adjoint(int(self.prec), 0, _dptr(self.u), _dptr(self.v), _dptr(self.plastic), _dptr(self.c),
                       _dptr(self.p), _dptr(self.work), _dptr(self.grad))

    def zero_(self):
        for t in (self.u, self.v, self.work, self.grad, self.plastic, self.c, self.p):
            if t is not None:
                t.zero_()
        return self


def new_adjoint(nbr, prec, with_plastic=False, with_diffusion=False, with_p=False, device="cuda"):
    import torch
    d, n = nbr.dim, nbr.n
    T = torch.float32 if prec == SPH_F32 else torch.float64
    z = lambda *s, dt=T: torch.zeros(s, dtype=dt, device=device)  # noqa: E731
    a = SphAdjoint(prec, z(d, n, dt=torch.float64), z(d, n), z(d * d, n), z(SPH_NGRAD, dt=torch.float64))
    if with_plastic:
        a.plastic = z(7, n)
    if with_diffusion:
        a.c = z(n)
    if with_diffusion or with_p:
        a.p = z(n, dt=torch.float64)
    return a


def sph_advance_multirate_backward(nbr, mat, st, cfg, tape, adj, stream=None):
    cs = st.cstruct(nbr)
    _check(lib().sph_advance_multirate_backward(nbr.handle, C.byref(mat), C.byref(cs), C.byref(cfg),
                                                C.byref(tape.cstruct(nbr, st)), C.byref(adj.cstruct(nbr)),
                                                _stream(stream)))
    tape.sync_out()


def sph_solid_relax_step_vjp(nbr, mat, st, adj, dt_s, stream=None):
    cs = st.cstruct(nbr)
    _check(lib().sph_solid_relax_step_vjp(nbr.handle, C.byref(mat), C.byref(cs), C.byref(adj.cstruct(nbr)),
                                          float(dt_s), _stream(stream)))


def sph_damping_sweep_vjp(nbr, mat, st, adj, eta, dt_s, stream=None):
    cs = st.cstruct(nbr)
    _check(lib().sph_damping_sweep_vjp(nbr.handle, C.byref(mat), C.byref(cs), C.byref(adj.cstruct(nbr)),
                                       float(eta), float(dt_s), _stream(stream)))


def sph_drift_vjp(nbr, st, adj, dt_s, stream=None):
    cs = st.cstruct(nbr)
    _check(lib().sph_drift_vjp(nbr.handle, C.byref(cs), C.byref(adj.cstruct(nbr)), float(dt_s),
                               _stream(stream)))


def sph_diffusion_step_vjp(nbr, mat, st, c_before, adj, D, dt_d, c_bc, stream=None):
    import torch
    cs = st.cstruct(nbr)
    _need(c_before, torch.float32 if st.prec == SPH_F32 else torch.float64, (nbr.n,), "c_before")
    _check(lib().sph_diffusion_step_vjp(nbr.handle, C.byref(mat), C.byref(cs), _dptr(c_before),
                                        C.byref(adj.cstruct(nbr)), float(D), float(dt_d), float(c_bc),
                                        _stream(stream)))


def sph_diffusion_step_coupled_vjp(nbr, mat, st, c_before, adj, D, dt_d, c_bc, nonlinear=0,
                                   stream=None):
    import torch
    cs = st.cstruct(nbr)
    _need(c_before, torch.float32 if st.prec == SPH_F32 else torch.float64, (nbr.n,), "c_before")
    _check(lib().sph_diffusion_step_coupled_vjp(nbr.handle, C.byref(mat), C.byref(cs), _dptr(c_before),
                                                C.byref(adj.cstruct(nbr)), float(D), float(dt_d),
                                                float(c_bc), int(nonlinear), _stream(stream)))


def _point_check(prec, n, **arrs):
    import torch
    T = torch.float32 if prec == SPH_F32 else torch.float64
    rows = {"H": 9, "plastic": 7, "p": 0, "P": 9, "Pbar": 9, "plastic_bar": 7, "Hbar": 9, "pbar": 0,
            "theta_bar": 5}
    for name, t in arrs.items():
        r = rows[name]
        _need(t, T, (r, n) if r else (n,), name)


def sph_constitutive(mat, prec, H, plastic=None, p=None, P=None, stream=None):
    """H [9][n] = F - I; returns P [9][n] (plastic updated in place)."""
    import torch
    n = H.shape[1]
    if P is None:
        P = torch.empty_like(H)
    _point_check(prec, n, H=H, plastic=plastic, p=p, P=P)
    _check(lib().sph_constitutive(C.byref(mat), int(prec), int(n), _dptr(H), _dptr(plastic), _dptr(p),
                                  _dptr(P), _stream(stream)))
    return P


def sph_constitutive_vjp(mat, prec, H, Pbar, plastic=None, plastic_bar=None, p=None, stream=None):
    """Returns (Hbar [9][n], pbar [n], theta_bar [5][n]); plastic_bar is replaced in place."""
    import torch
    n = H.shape[1]
    Hbar = torch.empty_like(H)
    pbar = torch.empty(n, dtype=H.dtype, device=H.device)
    thb = torch.empty(5, n, dtype=H.dtype, device=H.device)
    _point_check(prec, n, H=H, Pbar=Pbar, plastic=plastic, plastic_bar=plastic_bar, p=p, Hbar=Hbar,
                 pbar=pbar, theta_bar=thb)
    _check(lib().sph_constitutive_vjp(C.byref(mat), int(prec), int(n), _dptr(H), _dptr(plastic), _dptr(p),
                                      _dptr(Pbar), _dptr(plastic_bar), _dptr(Hbar), _dptr(pbar), _dptr(thb),
                                      _stream(stream)))
    return Hbar, pbar, thb


def sph_autotune(nbr, mat, st, eta, dt_s, with_adjoint=True, stream=None):
    """Time the launch-shape candidates on this handle and keep the fastest."""
    cs = st.cstruct(nbr)
    t = Tuning()
    _check(lib().sph_autotune(nbr.handle, C.byref(mat), C.byref(cs), float(eta), float(dt_s),
                              1 if with_adjoint else 0, C.byref(t), _stream(stream)))
    return t


def sph_set_tuning(nbr, prec, lpp_stress=2, lpp_momentum=4, lpp_adj_stress=2, lpp_adj_gather=4,
                   damp_lanes=(0,) * 8, damp_idle=(0,) * 8):
    t = Tuning(lpp_stress, lpp_momentum, lpp_adj_stress, lpp_adj_gather, (i32 * 8)(*damp_lanes),
               (i32 * 8)(*damp_idle), 0.0, 0.0, 0.0)
    _check(lib().sph_set_tuning(nbr.handle, int(prec), C.byref(t)))


def sph_get_tuning(nbr, prec):
    t = Tuning()
    _check(lib().sph_get_tuning(nbr.handle, int(prec), C.byref(t)))
    return t


def sph_profile_enable(nbr, enable=True):
    _check(lib().sph_profile_enable(nbr.handle, 1 if enable else 0))


def sph_profile_classes(nbr, classes=None):
    """Time only these kernel classes (names of SPH_KERNEL_NAMES or indices);
    None: all."""
    if classes is None:
        mask = 0xFFFFFFFF
    else:
        mask = 0
        for c in classes:
            mask |= 1 << (SPH_KERNEL_NAMES.index(c) if isinstance(c, str) else int(c))
    _check(lib().sph_profile_classes(nbr.handle, mask))


def sph_profile_read(nbr):
    """{kernel class: (launches, total ms)} of the launches timed so far."""
    out = {}
    for k, name in enumerate(SPH_KERNEL_NAMES):
        cnt, ms = i64(0), dbl(0.0)
        _check(lib().sph_profile_read(nbr.handle, k, C.byref(cnt), C.byref(ms)))
        out[name] = (cnt.value, ms.value)
    return out
