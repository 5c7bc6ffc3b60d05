"""FP64 CPU oracle of the TL-SPH multi-time-step hot path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never loads it, and the
two share no source.  ``liboracle.so`` is the plain FP64 oracle;
``liboracle_cs.so`` is the same source compiled with complex ``real``, used as a
complex-step derivative oracle (Im(f(x + i e)) / e = f'(x) to rounding).

Arrays are numpy, structure-of-arrays ``[component, n]`` in the cell-sorted
order that the build returns (``perm[s]`` = input id of sorted particle s).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_LIBS = {False: os.path.join(_HERE, "liboracle.so"), True: os.path.join(_HERE, "liboracle_cs.so"),
         "omp": os.path.join(_HERE, "liboracle_omp.so")}

LE, NH, J2 = 0, 1, 2
LOAD, DIFFUSION, DIFFUSION_COUPLED = 0, 1, 2
FIXED, CDIR, GRIP = 1, 2, 4


def build(force: bool = True) -> None:
    """Compile the oracle variants with gcc (no FMA contraction): the plain
    FP64 oracle, the complex-step one, and the OpenMP build that only the
    all-core CPU baseline of the benchmark loads."""
    for kind, out in _LIBS.items():
        if not force and os.path.exists(out) and os.path.getmtime(out) > os.path.getmtime(_SRC):
            continue
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11", "-o", out, _SRC, "-lm"]
        if kind is True:
            cmd.insert(1, "-DORC_COMPLEX")
        elif kind == "omp":
            cmd.insert(1, "-fopenmp")
        subprocess.run(cmd, check=True)


_cache: dict = {}


def _lib(cplx):
    """cplx: False (FP64), True (complex step) or "omp" (FP64, OpenMP)."""
    if cplx in _cache:
        return _cache[cplx]
    path = _LIBS[cplx]
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        build(force=True)
    lib = C.CDLL(path)
    vp, i64, dbl, i32 = C.c_void_p, C.c_int64, C.c_double, C.c_int
    lib.orc_kernel_W.restype = dbl
    lib.orc_kernel_W.argtypes = [i32, dbl, dbl]
    lib.orc_kernel_dW_over_r.restype = dbl
    lib.orc_kernel_dW_over_r.argtypes = [i32, dbl, dbl]
    lib.orc_create.restype = vp
    lib.orc_create.argtypes = [i32, i64, vp, vp, dbl, C.POINTER(C.c_int)]
    lib.orc_destroy.argtypes = [vp]
    lib.orc_sizes.argtypes = [vp, vp]
    lib.orc_grid.argtypes = [vp, vp, vp]
    lib.orc_get_build.argtypes = [vp] * 9
    lib.orc_get_schedule.argtypes = [vp] * 8
    lib.orc_constitutive.restype = i32
    cplx_t = cplx is True
    lib.orc_constitutive.argtypes = [vp, vp, vp, _real_t(cplx_t), vp]
    lib.orc_displacement_gradient.argtypes = [vp, vp, vp]
    lib.orc_stress.restype = i32
    lib.orc_stress.argtypes = [vp] * 7
    lib.orc_momentum.argtypes = [vp] * 5
    lib.orc_mixture_flux.argtypes = [vp] * 7
    lib.orc_solid_step.restype = i32
    lib.orc_solid_step.argtypes = [vp, vp, dbl, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.orc_damping_sweep.argtypes = [vp, dbl, dbl, dbl, vp, vp, dbl, vp]
    lib.orc_drift_ke.restype = _real_t(cplx_t)
    lib.orc_drift_ke.argtypes = [vp, dbl, dbl, vp, vp, vp, dbl, vp]
    lib.orc_load_step.argtypes = [vp, dbl, vp, vp, vp]
    lib.orc_diffusion_step.argtypes = [vp, _real_t(cplx_t), dbl, dbl, _real_t(cplx_t), dbl, vp, vp, vp, vp]
    lib.orc_diffusion_step_coupled.argtypes = [vp, _real_t(cplx_t), dbl, dbl, _real_t(cplx_t), dbl, C.c_int,
                                               vp, vp, vp, vp, vp]
    lib.orc_default_steps.argtypes = [vp, vp, dbl, vp, vp]
    lib.orc_advance.restype = i32
    lib.orc_advance.argtypes = [vp] * 16
    _cache[cplx] = lib
    return lib


class _Cplx(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


def _real_t(cplx):
    return _Cplx if cplx else C.c_double


def _to_real(x, cplx):
    if cplx:
        z = complex(x)
        return _Cplx(z.real, z.imag)
    return float(x)


def _material_t(cplx):
    R = _real_t(cplx)

    class Material(C.Structure):
        _fields_ = [("model", C.c_int32), ("pad_", C.c_int32), ("E", R), ("nu", C.c_double),
                    ("rho0", C.c_double), ("sigma0", R), ("sigma_inf", R), ("delta", R), ("H", R),
                    ("C_swell", R), ("c0", C.c_double), ("rho_l0", C.c_double)]
    return Material


def _cfg_t(cplx):
    R = _real_t(cplx)

    class Cfg(C.Structure):
        _fields_ = [("n_slow", C.c_int32), ("slow_kind", C.c_int32), ("dt_slow", C.c_double),
                    ("dt_s", C.c_double), ("eta", C.c_double), ("k_max", C.c_int64),
                    ("fixed_inner", C.c_int64), ("ke_tol", C.c_double), ("D", R), ("c_bc", C.c_double),
                    ("nonlinear", C.c_int32), ("pad2_", C.c_int32)]
    return Cfg


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Oracle:
    """One particle set: build (grid, sort, neighbours, B0, schedule) + steps."""

    def __init__(self, dim, X_id, V_id, h, complex_step=False, openmp=False):
        self.cplx = bool(complex_step)
        if openmp and self.cplx:
            raise ValueError("the OpenMP build is FP64 only")
        self.lib = _lib("omp" if openmp else self.cplx)
        self.dtype = np.complex128 if self.cplx else np.float64
        X_id = np.ascontiguousarray(X_id, dtype=np.float64)
        V_id = np.ascontiguousarray(V_id, dtype=np.float64)
        assert X_id.shape[0] == dim and V_id.shape == (X_id.shape[1],)
        self.dim, self.n, self.h = dim, X_id.shape[1], float(h)
        err = C.c_int(0)
        self._h = self.lib.orc_create(dim, self.n, _ptr(X_id), _ptr(V_id), float(h), C.byref(err))
        if not self._h:
            raise RuntimeError(f"orc_create failed with code {err.value}")
        sz = np.zeros(10, np.int64)
        self.lib.orc_sizes(self._h, _ptr(sz))
        (self.n, self.n_pairs, self.n_upairs, self.n_cells, nc0, nc1, nc2, self.n_anchors,
         self.max_level, self.max_deg) = [int(x) for x in sz]
        self.ncell = (nc0, nc1, nc2)
        org = np.zeros(3)
        inv = C.c_double(0)
        self.lib.orc_grid(self._h, _ptr(org), C.byref(inv))
        self.origin, self.inv_rc = org, inv.value
        n, d = self.n, dim
        self.key = np.zeros(n, np.uint32)
        self.perm = np.zeros(n, np.uint32)
        self.cell_start = np.zeros(self.n_cells + 1, np.uint32)
        self.nbr_off = np.zeros(n + 1, np.int64)
        self.nbr_idx = np.zeros(max(self.n_pairs, 1), np.uint32)
        self.X = np.zeros((d, n))
        self.V = np.zeros(n)
        self.B0 = np.zeros((d * d, n))
        self.lib.orc_get_build(self._h, _ptr(self.key), _ptr(self.perm), _ptr(self.cell_start),
                               _ptr(self.nbr_off), _ptr(self.nbr_idx), _ptr(self.X), _ptr(self.V),
                               _ptr(self.B0))
        self.nbr_idx = self.nbr_idx[: self.n_pairs]
        npu = max(self.n_upairs, 1)
        self.sched_a = np.zeros(npu, np.uint32)
        self.sched_b = np.zeros(npu, np.uint32)
        self.sched_level = np.zeros(npu, np.uint32)
        self.anchor_key = np.zeros(max(self.n_anchors, 1), np.uint32)
        self.anchor_off = np.zeros(self.n_anchors + 1, np.int64)
        self.anchor_nlev = np.zeros(max(self.n_anchors, 1), np.uint32)
        self.color_off = np.zeros(9, np.int64)
        self.lib.orc_get_schedule(self._h, _ptr(self.sched_a), _ptr(self.sched_b),
                                  _ptr(self.sched_level), _ptr(self.anchor_key),
                                  _ptr(self.anchor_off), _ptr(self.anchor_nlev), _ptr(self.color_off))
        self.sched_a = self.sched_a[: self.n_upairs]
        self.sched_b = self.sched_b[: self.n_upairs]
        self.sched_level = self.sched_level[: self.n_upairs]
        self.anchor_key = self.anchor_key[: self.n_anchors]
        self.anchor_nlev = self.anchor_nlev[: self.n_anchors]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self.lib.orc_destroy(h)
            self._h = None

    # -- helpers --------------------------------------------------------
    def arr(self, *shape):
        return np.zeros(shape, self.dtype)

    def _a(self, x):
        if x is None:
            return None
        assert x.dtype == self.dtype and x.flags.c_contiguous, (x.dtype, self.dtype)
        return x

    def material(self, model, E, nu, rho0, sigma0=0.0, sigma_inf=0.0, delta=0.0, H=0.0,
                 C_swell=0.0, c0=0.0, rho_l0=0.0):
        M = _material_t(self.cplx)
        r = lambda x: _to_real(x, self.cplx)  # noqa: E731
        return M(int(model), 0, r(E), float(nu), float(rho0), r(sigma0), r(sigma_inf), r(delta),
                 r(H), r(C_swell), float(c0), float(rho_l0))

    def cfg(self, n_slow, slow_kind, dt_slow, dt_s=0.0, eta=0.0, k_max=0, fixed_inner=0, ke_tol=0.0,
            D=0.0, c_bc=0.0, nonlinear=0):
        Cf = _cfg_t(self.cplx)
        return Cf(int(n_slow), int(slow_kind), float(dt_slow), float(dt_s), float(eta), int(k_max),
                  int(fixed_inner), float(ke_tol), _to_real(D, self.cplx), float(c_bc), int(nonlinear), 0)

    @staticmethod
    def _from_real(x):
        return complex(x.re, x.im) if isinstance(x, _Cplx) else x

    def default_steps(self, mat, D=0.0):
        """(dt_s, dt_d) of Sec. 4.1 for this particle set and material."""
        a, b = C.c_double(0), C.c_double(0)
        self.lib.orc_default_steps(self._h, C.byref(mat), float(D), C.byref(a), C.byref(b))
        return a.value, b.value

    # -- kernel ---------------------------------------------------------
    def W(self, r):
        return self.lib.orc_kernel_W(self.dim, self.h, float(r))

    def dW_over_r(self, r):
        return self.lib.orc_kernel_dW_over_r(self.dim, self.h, float(r))

    # -- steps ----------------------------------------------------------
    def constitutive(self, mat, F=None, plastic7=None, p=0.0, H=None):
        """Stress of one particle from F (or from H = F - I).  plastic7 holds
        Cbar_p^-1 - I (xx yy zz xy yz xz) and alpha; zeros = virgin state."""
        if H is None:
            H = np.asarray(F, dtype=self.dtype).reshape(3, 3) - np.eye(3)
        H = np.ascontiguousarray(H, dtype=self.dtype).reshape(9)
        pl = (np.zeros(7, self.dtype) if plastic7 is None
              else np.ascontiguousarray(plastic7, dtype=self.dtype).copy())
        P = np.zeros(9, self.dtype)
        rc = self.lib.orc_constitutive(C.byref(mat), _ptr(H), _ptr(pl), _to_real(p, self.cplx), _ptr(P))
        return rc, P.reshape(3, 3), pl

    def displacement_gradient(self, u):
        H9 = self.arr(9, self.n)
        self.lib.orc_displacement_gradient(self._h, _ptr(self._a(u)), _ptr(H9))
        return H9

    def deformation_gradient(self, u):
        F9 = self.displacement_gradient(u)
        F9[0] += 1.0
        F9[4] += 1.0
        F9[8] += 1.0
        return F9

    def stress(self, mat, H9, plastic=None, p=None):
        """Stress from H9 = F - I ([9, n]); returns (rc, P9, PB)."""
        P9 = self.arr(9, self.n)
        PB = self.arr(self.dim * self.dim, self.n)
        rc = self.lib.orc_stress(self._h, C.byref(mat), _ptr(self._a(H9)), _ptr(self._a(plastic)),
                                 _ptr(self._a(p)), _ptr(P9), _ptr(PB))
        return rc, P9, PB

    def momentum(self, mat, PB, c=None):
        acc = self.arr(self.dim, self.n)
        self.lib.orc_momentum(self._h, C.byref(mat), _ptr(self._a(PB)), _ptr(self._a(c)), _ptr(acc))
        return acc

    def mixture_flux(self, mat, H9, v, c, q, PB):
        """PB -= rho_l0 v^l (x) Q B0 in place (mixture momentum flux)."""
        self.lib.orc_mixture_flux(self._h, C.byref(mat), _ptr(self._a(H9)), _ptr(self._a(v)),
                                  _ptr(self._a(c)), _ptr(self._a(q)), _ptr(self._a(PB)))

    def solid_step(self, mat, dt, u, v, plastic=None, p=None, flags=None, c=None, q=None):
        PB = self.arr(self.dim * self.dim, self.n)
        acc = self.arr(self.dim, self.n)
        rc = self.lib.orc_solid_step(self._h, C.byref(mat), float(dt), _ptr(self._a(u)), _ptr(self._a(v)),
                                     _ptr(self._a(plastic)), _ptr(self._a(p)), _ptr(flags), _ptr(PB), _ptr(acc),
                                     _ptr(self._a(c)), _ptr(self._a(q)))
        return rc, PB, acc

    def damping_sweep(self, rho0, eta, dt, v, flags=None, rho_l0=0.0, c=None):
        self.lib.orc_damping_sweep(self._h, float(rho0), float(eta), float(dt), _ptr(self._a(v)), _ptr(flags),
                                   float(rho_l0), _ptr(self._a(c)))

    def drift_ke(self, rho0, dt, u, v, flags=None, rho_l0=0.0, c=None):
        ke = self.lib.orc_drift_ke(self._h, float(rho0), float(dt), _ptr(self._a(u)), _ptr(self._a(v)),
                                   _ptr(flags), float(rho_l0), _ptr(self._a(c)))
        return self._from_real(ke)

    def load_step(self, dt_l, u, vgrip, flags):
        self.lib.orc_load_step(self._h, float(dt_l), _ptr(self._a(u)), _ptr(self._a(vgrip)), _ptr(flags))

    def diffusion_step(self, D, dt_d, c_bc, C_swell, c0, c, q, p, flags=None):
        self.lib.orc_diffusion_step(self._h, _to_real(D, self.cplx), float(dt_d), float(c_bc),
                                    _to_real(C_swell, self.cplx), float(c0), _ptr(self._a(c)),
                                    _ptr(self._a(q)), _ptr(self._a(p)), _ptr(flags))

    def diffusion_step_coupled(self, D, dt_d, c_bc, C_swell, c0, nonlinear, u, c, q, p, flags=None):
        """Two-way coupled diffusion step: c is the fluid content per reference
        volume, the saturation c / J follows u; q receives the reference flux."""
        self.lib.orc_diffusion_step_coupled(self._h, _to_real(D, self.cplx), float(dt_d), float(c_bc),
                                            _to_real(C_swell, self.cplx), float(c0), int(nonlinear),
                                            _ptr(self._a(u)), _ptr(self._a(c)), _ptr(self._a(q)),
                                            _ptr(self._a(p)), _ptr(flags))

    def advance(self, mat, cfg, u, v, plastic=None, c=None, q=None, p=None, vgrip=None, flags=None,
                k_sched=None, acc=None):
        """Multi-time-step run; `acc` ([d, n], optional) receives the last
        inner step's momentum sum per unit mass, fixed particles included."""
        k_out = np.zeros(cfg.n_slow, np.int64)
        ke_out = np.zeros(cfg.n_slow)
        conv = np.zeros(cfg.n_slow, np.int32)
        if k_sched is not None:
            k_sched = np.ascontiguousarray(k_sched, dtype=np.int64)
        rc = self.lib.orc_advance(self._h, C.byref(mat), C.byref(cfg), _ptr(self._a(u)), _ptr(self._a(v)),
                                  _ptr(self._a(plastic)), _ptr(self._a(c)), _ptr(self._a(q)), _ptr(self._a(p)),
                                  _ptr(self._a(vgrip)), _ptr(flags), _ptr(k_sched), _ptr(k_out), _ptr(ke_out),
                                  _ptr(conv), _ptr(self._a(acc)))
        return rc, k_out, ke_out, conv
