"""Seeded synthetic inputs: particle lattices, boundary flags and parameters.

This module only *generates inputs* (positions, volumes, flags, prescribed
grip velocities, material and schedule parameters).  It holds none of the
method's arithmetic: kernel sums, moduli conversions inside the method, time
step formulas and every SPH operator live on each side separately (the GPU
library and the CPU oracle).  Both sides draw their inputs from here.

Geometry follows the paper's test shapes (a bar stretched by grips at its
ends, a thin strip or plate swelling by water diffusion, Sec. 5), at the sizes
and parameter values of the five benchmark workloads:

  bar2d     2D bar 40 x 8, linear elastic, grips at both ends, loading.
  strip2d   2D strip 200 x 10, neo-Hookean + swelling, diffusion from the top.
  neck3d    3D bar 100 x 20 x 20, J2 nonlinear hardening, symmetric pull.
  plate3d   3D plate 500 x 500 x 4, neo-Hookean + swelling, diffusion patch.
  necking2d the paper's 2D necking bar (53.334 x 12.826 mm, 1.8% imperfection).
  necking3d the paper's 3D necking cylinder (r 6.413 mm, 53.334 mm, dp 0.3 mm).
  strips2d  64 strips of log-uniform sizes (batched parameter sweep).

Damping viscosity eta: the bars use the paper's 1e4.  For the swelling strip
and plate, whose spacings (12.5 and 31.25 micrometres) are far finer than the
paper's, the paper's 1e3 / 1e4 put the velocity-diffusion number
eta dt_s / (rho dp^2) near 100-400, where the sequential pairwise damping sweep
destabilises the explicit step (measured on the oracle: stable up to about 1,
divergent beyond about 3).  Those workloads use eta with a diffusion number
near 1 (strip 10, plate 20, sweep 5), fixed here once.

Positions are X = ((i + 1/2) dp, (j + 1/2) dp, (k + 1/2) dp) with particle id
i + nx (j + ny k); jitter, when asked for, is U(-a dp, a dp) drawn with
numpy.default_rng(seed) as an (n, dim) array in id order (x, then y, then z).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

FIXED, CDIR, GRIP = 1, 2, 4
LE, NH, J2 = 0, 1, 2
LOAD, DIFFUSION, DIFFUSION_COUPLED = 0, 1, 2


def lattice(shape, dp, jitter=0.0, seed=None):
    """Reference positions [dim, n] (float64) of a cartesian particle lattice."""
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    idx = np.indices(shape[::-1]).reshape(dim, -1)[::-1]  # idx[0] fastest
    X = (idx.astype(np.float64) + 0.5) * dp
    if jitter:
        rng = np.random.default_rng(seed)
        X = X + rng.uniform(-jitter * dp, jitter * dp, size=(X.shape[1], dim)).T
    return np.ascontiguousarray(X), idx


@dataclass
class Case:
    name: str
    dim: int
    shape: tuple
    dp: float
    X: np.ndarray                 # [dim, n] input order
    V: np.ndarray                 # [n]
    h: float
    flags: np.ndarray             # [n] uint8
    vgrip: np.ndarray | None      # [dim, n] prescribed grip velocity (loading)
    c_init: np.ndarray | None     # [n] initial saturation
    material: dict
    run: dict                     # multirate schedule parameters
    observable: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.X.shape[1]


def _sizes_ok(shape):
    for s in shape:
        if s < 1:
            raise ValueError("lattice extent must be positive")


def bar2d(nx=40, ny=8, dp=0.25e-3, grip_layers=3, pull=1.0e-3, dt_l=1.0e-3, n_slow=100,
          eta=1.0e4, ke_rel=1.0e-8, affine=False):
    """2D bar stretched in x.  Left `grip_layers` columns clamped; right ones
    moved at `pull` m/s.  With `affine`, both grips follow the homogeneous
    plane-strain uniaxial field u_x = e X, u_y = -nu/(1-nu) e Y (the elastic
    analytic solution), so the converged interior is that affine field."""
    _sizes_ok((nx, ny))
    X, idx = lattice((nx, ny), dp)
    n = X.shape[1]
    V = np.full(n, dp * dp)
    E, nu, rho = 210.0e9, 0.3, 7850.0
    flags = np.zeros(n, np.uint8)
    vgrip = np.zeros((2, n))
    left = idx[0] < grip_layers
    right = idx[0] >= nx - grip_layers
    flags[left | right] = FIXED
    L = nx * dp
    if affine:
        # strain rate of the homogeneous field (whole bar length L between the
        # grip mid-planes is irrelevant: the field is affine everywhere)
        erate = pull / L
        grips = left | right
        flags[grips] |= GRIP
        xc = X[0] - 0.5 * L
        yc = X[1] - 0.5 * ny * dp
        vgrip[0, grips] = erate * xc[grips]
        vgrip[1, grips] = -nu / (1.0 - nu) * erate * yc[grips]
    else:
        flags[right] |= GRIP
        vgrip[0, right] = pull
    # reference energy 1/2 F delta with the plane-strain bar stiffness
    W = ny * dp
    L_free = (nx - 2 * grip_layers) * dp
    delta_total = pull * dt_l * n_slow
    F_ref = E / (1.0 - nu * nu) * W * delta_total / L_free
    E_ref = 0.5 * F_ref * delta_total
    return Case("bar2d", 2, (nx, ny), dp, X, V, 1.3 * dp, flags, vgrip, None,
                dict(model=LE, E=E, nu=nu, rho0=rho),
                dict(n_slow=n_slow, slow_kind=LOAD, dt_slow=dt_l, eta=eta, ke_tol=ke_rel * E_ref,
                     k_max=0, fixed_inner=0, D=0.0, c_bc=0.0),
                dict(E_ref=E_ref, erate=pull / L))


def strip2d(nx=200, ny=10, dp=12.5e-6, clamp_layers=3, E=100.0e6, nu=0.4, D=1.0e-10,
            n_slow=100, eta=10.0, k_max=100000, fixed_inner=0, ke_frac=1.0e-8):
    """2D strip, water entering through the top row (Dirichlet c = a = 0.4),
    swelling through p = C (c - c0); both ends clamped."""
    _sizes_ok((nx, ny))
    X, idx = lattice((nx, ny), dp)
    n = X.shape[1]
    V = np.full(n, dp * dp)
    rho, C_swell, a_por = 2000.0, 3.0e6, 0.4
    flags = np.zeros(n, np.uint8)
    flags[(idx[0] < clamp_layers) | (idx[0] >= nx - clamp_layers)] |= FIXED
    flags[idx[1] == ny - 1] |= CDIR
    c_init = np.zeros(n)
    c_init[idx[1] == ny - 1] = a_por      # the boundary value holds from t = 0
    # density kinetic energy sum(1/2 m v^2) / sum(V) <= frac * C * a; the
    # paper's frac = 5e-4 stops after a single inner step at this spacing, so
    # the workload uses 1e-8 (about 150-250 inner steps per diffusion step)
    ke_tol = ke_frac * C_swell * a_por * V.sum()
    mid = (idx[0] == nx // 2) & (idx[1] == ny - 1)
    return Case("strip2d", 2, (nx, ny), dp, X, V, 1.3 * dp, flags, None, c_init,
                dict(model=NH, E=E, nu=nu, rho0=rho, C_swell=C_swell, c0=0.0),
                dict(n_slow=n_slow, slow_kind=DIFFUSION, dt_slow=0.0, eta=eta, ke_tol=ke_tol,
                     k_max=k_max, fixed_inner=fixed_inner, D=D, c_bc=a_por),
                dict(J_index=np.nonzero(mid)[0], J_component=1))


def neck3d(nx=100, ny=20, nz=20, dp=0.53334e-3, grip_layers=3, total_stretch=7.0e-3,
           n_slow=100, dt_l=1.0, fixed_inner=1000, eta=1.0e4, jitter=0.01, seed=3):
    """3D bar with J2 plasticity, pulled symmetrically at both ends."""
    _sizes_ok((nx, ny, nz))
    X, idx = lattice((nx, ny, nz), dp, jitter=jitter, seed=seed)
    n = X.shape[1]
    V = np.full(n, dp ** 3)
    mu, K = 80.1938e9, 164.21e9       # shear and bulk moduli of the necking table
    E = 9.0 * K * mu / (3.0 * K + mu)
    nu = (3.0 * K - 2.0 * mu) / (2.0 * (3.0 * K + mu))
    flags = np.zeros(n, np.uint8)
    vgrip = np.zeros((3, n))
    left = idx[0] < grip_layers
    right = idx[0] >= nx - grip_layers
    flags[left | right] = FIXED | GRIP
    vpull = 0.5 * total_stretch / (n_slow * dt_l)
    vgrip[0, left] = -vpull
    vgrip[0, right] = vpull
    return Case("neck3d", 3, (nx, ny, nz), dp, X, V, 1.3 * dp, flags, vgrip, None,
                dict(model=J2, E=E, nu=nu, rho0=7850.0, sigma0=200.0e6, sigma_inf=400.0e6,
                     delta=16.0, H=0.0),
                dict(n_slow=n_slow, slow_kind=LOAD, dt_slow=dt_l, eta=eta, ke_tol=0.0, k_max=0,
                     fixed_inner=fixed_inner, D=0.0, c_bc=0.0))


# Necking table (Sec. 5.1): shear and bulk moduli, initial and saturation flow
# stress, saturation exponent, linear hardening coefficient
NECK_TABLE = dict(mu=80.1938e9, K=164.21e9, sigma0=450.0e6, sigma_inf=715.0e6, delta=16.93,
                  H=129.24e6)
NECK_LENGTH, NECK_WIDTH, NECK_RADIUS = 53.334e-3, 12.826e-3, 6.413e-3


def _neck_material(rho0=7850.0):
    t = NECK_TABLE
    mu, K = t["mu"], t["K"]
    E = 9.0 * K * mu / (3.0 * K + mu)
    nu = (3.0 * K - 2.0 * mu) / (2.0 * (3.0 * K + mu))
    return dict(model=J2, E=E, nu=nu, rho0=rho0, sigma0=t["sigma0"], sigma_inf=t["sigma_inf"],
                delta=t["delta"], H=t["H"])


def _taper(x, x_c, half_length, imperfection):
    """Cross-section scale of the imperfect specimen: 1 - imperfection at the
    centre, rising linearly to 1 at the specimen's ends (and beyond)."""
    return 1.0 - imperfection * np.clip(1.0 - np.abs(x - x_c) / half_length, 0.0, 1.0)


def _neck_run(n_slow, t_end, inner, eta):
    return dict(n_slow=n_slow, slow_kind=LOAD, dt_slow=t_end / n_slow, eta=eta, ke_tol=0.0,
                k_max=0, fixed_inner=inner, D=0.0, c_bc=0.0)


def necking2d(across=50, grip_layers=3, total_stretch=10.0e-3, t_end=100.0, n_slow=10000,
              inner=33, eta=1.0e4, imperfection=0.018):
    """2D tensile necking bar (Sec. 5.1), plane strain.

    The specimen is 53.334 x 12.826 mm with dp = width / `across` (0.25652 mm
    at 50), its width reduced by `imperfection` at the centre, tapering
    linearly to the full width at its ends: y is scaled about the centre line
    and the volumes with it.  `grip_layers` extra columns at each end are
    the grips, pulled apart symmetrically at total_stretch / (2 t_end) each.
    Loading is displacement control in `n_slow` increments; every increment
    is followed by `inner` relaxation steps (see the workload notes for why a
    fixed count).  Observables, as weights: the reaction force per unit depth
    on the right grip (`w_acc`, applied to the momentum sum per unit mass of
    the last inner step) and the inward displacement of the width at the
    centre section, averaged over its top and bottom particles (`w_u`)."""
    _sizes_ok((across,))
    dp = NECK_WIDTH / across
    nxs = int(round(NECK_LENGTH / dp))
    nx, ny = nxs + 2 * grip_layers, across
    X, idx = lattice((nx, ny), dp)
    n = X.shape[1]
    x_c, y_c = 0.5 * nx * dp, 0.5 * ny * dp
    s = _taper(X[0], x_c, 0.5 * nxs * dp, imperfection)
    X[1] = y_c + (X[1] - y_c) * s
    V = dp * dp * s
    mat = _neck_material()
    flags = np.zeros(n, np.uint8)
    vgrip = np.zeros((2, n))
    left = idx[0] < grip_layers
    right = idx[0] >= nx - grip_layers
    flags[left | right] = FIXED | GRIP
    v_pull = 0.5 * total_stretch / t_end
    vgrip[0, left] = -v_pull
    vgrip[0, right] = v_pull
    w_acc = np.zeros((2, n))
    w_acc[0, right] = -mat["rho0"] * V[right]
    centre = np.isin(idx[0], [(nx - 1) // 2, nx // 2])
    top, bot = centre & (idx[1] == ny - 1), centre & (idx[1] == 0)
    w_u = np.zeros((2, n))
    w_u[1, top] = -0.5 / top.sum()
    w_u[1, bot] = 0.5 / bot.sum()
    return Case("necking2d", 2, (nx, ny), dp, X, V, 1.3 * dp, flags, vgrip, None, mat,
                _neck_run(n_slow, t_end, inner, eta),
                dict(w_acc=w_acc, w_u=w_u, v_pull=v_pull, length=nxs * dp, width=NECK_WIDTH,
                     radius=0.5 * NECK_WIDTH, total_stretch=total_stretch,
                     J_index=np.nonzero(top)[0], J_component=1))


def necking3d(dp=0.3e-3, grip_layers=3, total_stretch=14.0e-3, t_end=100.0, n_slow=10000,
              inner=32, eta=1.0e4, imperfection=0.018):
    """3D tensile necking cylinder (Sec. 5.2): radius 6.413 mm, length
    53.334 mm, axis along x.  Particles are the cubic-lattice sites (spacing
    dp, sites at half-integer offsets from the axis) within the radius; the
    radius is reduced by `imperfection` at the centre, tapering linearly to
    the ends (y, z scaled about the axis, volumes by the square of the
    scale).  `grip_layers` extra slices at each end are the grips, pulled
    apart at total_stretch / (2 t_end) each (0.7e-4 m/s, 7 mm per end).
    Observables: the reaction force on the right grip (`w_acc`) and the
    inward radial displacement of the outer ring of the centre section
    (`w_u`)."""
    R = NECK_RADIUS
    m = int(np.ceil(R / dp))
    nxs = int(round(NECK_LENGTH / dp))
    nx = nxs + 2 * grip_layers
    Xb, idx = lattice((nx, 2 * m, 2 * m), dp)
    yz = Xb[1:] - m * dp
    rho = np.sqrt((yz ** 2).sum(axis=0))
    keep = rho <= R
    X = np.ascontiguousarray(np.vstack([Xb[:1], yz])[:, keep])
    idx = idx[:, keep]
    rho = rho[keep]
    n = X.shape[1]
    x_c = 0.5 * nx * dp
    s = _taper(X[0], x_c, 0.5 * nxs * dp, imperfection)
    X[1:] *= s
    V = dp ** 3 * s * s
    mat = _neck_material()
    flags = np.zeros(n, np.uint8)
    vgrip = np.zeros((3, n))
    left = idx[0] < grip_layers
    right = idx[0] >= nx - grip_layers
    flags[left | right] = FIXED | GRIP
    v_pull = 0.5 * total_stretch / t_end
    vgrip[0, left] = -v_pull
    vgrip[0, right] = v_pull
    w_acc = np.zeros((3, n))
    w_acc[0, right] = -mat["rho0"] * V[right]
    centre = np.isin(idx[0], [(nx - 1) // 2, nx // 2])
    ring = centre & (rho > rho[centre].max() - 0.5 * dp)
    w_u = np.zeros((3, n))
    w_u[1, ring] = -(X[1, ring] / np.sqrt(X[1, ring] ** 2 + X[2, ring] ** 2)) / ring.sum()
    w_u[2, ring] = -(X[2, ring] / np.sqrt(X[1, ring] ** 2 + X[2, ring] ** 2)) / ring.sum()
    return Case("necking3d", 3, (nx, 2 * m, 2 * m), dp, X, V, 1.3 * dp, flags, vgrip, None, mat,
                _neck_run(n_slow, t_end, inner, eta),
                dict(w_acc=w_acc, w_u=w_u, v_pull=v_pull, length=nxs * dp, radius=R,
                     total_stretch=total_stretch, J_index=np.nonzero(ring)[0], J_component=1))


def plate3d(nx=500, ny=500, nz=4, dp=31.25e-6, clamp_layers=3, patch=0.3, wet_layers=2,
            E=100.0e6, nu=0.4, D=1.0e-10, C_swell=3.0e6, n_slow=50, fixed_inner=1000,
            eta=20.0):
    """3D thin plate, clamped on its four side faces, wetted on the top layers
    of a central patch; observable = mean u_z of the centre columns."""
    _sizes_ok((nx, ny, nz))
    X, idx = lattice((nx, ny, nz), dp)
    n = X.shape[1]
    V = np.full(n, dp ** 3)
    flags = np.zeros(n, np.uint8)
    side = ((idx[0] < clamp_layers) | (idx[0] >= nx - clamp_layers) |
            (idx[1] < clamp_layers) | (idx[1] >= ny - clamp_layers))
    flags[side] |= FIXED
    px0 = int(round(nx * (1 - patch) / 2)); px1 = nx - px0
    py0 = int(round(ny * (1 - patch) / 2)); py1 = ny - py0
    wet = ((idx[0] >= px0) & (idx[0] < px1) & (idx[1] >= py0) & (idx[1] < py1) &
           (idx[2] >= nz - wet_layers))
    flags[wet] |= CDIR
    c_init = np.zeros(n)
    c_init[wet] = 0.4                     # the boundary value holds from t = 0
    ci, cj = (nx - 1) // 2, (ny - 1) // 2
    centre = np.isin(idx[0], [ci, ci + 1]) & np.isin(idx[1], [cj, cj + 1])
    return Case("plate3d", 3, (nx, ny, nz), dp, X, V, 1.3 * dp, flags, None, c_init,
                dict(model=NH, E=E, nu=nu, rho0=2000.0, C_swell=C_swell, c0=0.0),
                dict(n_slow=n_slow, slow_kind=DIFFUSION, dt_slow=0.0, eta=eta, ke_tol=0.0,
                     k_max=0, fixed_inner=fixed_inner, D=D, c_bc=0.4),
                dict(J_index=np.nonzero(centre)[0], J_component=2))


def strips_sweep(n_strips=64, seed=5, dp=12.5e-6, n_min=1000, n_max=50000, rows=10,
                 n_slow=10, fixed_inner=200):
    """Batched sweep: strips of log-uniform size with E ~ U(50, 200) MPa and
    D ~ LogU(1e-11, 1e-9); draws in this order: sizes, E, D."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(np.log(n_min), np.log(n_max), n_strips))).astype(int)
    Es = rng.uniform(50.0e6, 200.0e6, n_strips)
    Ds = np.exp(rng.uniform(np.log(1e-11), np.log(1e-9), n_strips))
    out = []
    for N, E, D in zip(sizes, Es, Ds):
        ncol = max(int(round(N / rows)), 8)
        out.append(strip2d(nx=ncol, ny=rows, dp=dp, E=float(E), D=float(D), n_slow=n_slow,
                           fixed_inner=fixed_inner, eta=5.0))
    return out


@dataclass
class Batch:
    """Several specimens as one particle set, specimen after specimen in input
    order.  Each specimen keeps its own cell grid, so they may overlap in
    space; `batch(..., stack=True)` still stacks them along y for clarity."""
    cases: list
    X: np.ndarray          # [dim, n] input order, specimen after specimen
    V: np.ndarray
    h: float
    flags: np.ndarray
    c_init: np.ndarray
    spec: np.ndarray       # [n] int32 specimen id
    offsets: np.ndarray    # [n_spec + 1] input-order ranges
    material: dict         # shared values (E is per specimen)
    run: dict              # shared schedule (D per specimen; each side derives the step sizes)
    E: np.ndarray
    D: np.ndarray

    @property
    def n(self):
        return self.X.shape[1]

    @property
    def dim(self):
        return self.X.shape[0]


def batch(cs, gap_dp=4.0, stack=True):
    """2D diffusion specimens of equal dp, h, nu, rho0, C_swell, eta and
    schedule as one Batch; per-specimen E and D (the step sizes that follow
    from them are left to each side)."""
    c0 = cs[0]
    dp, h = c0.dp, c0.h
    Xs, y0, offs = [], 0.0, [0]
    for c in cs:
        assert c.dim == 2 and c.dp == dp and c.h == h
        X = c.X.copy()
        if stack:
            X[1] += y0 - X[1].min() + 0.5 * dp
            y0 = X[1].max() + gap_dp * dp
        Xs.append(X)
        offs.append(offs[-1] + c.n)
    E = np.array([c.material["E"] for c in cs])
    D = np.array([c.run["D"] for c in cs])
    m = c0.material
    spec = np.concatenate([np.full(c.n, i, np.int32) for i, c in enumerate(cs)])
    return Batch(list(cs), np.hstack(Xs), np.concatenate([c.V for c in cs]), h,
                 np.concatenate([c.flags for c in cs]), np.concatenate([c.c_init for c in cs]),
                 spec, np.array(offs), dict(m), dict(c0.run), E, D)


def by_name(name, **kw):
    return {"bar2d": bar2d, "strip2d": strip2d, "neck3d": neck3d, "plate3d": plate3d,
            "necking2d": necking2d, "necking3d": necking3d}[name](**kw)
