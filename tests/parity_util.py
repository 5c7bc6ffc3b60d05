"""Shared helpers of the GPU parity tests: build both sides on the same seeded
input and move arrays between numpy (oracle) and torch (HIP library)."""
import numpy as np

from paper_2309_04010_amd import binding as B
from paper_2309_04010_amd import cases

TOL = {B.SPH_F64: 1e-10, B.SPH_F32: 1e-4}


def rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    scale = np.abs(want).max() if want.size else 0.0
    if scale == 0.0:
        return float(np.abs(got).max()) if got.size else 0.0
    return float(np.abs(got - want).max() / scale)


def rel_err_elem(got, want, floor):
    """Largest elementwise error relative to |want| + floor * max|want|: small
    entries are held to nearly their own size, not to the field's maximum."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    if not want.size:
        return 0.0
    scale = np.abs(want) + floor * np.abs(want).max()
    if not np.all(scale > 0):
        return float(np.abs(got - want).max())
    return float((np.abs(got - want) / scale).max())


def dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.contiguous().cuda()


def host(t):
    return t.detach().double().cpu().numpy() if t.dtype.is_floating_point else t.cpu().numpy()


def torch_dtype(prec):
    import torch
    return torch.float32 if prec == B.SPH_F32 else torch.float64


def build_pair(oracle_mod, dim, X, V, h):
    """Oracle and GPU neighbourhoods of one input."""
    o = oracle_mod.Oracle(dim, X, V, h)
    nb = B.sph_build_neighbors(dev(X), dev(V), h)
    return o, nb


def material_pair(o, kw):
    return o.material(**kw), B.material(**{k: v for k, v in kw.items()})


def jittered(shape, dp=1e-3, jitter=0.1, seed=0):
    X, idx = cases.lattice(shape, dp, jitter=jitter, seed=seed)
    return X, np.full(X.shape[1], dp ** len(shape)), 1.3 * dp
