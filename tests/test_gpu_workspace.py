"""The per-step scratch handed in by the caller (sph_workspace_size,
sph_set_workspace): a taped forward + reverse run, and the whole-run graph,
give bitwise the results of the handle's own scratch, also when the caller's
memory held other bytes before it was handed in (the gradient partials are
cleared and the damping records laid out again); going back to the
handle's own scratch keeps them; a workspace that is too small or not at a
256-byte boundary is refused."""
import numpy as np
import pytest
import torch

from paper_2309_04010_amd import adjoint as A
from paper_2309_04010_amd import binding as B
from paper_2309_04010_amd import cases

from .parity_util import dev

pytestmark = pytest.mark.gpu


def _run(pr, th, w):
    u = pr.forward(th).clone()
    g = pr.backward(w, recompute=True)
    return u, g.clone(), pr.adj.u.clone()


@pytest.mark.parametrize("prec", [B.SPH_F64, B.SPH_F32], ids=["f64", "f32"])
def test_caller_workspace_equals_own(oracle_mod, prec):
    print(f"[workspace] strip2d prec={prec}", flush=True)
    c = cases.strip2d(nx=24, ny=6, n_slow=3, fixed_inner=20, k_max=0)
    pr = A.MultirateProblem(c, prec, k_hist=20)
    th = pr.theta0()
    w = dev(np.random.default_rng(5).normal(0.0, 1.0, (2, c.n)))
    ref = _run(pr, th, w)
    need = B.sph_workspace_size(pr.nb)
    assert need > 0
    ws = torch.full((need + 512,), 0xAB, dtype=torch.uint8, device="cuda")
    assert ws.data_ptr() % 256 == 0
    B.sph_set_workspace(pr.nb, ws)
    got = _run(pr, th, w)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    # a second run on the caller's scratch, then back to the handle's own
    got2 = _run(pr, th, w)
    assert all(torch.equal(a, b) for a, b in zip(ref, got2))
    B.sph_set_workspace(pr.nb, None)
    got3 = _run(pr, th, w)
    assert all(torch.equal(a, b) for a, b in zip(ref, got3))
    pr.close()


def test_caller_workspace_whole_run_graph(oracle_mod):
    """The cached whole-run graph is dropped when the scratch moves: the
    graph launched on the caller's workspace equals the eager pair."""
    c = cases.strip2d(nx=20, ny=6, n_slow=2, fixed_inner=12, k_max=0)
    pr = A.MultirateProblem(c, B.SPH_F64, k_hist=12)
    th = pr.theta0()
    w = dev(np.random.default_rng(3).normal(0.0, 1.0, (2, c.n)))

    def graph():
        pr.reset()
        a = pr.adj.zero_()
        a.u.copy_(w)
        B.sph_advance_multirate_graph(pr.nb, pr._material(th), pr.st, pr._cfg(th), pr.tape, a)
        return pr.st.u.clone(), a.grad.clone()

    pr.forward(th)
    ge = pr.backward(w).clone()
    ue = pr.st.u.clone()
    u1, g1 = graph()                     # recorded on the handle's own scratch
    assert torch.equal(u1, ue) and torch.equal(g1, ge)
    ws = torch.full((B.sph_workspace_size(pr.nb),), 7, dtype=torch.uint8, device="cuda")
    B.sph_set_workspace(pr.nb, ws)
    u2, g2 = graph()                     # recorded again on the caller's
    assert torch.equal(u2, ue) and torch.equal(g2, ge)
    pr.close()


def test_workspace_rejects_small_or_misaligned(oracle_mod):
    c = cases.strip2d(nx=12, ny=4, n_slow=1, fixed_inner=5, k_max=0)
    nb = B.sph_build_neighbors(dev(c.X), dev(c.V), c.h)
    need = B.sph_workspace_size(nb)
    small = torch.zeros((need - 1,), dtype=torch.uint8, device="cuda")
    with pytest.raises(B.SphError) as e:
        B.sph_set_workspace(nb, small)
    assert e.value.code == B.SPH_E_ARG
    big = torch.zeros((need + 512,), dtype=torch.uint8, device="cuda")
    with pytest.raises(B.SphError) as e:
        B.sph_set_workspace(nb, big[1:])
    assert e.value.code == B.SPH_E_ARG
    assert B.sph_workspace_size(nb) == need
    nb.close()
