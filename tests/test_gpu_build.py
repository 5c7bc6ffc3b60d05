"""GPU parity of the neighbour build (integer work: bit-exact).

Cell keys, the stable radix sort (perm), cell ranges, CSR neighbour lists and
the damping schedule (pairs, levels, anchors, colour ranges) must equal the
oracle's exactly; the sorted positions/volumes are gathers (exact) and the
FP64 correction matrices agree to 1e-12.
"""
import numpy as np
import pytest

from paper_2309_04010_amd import binding as B
from paper_2309_04010_amd import cases

from .parity_util import build_pair, jittered, rel_err

pytestmark = pytest.mark.gpu

CASES = [
    ("bar2d-40x8", lambda: (lambda c: (2, c.X, c.V, c.h))(cases.bar2d())),
    ("strip2d-200x10", lambda: (lambda c: (2, c.X, c.V, c.h))(cases.strip2d())),
    ("jitter2d-37x23", lambda: (2, *jittered((37, 23), jitter=0.2, seed=1))),
    ("jitter3d-11x9x7", lambda: (3, *jittered((11, 9, 7), jitter=0.2, seed=2))),
    ("plate3d-40x40x4", lambda: (lambda c: (3, c.X, c.V, c.h))(cases.plate3d(nx=40, ny=40))),
    ("random3d", lambda: (3, np.random.default_rng(4).uniform(0, 9e-3, (3, 3000)),
                          np.full(3000, 2.4e-10), 1.0e-3)),
    ("tiny2d-2x2", lambda: (2, *jittered((2, 2), jitter=0.0))),
    ("line3d-1cell", lambda: (3, *jittered((3, 3, 3), jitter=0.05, seed=9))),
]


def _compare(o, nb):
    assert nb.info.n == o.n
    assert nb.info.n_pairs == o.n_pairs and nb.info.n_upairs == o.n_upairs
    assert nb.info.n_cells == o.n_cells and tuple(nb.info.ncell) == tuple(o.ncell)
    assert nb.info.max_deg == o.max_deg and nb.info.max_level == o.max_level
    assert nb.info.n_anchors == o.n_anchors
    assert list(nb.info.color_off) == o.color_off.tolist()
    assert np.array_equal(np.array(nb.info.origin), o.origin)
    for name, want in [("key", o.key), ("perm", o.perm), ("cell_start", o.cell_start),
                       ("nbr_off", o.nbr_off), ("nbr_idx", o.nbr_idx), ("sched_a", o.sched_a),
                       ("sched_b", o.sched_b), ("sched_level", o.sched_level),
                       ("anchor_key", o.anchor_key), ("anchor_off", o.anchor_off),
                       ("anchor_nlev", o.anchor_nlev)]:
        got = nb.host(name)
        assert got.shape == want.shape, name
        assert np.array_equal(got, want), f"{name} differs at {np.nonzero(got != want)[0][:8]}"
    assert np.array_equal(nb.host("X"), o.X)
    assert np.array_equal(nb.host("V"), o.V)
    assert rel_err(nb.host("B0"), o.B0) < 1e-12


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_build_bit_exact(oracle_mod, name, make):
    dim, X, V, h = make()
    print(f"[build parity] {name} n={X.shape[1]}", flush=True)
    o, nb = build_pair(oracle_mod, dim, X, V, h)
    _compare(o, nb)
    nb.close()


def test_build_full_size_plate(oracle_mod):
    """The 500 x 500 x 4 plate (1M particles) at full size: bit-exact too."""
    c = cases.plate3d()
    print(f"[build parity] plate3d full n={c.n}", flush=True)
    o, nb = build_pair(oracle_mod, 3, c.X, c.V, c.h)
    _compare(o, nb)
    nb.close()


def test_build_errors(oracle_mod):
    from .parity_util import dev
    X = np.stack([np.arange(10.0), np.zeros(10)])
    with pytest.raises(B.SphError) as e:
        B.sph_build_neighbors(dev(X), dev(np.ones(10)), 1.3)
    assert e.value.code == B.SPH_E_NUMERIC
    with pytest.raises(B.SphError) as e:
        B.sph_build_neighbors(dev(np.zeros((4, 10))), dev(np.ones(10)), 1.3)
    assert e.value.code == B.SPH_E_UNSUPPORTED
    with pytest.raises(B.SphError) as e:
        B.sph_build_neighbors(dev(X), dev(np.ones(10)), -1.0)
    assert e.value.code == B.SPH_E_ARG
    # no particles
    with pytest.raises(B.SphError) as e:
        B.sph_build_neighbors(dev(np.zeros((3, 0))), dev(np.zeros(0)), 1.0)
    assert e.value.code == B.SPH_E_ARG
