"""Per-kernel timing: every kernel class by default, only the selected classes
after sph_profile_classes, nothing while disabled (enabling or disabling
resets the counters)."""
import numpy as np
import pytest

from paper_2309_04010_amd import binding as B
from paper_2309_04010_amd import cases

from .parity_util import dev

pytestmark = pytest.mark.gpu


def test_profile_classes():
    c = cases.strip2d(nx=40, ny=8, n_slow=1, fixed_inner=6, k_max=0)
    nb = B.sph_build_neighbors(dev(c.X), dev(c.V), c.h)
    st = B.new_state(nb, B.SPH_F64, with_diffusion=True)
    st.flags = dev(c.flags[nb.host("perm").astype(np.int64)])
    mat = B.material(**c.material)
    cfg = B.multirate_cfg(**c.run)

    B.sph_profile_enable(nb, True)
    B.sph_advance_multirate(nb, mat, st, cfg)
    every = B.sph_profile_read(nb)
    for k in ("stress", "momentum", "damping", "drift_ke", "diff_grad", "diff_div"):
        assert every[k][0] > 0 and every[k][1] > 0, k
    assert every["damping"][0] == 6 * nb.info.n_colors

    B.sph_profile_classes(nb, ["damping"])
    B.sph_profile_enable(nb, True)  # resets the counters
    B.sph_advance_multirate(nb, mat, st, cfg)
    only = B.sph_profile_read(nb)
    assert only["damping"][0] == every["damping"][0]
    assert all(v[0] == 0 for k, v in only.items() if k != "damping")

    B.sph_profile_enable(nb, False)  # resets the counters; nothing is timed
    B.sph_profile_classes(nb, None)
    B.sph_advance_multirate(nb, mat, st, cfg)
    assert all(v[0] == 0 for v in B.sph_profile_read(nb).values())
    nb.close()
