"""The seeded input generators: shapes, ranges, neutrality and reproducibility."""
import numpy as np
import pytest

import workloads as wl


@pytest.mark.parametrize("idx,n", [(1, None), (2, None), (3, 20000), (4, None), (4, 1000), (4, 24)])
def test_config_inputs(idx, n):
    c = wl.make_config(idx, n_override=n)
    pos, q = c["pos"], c["q"]
    Lx, Ly, Lz = c["box"]
    assert pos.shape == (len(q), 3)
    assert np.all((pos[:, 0] >= 0) & (pos[:, 0] < Lx) & (pos[:, 1] >= 0) & (pos[:, 1] < Ly))
    assert np.all((pos[:, 2] >= 0) & (pos[:, 2] <= Lz))
    assert q.sum() == 0.0
    if idx == 4:
        assert set(np.unique(np.abs(q))) <= {1.0, 2.0}
        assert (q > 0).sum() == (q < 0).sum()
    else:
        assert set(np.unique(q)) == {-1.0, 1.0}
    c2 = wl.make_config(idx, n_override=n)
    assert np.array_equal(c2["pos"], pos) and np.array_equal(c2["q"], q)


def test_surface_excess_layers():
    c = wl.make_config(3, n_override=20000)
    z, q = c["pos"][:, 2], c["q"]
    n_ex = 20000 // 20
    # the excess cations sit in z < 1 and the excess anions in z > Lz - 1
    assert (q[z < 1.0] > 0).sum() - (q[z < 1.0] < 0).sum() > 0.8 * n_ex
    assert (q[z > 9.0] < 0).sum() - (q[z > 9.0] > 0).sum() > 0.8 * n_ex
