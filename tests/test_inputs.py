"""The seeded input builders: shapes, normalisations and the wedge model."""
import math

import numpy as np

from paper_2308_06152_amd import inputs


def test_point_and_gaussian_sources_integrate_to_one():
    w = inputs.small_plain()
    b = w.rhs()
    assert b.shape == (w.ny, w.nx) and np.count_nonzero(b) == 1
    assert abs(b.sum() * w.hx * w.hy - 1) < 1e-12
    g = inputs.gaussian_source(257, 257, 1 / 256, 1 / 256, 128, 128, 2 / 256)
    assert abs(g.sum() / 256**2 - 1) < 1e-12
    assert g[128, 128] == g.max() and g[128, 127] == g[128, 129] == g[127, 128]


def test_wedge_layers_and_interfaces():
    w = inputs.wedge(1153, 1921)
    assert w.hx == w.hy == 600 / 1152
    c = inputs.wedge_velocity(w.nx, w.ny, w.hx, w.hy)
    assert c.shape == (1921, 1153)
    # top row 2000, bottom row 3000, every column passes 2000 -> 1500 -> 3000
    assert (c[-1] == 2000).all() and (c[0] == 3000).all()
    for i in (0, 576, 1152):
        col = c[:, i][::-1]  # from the top down
        changes = np.flatnonzero(np.diff(col)) + 1
        assert list(col[np.r_[0, changes]]) == [2000.0, 1500.0, 3000.0]
        x = i * w.hx
        up, lo = inputs.wedge_interfaces(x)
        y_first_1500 = -(changes[0]) * w.hy
        y_first_3000 = -(changes[1]) * w.hy
        assert up - w.hy - 1e-9 <= y_first_1500 < up
        assert lo - w.hy - 1e-9 <= y_first_3000 < lo
    k = w.kfield()
    assert abs(k.max() - 2 * math.pi * 40 / 1500) < 1e-15
    assert k.max() * w.hx < 0.09
    b = w.rhs()
    assert b[-1, 576] == 1 / (w.hx * w.hy) and np.count_nonzero(b) == 1


def test_wedge_scaled_grids_keep_kh():
    for nx, ny in ((73, 121), (145, 241), (577, 961)):
        w = inputs.wedge(nx, ny)
        assert abs(w.kfield().max() * w.hx - 2 * math.pi * 40 / 1500 * 600 / 1152) < 1e-12


def test_layered_model_and_sources():
    w = inputs.layered()
    assert (w.nx, w.ny, w.hx) == (2049, 1025, 5.0)
    c = inputs.layered_velocity(w.nx, w.ny, w.hx)
    assert c.min() >= 1275.0 - 1e-9 and c.max() <= 4500 * 1.15 + 1e-9
    # kh <= 0.49 at 20 Hz
    assert 2 * math.pi * 20 / c.min() * w.hx <= 0.49 + 1e-12
    # far from the anomalies each layer is constant along x
    assert len(np.unique(np.round(c[-1, :3], 9))) == 1
    b = w.sources()
    assert b.shape == (64, 1025, 2049)
    for s in (0, 17, 63):
        assert b[s, 1025 - 1 - 5, 16 + 32 * s] == 1 / 25.0
        assert np.count_nonzero(b[s]) == 1
