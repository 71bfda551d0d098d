"""Voronoi areal weights (CPU): closed forms and invariants."""
import numpy as np
import pytest

from paper_2011_11120_amd import geometry, synth


def test_regular_grid_cells_are_dx_squared():
    gx, gy = synth.grid_xy(5, 4, 15.0)
    w = geometry.voronoi_areas(gx, gy)
    assert np.allclose(w, 225.0, rtol=2e-3)


def test_two_points_split_the_rectangle():
    w = geometry.voronoi_areas([0.0, 10.0], [0.0, 0.0], bounds=(-5.0, 15.0, -4.0, 4.0), pixel=0.05)
    assert np.allclose(w, [80.0, 80.0], rtol=1e-6)


def test_areas_sum_to_the_rectangle():
    rng = np.random.default_rng(0)
    x, y = rng.uniform(0, 100, 40), rng.uniform(0, 60, 40)
    w = geometry.voronoi_areas(x, y, bounds=(0.0, 100.0, 0.0, 60.0), pixel=0.25)
    assert abs(w.sum() - 6000.0) < 1e-6 * 6000.0
    assert np.all(w > 0)


def test_random_half_grid_doubles_the_mean_area():
    """The paper's irregular case: a random half of a 15 m grid; mean cell ~ 2 * 15^2."""
    nx = 30
    idx = synth.irregular_subset(nx, nx, 0.5)
    assert idx.size == nx * nx // 2 and np.all(np.diff(idx) > 0)
    gx, gy = synth.grid_xy(nx, nx, 15.0)
    w = geometry.voronoi_areas(gx[idx], gy[idx], bounds=(-7.5, 442.5, -7.5, 442.5), pixel=0.75)
    assert abs(w.mean() - 2 * 225.0) < 1e-6 * 450.0
    assert w.std() > 0.1 * w.mean()  # irregular: the cells differ


@pytest.mark.parametrize("sigma", [40.0, 90.0])
def test_voronoi_quadrature_of_a_smooth_field(sigma):
    """Voronoi-weighted sums integrate a smooth field over the surface far better than equal weights."""
    from scipy.special import erf
    nx, dx, c = 30, 15.0, 217.5
    idx = synth.irregular_subset(nx, nx, 0.5)
    gx, gy = synth.grid_xy(nx, nx, dx)
    b = (-7.5, 442.5, -7.5, 442.5)
    w = geometry.voronoi_areas(gx[idx], gy[idx], bounds=b, pixel=0.75)
    f = np.exp(-((gx[idx] - c) ** 2 + (gy[idx] - c) ** 2) / (2 * sigma ** 2))
    side = sigma * np.sqrt(np.pi / 2) * (erf((b[1] - c) / (sigma * np.sqrt(2))) - erf((b[0] - c) / (sigma * np.sqrt(2))))
    exact = side * side
    vor = abs(np.sum(f * w) - exact) / exact
    uni = abs(np.sum(f) * (450.0 ** 2 / idx.size) - exact) / exact
    assert vor < 2e-3 and vor < 0.1 * uni
