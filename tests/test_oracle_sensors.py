"""Pins for the point-sensor operator (Sec. 2.2)."""
import numpy as np
import pytest

from oracle import sensors as osens
from paper_2505_08482_amd.inputs import circle_sensors, pixel_centres


def test_weights_are_a_partition_of_unity():
    S = osens.sensor_matrix(40, 40, 1e-4, circle_sensors(37, 13.3e-4))
    W = S.toarray()
    assert (W >= 0).all()
    assert np.allclose(W.sum(axis=1), 1.0, atol=1e-15)
    assert ((W > 0).sum(axis=1) <= 4).all()


def test_sensor_on_a_cell_centre_samples_that_pixel():
    n, dx = 20, 1e-4
    xc = pixel_centres(n) * dx
    xy = np.array([[xc[3], xc[11]], [xc[15], xc[4]]])
    rng = np.random.default_rng(0)
    p = rng.standard_normal((2, n, n))
    d = osens.sample(osens.sensor_matrix(n, n, dx, xy), p)
    assert np.allclose(d[:, 0], p[:, 11, 3], atol=1e-14)
    assert np.allclose(d[:, 1], p[:, 4, 15], atol=1e-14)


def test_bilinear_is_exact_for_affine_fields():
    n, dx = 30, 1e-4
    X, Y = np.meshgrid(pixel_centres(n) * dx, pixel_centres(n) * dx)
    field = 3.0 + 2.0e3 * X - 7.0e3 * Y
    xy = circle_sensors(50, 9.7e-4)
    d = osens.sample(osens.sensor_matrix(n, n, dx, xy), field[None])
    assert np.allclose(d[0], 3.0 + 2.0e3 * xy[:, 0] - 7.0e3 * xy[:, 1], atol=1e-12)


def test_injection_is_the_transpose():
    n, dx, m = 24, 1e-4, 19
    S = osens.sensor_matrix(n, n, dx, circle_sensors(m, 8.1e-4))
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, n, n))
    r = rng.standard_normal((3, m))
    assert np.isclose(np.sum(osens.sample(S, x) * r), np.sum(x * osens.inject(S, r, n, n)), rtol=1e-14)


def test_out_of_range_sensor_raises():
    with pytest.raises(ValueError):
        osens.sensor_matrix(10, 10, 1e-4, np.array([[4.9e-4, 0.0]]))
