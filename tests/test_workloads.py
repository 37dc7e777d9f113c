"""The seeded input generators: banded sub-sampling equals sub-sampling every
cell, volumes match the shapes, wall faces carry no flow, draws are repeatable."""
import math

import numpy as np
import pytest

from paper_2012_11744_amd import workloads as W


def _ball_inside(centres, radii, per):
    def f(x, y, z):
        out = np.zeros(np.shape(x), dtype=bool)
        for (cx, cy, cz), r in zip(centres, radii):
            d = []
            for v, c, p in ((x, cx, per[0]), (y, cy, per[1]), (z, cz, per[2])):
                dd = v - c
                if p:
                    dd = dd - np.round(dd)
                d.append(dd)
            out |= d[0] ** 2 + d[1] ** 2 + d[2] ** 2 < r * r
        return out
    return f


def test_config1_matches_brute_force():
    w = W.config1(16)
    C = W.brute_force_fraction(w.n, w.h, _ball_inside([[0.5, 0.5, 0.5]], [0.25], (1, 1, 1)))
    assert np.array_equal(w.liquid_fraction, C)
    assert np.allclose(w.rho, 10.0 * C + 1.0 * (1 - C))


def test_config2_matches_brute_force():
    w = W.config2(32)
    g = w.geometry
    gas = W.brute_force_fraction(w.n, w.h, _ball_inside(g["centres"], g["radii"], (0, 0, 0)))
    assert np.array_equal(w.liquid_fraction, 1.0 - gas)
    # gravity on interior z faces only, wall faces zero
    assert np.all(w.us[2][0] == 0.0)
    assert np.all(w.us[0][:, :, 0] == 0.0) and np.all(w.us[1][:, 0, :] == 0.0)


def test_config3_matches_brute_force():
    w = W.config3(32)
    g = w.geometry
    balls = _ball_inside(g["centres"], g["radii"], (1, 1, 0))

    def inside(x, y, z):
        return (z < 0.5 + 0.05 * np.sin(2 * np.pi * x / 0.25)) | balls(x, y, z)
    C = W.brute_force_fraction(w.n, w.h, inside)
    assert np.array_equal(w.liquid_fraction, C)
    assert w.rho.min() == pytest.approx(1.2) and w.rho.max() == pytest.approx(1000.0)
    assert np.all(w.us[2][0] == 0.0)


def test_config5_matches_brute_force():
    w = W.config5(32)
    g = w.geometry

    def inside(x, y, z):
        th = np.arctan2(z - 0.5, y - 0.5)
        r = 0.1 + sum(0.01 * np.cos(2 * np.pi * g["k"][m] * x + g["n"][m] * th + g["phase"][m])
                      for m in range(5))
        return np.hypot(y - 0.5, z - 0.5) < r
    C = W.brute_force_fraction(w.n, w.h, inside)
    assert np.array_equal(w.liquid_fraction, C)


def test_sphere_volume():
    """The sub-sampled sphere volume is 4 pi R^3 / 3 up to the sub-sampling error."""
    w = W.config1(64)
    vol = w.liquid_fraction.sum() * w.h ** 3
    exact = 4.0 / 3.0 * math.pi * 0.25 ** 3
    assert abs(vol - exact) / exact < 2e-3
    assert w.liquid_fraction.min() == 0.0 and w.liquid_fraction.max() == 1.0


def test_repeatable_and_seeded():
    a = W.config4(16)
    b = W.config4(16)
    assert np.array_equal(a.us[0], b.us[0]) and np.array_equal(a.w, b.w)
    c = W.random_case((8, 6, 4), (0, 1, 0), seed=1)
    d = W.random_case((8, 6, 4), (0, 1, 0), seed=2)
    assert not np.array_equal(c.us[0], d.us[0])
    assert c.rho.shape == (4, 6, 8)
    assert np.all(c.us[1][:, 0, :] == 0.0)
