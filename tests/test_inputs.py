"""The seeded input generators: reproducibility, containment, non-overlap."""
import math

import numpy as np
import pytest

import seeded_inputs as si


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg5"])
def test_profiles_reproducible_and_valid(name):
    wl = si.WORKLOADS[name]
    for seed in range(6):
        a = si.draw_profile(wl, seed)
        assert a == si.draw_profile(wl, seed)
        half = wl.side / 2
        for s in a:
            assert abs(s.cx) + s.bound_radius <= half and abs(s.cy) + s.bound_radius <= half
        for i in range(len(a)):
            for j in range(i):
                d = math.hypot(a[i].cx - a[j].cx, a[i].cy - a[j].cy)
                assert d > a[i].bound_radius + a[j].bound_radius
        if name == "cfg1":
            assert len(a) == 2 and all(1.5 <= s.eps_r.real <= 2.5 for s in a)
        if name == "cfg2":
            assert 1 <= len(a) <= 3 and all(2.0 <= s.eps_r.real <= 4.0 for s in a)


def test_rasterize_area_fraction():
    lam = si.WORKLOADS["cfg1"].wavelength
    side = 2 * lam
    r = 0.3 * lam
    eps = si.rasterize([si.Shape("ellipse", 0.0, 0.0, r, r, 0.0, 3.0)], 64, side)
    area = np.sum(eps.real - 1.0) / 2.0 * (side / 64) ** 2
    assert abs(area / (math.pi * r * r) - 1) < 0.01
    assert np.all(eps.real >= 1.0) and np.all(eps.real <= 3.0)


def test_antennas_on_circle():
    xy = si.antenna_positions(8, 2.0)
    assert np.allclose(np.hypot(xy[:, 0], xy[:, 1]), 2.0)
    assert np.allclose(xy[0], [2.0, 0.0])
    jt, jr = si.draw_jitter(3, 8, 8, 2.0)
    assert np.max(np.abs(jt)) <= math.radians(2.0)
    assert not np.array_equal(jt, jr)


def test_uneven_shapes_recipe():
    a = si.uneven_shapes(300, seed=5)
    assert a == si.uneven_shapes(300, seed=5)
    assert all(M in (32, 48, 64, 96, 128) and n in (16, 24, 32, 48, 64) and K % 2 == 1 and 7 <= K <= min(21, M)
               for M, n, K in a)
    assert len(set(a)) > 40  # genuinely uneven
    assert {M for M, _, _ in a} == {32, 48, 64, 96, 128}
    small = si.uneven_shapes(50, seed=1, grids=(8,), truncations=(5, 7, 9))
    assert all(K <= 8 for _, _, K in small)
