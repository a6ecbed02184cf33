"""Checks of the seeded input generators (determinism, shapes, the properties each recipe
states).  CPU only."""
import math

import numpy as np

import workloads as wl


def test_deterministic_and_shapes():
    a, _ = wl.sine_modes(16, 3)
    b, _ = wl.sine_modes(16, 3)
    assert a.shape == (16, 16, 16) and a.dtype == np.float64 and np.array_equal(a, b)
    c = wl.gaussian_clumps(16, 2)
    assert np.array_equal(c, wl.gaussian_clumps(16, 2)) and abs(c.mean()) < 1e-12
    g = wl.lognormal_grf(16, 2, remove_mean=False)
    assert np.all(g > 0)


def test_sphere_mass_by_volume_fraction():
    """10^3 sub-cell sampling of the cut cells gives the sphere's volume closely."""
    rho, c = wl.uniform_sphere(64, 4)
    vol = rho.sum() / 64 ** 3
    assert abs(vol - 4 * math.pi * 0.25 ** 3 / 3) / vol < 1e-3
    assert np.linalg.norm(c - 0.5) <= 0.05 + 1e-15


def test_clumps_match_direct_sum():
    """The matrix-product evaluation equals the clump-by-clump sum to round-off."""
    n = 32
    rho = wl.gaussian_clumps(n, 8, n_clumps=4, remove_mean=False)
    rng = np.random.default_rng(8)
    centres = rng.uniform(0, 1, (4, 3))
    widths = rng.uniform(0.01, 0.05, 4)
    amps = rng.lognormal(0, 1, 4)
    x = (np.arange(n) + 0.5) / n
    full = np.ones((n, n, n))
    for cc, w, a in zip(centres, widths, amps):
        g = []
        for d in range(3):
            dd = np.abs(x - cc[d])
            dd = np.minimum(dd, 1 - dd)
            g.append(np.exp(-0.5 * (dd / w) ** 2))
        full += a * g[2][:, None, None] * g[1][None, :, None] * g[0][None, None, :]
    assert np.max(np.abs(full - rho)) < 1e-12


def test_serving_trace():
    t = wl.serving_trace(100, 1, rate=50.0)
    assert len(t) == 100 and all(t[i]["t"] <= t[i + 1]["t"] for i in range(99))
    assert {r["n"] for r in t} <= {64, 128, 256, 512}
