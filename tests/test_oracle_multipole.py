"""Pins of the oracle's multipole boundary (Appendix A): the harmonic table obeys the
addition theorem, the truncated expansion converges to the brute-force potential with the
expected (r'/r)^5 error, the sphere is a pure monopole, dipoles vanish about the centre of
mass, and a multipole-bounded solve reproduces the analytic sphere potential.  CPU only."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import MULTIPOLE


def _legendre(l, x):
    return [1.0, x, 0.5 * (3 * x * x - 1), 0.5 * (5 * x ** 3 - 3 * x),
            (35 * x ** 4 - 30 * x * x + 3) / 8.0][l]


def test_addition_theorem():
    """Point masses at a and unit G: the l-term of the expansion is -m r'^l P_l(cos g) / r^(l+1),
    so the table's real harmonics satisfy the addition theorem for every l <= 4."""
    rng = np.random.default_rng(0)
    for _ in range(5):
        a = rng.uniform(-0.2, 0.2, 3)
        b = rng.uniform(-1, 1, 3) * 3
        n = 1
        rho = np.ones((1, 1, 1))        # one cell of mass dx^3 at (dx/2, dx/2, dx/2)
        dx = 1.0
        origin = np.array([0.5, 0.5, 0.5]) - a
        for lmax in range(5):
            o, q = oracle.multipole_moments(rho, dx, lmax=lmax, origin=origin)
            phi = oracle.multipole_potential(*(origin + b), q, o, lmax=lmax)
            ra, rb = np.linalg.norm(a), np.linalg.norm(b)
            cg = float(a @ b) / (ra * rb)
            ref = -sum(ra ** l * _legendre(l, cg) / rb ** (l + 1) for l in range(lmax + 1))
            assert math.isclose(phi, ref, rel_tol=1e-12, abs_tol=1e-15), (lmax, phi, ref)


def test_far_field_matches_brute_force():
    """The l <= 4 expansion of a lumpy density approaches -G sum rho dV / |r - r'| with the
    truncation error shrinking like (r'/r)^5."""
    n = 16
    rho = wl.gaussian_clumps(n, 4, n_clumps=6, background=0.0, remove_mean=False)
    dx = 1.0 / n
    o, q = oracle.multipole_moments(rho, dx, lmax=4)
    x = (np.arange(n) + 0.5) * dx
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    m = rho.transpose(2, 1, 0) * dx ** 3

    def brute(p):
        r = np.sqrt((X - p[0]) ** 2 + (Y - p[1]) ** 2 + (Z - p[2]) ** 2)
        return -np.sum(m / r)

    d = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    errs = []
    for dist in (2.0, 4.0, 8.0):
        p = o + dist * d
        errs.append(abs(oracle.multipole_potential(*p, q, o) - brute(p)) / abs(brute(p)))
    assert errs[0] < 1e-3
    assert errs[1] < errs[0] / 16 and errs[2] < errs[1] / 16, errs


def test_sphere_is_monopole_and_dipole_vanishes():
    n = 32
    rho, c = wl.uniform_sphere(n, 1)
    o, q = oracle.multipole_moments(rho, 1.0 / n, lmax=4)
    mass = rho.sum() / n ** 3
    assert math.isclose(q[0], mass, rel_tol=1e-12)     # Q_00 = sqrt(4 pi) Y_00 M = M
    assert np.max(np.abs(q[1:4])) < 1e-14 * mass          # dipoles about the centre of mass
    assert np.max(np.abs(q[4:])) < 2e-4 * mass * 0.25 ** 2  # sphere: higher moments ~ voxel noise
    assert np.allclose(o, c, atol=1e-3)


def test_multipole_solve_matches_analytic_sphere():
    """Open boundaries from the expansion about the centre of mass: the converged potential
    agrees with the analytic sphere potential to truncation-error level (Sec. 4.2, App. A)."""
    errs = []
    for n in (16, 32):
        rho, c = wl.uniform_sphere(n, 6)
        mass = rho.sum() / n ** 3
        phi, hist, st = oracle.solve(rho, 1.0 / n, [MULTIPOLE] * 6, lmax=4, tol=1e-11, max_cycles=60)
        assert st == oracle.OK
        x = (np.arange(n) + 0.5) / n
        ana = wl.sphere_potential(x[None, None, :], x[None, :, None], x[:, None, None], c, 0.25, mass)
        errs.append(np.sqrt(np.mean((phi - ana) ** 2)) / np.sqrt(np.mean(ana ** 2)))
    assert errs[0] < 5e-3 and errs[1] < errs[0] / 2.5, errs


def test_multipole_faces_match_point_evaluation():
    """Per-level face arrays hold the expansion evaluated at that level's face points,
    extension ring included."""
    n = 8
    rho, c = wl.uniform_sphere(n, 0)
    s = oracle.State(rho, 1.0 / n, [MULTIPOLE] * 6, lmax=4)
    o, q = s.origin_moments()
    for level in (3, 1):
        nl = 1 << level
        hl = 1.0 / nl
        b = s.face(level, 3)                    # +y face, transverse (x, z)
        for t2 in (-1, 0, nl):
            for t1 in (-1, 2 % nl, nl):
                p = ((t1 + 0.5) * hl, 1.0, (t2 + 0.5) * hl)
                assert math.isclose(b[t2 + 1, t1 + 1], oracle.multipole_potential(*p, q, o), rel_tol=1e-14)
