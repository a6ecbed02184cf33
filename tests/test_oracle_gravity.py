"""Pins of the oracle's gravitational acceleration (eq. acceleration, cell-centred source-term
scheme of Sec. 2.4) against facts that do not come from that function: closed forms of the
differences of sine modes and polynomials, the discrete divergence theorem (div of the face
field = -L_h phi, with L_h from the independently pinned defect operator), zero curl, the
boundary rules' surface values, and the analytic field of a uniform sphere.  CPU only."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import FIXED, MULTIPOLE, PERIODIC, ZERO_GRADIENT

KIND_SETS = [
    [PERIODIC] * 6,
    [FIXED] * 6,
    [ZERO_GRADIENT] * 6,
    [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, ZERO_GRADIENT],
    [FIXED, ZERO_GRADIENT, PERIODIC, PERIODIC, ZERO_GRADIENT, FIXED],
]


def centres(n):
    return (np.arange(n) + 0.5) / n


def random_faces(n, seed):
    rng = np.random.default_rng(seed)
    return [oracle.extend_face(rng.uniform(-1, 1, (n, n))) for _ in range(6)]


def test_sine_mode_closed_form():
    """phi = sin(2 pi m x + a) on a periodic grid: the face difference is
    -2 sin(pi m h) cos(2 pi m x_face + a) / h and the cell mean is
    -sin(2 pi m h) cos(2 pi m x_cell + a) / h, exactly (trigonometric identities)."""
    n = 16
    h = 1.0 / n
    x = centres(n)
    m, a = 3, 0.4
    px = np.sin(2 * math.pi * m * x + a)
    for axis in range(3):
        shape = [1, 1, 1]
        shape[2 - axis] = n
        phi = np.broadcast_to(px.reshape(shape), (n, n, n)).copy()
        g, (fx, fy, fz) = oracle.gravity(phi, h, PERIODIC, faces=True)
        want_c = -math.sin(2 * math.pi * m * h) * np.cos(2 * math.pi * m * x + a) / h
        xf = np.arange(n + 1) / n
        want_f = -2 * math.sin(math.pi * m * h) * np.cos(2 * math.pi * m * xf + a) / h
        got_c = np.moveaxis(g[axis], 2 - axis, 2)
        assert np.max(np.abs(got_c - want_c[None, None, :])) < 1e-12 * n
        face = (fx, fy, fz)[axis]
        got_f = np.moveaxis(face, 2 - axis, 2)
        assert got_f.shape[2] == n + 1
        assert np.max(np.abs(got_f - want_f[None, None, :])) < 1e-12 * n
        for b in range(3):
            if b != axis:
                assert np.max(np.abs(g[b])) == 0.0


def test_quadratic_interior_exact():
    """The mean of two one-sided differences is the central difference, exact for quadratics:
    phi = x^2 + 3 y z gives g = (-2x, -3z, -3y) in every cell away from the surface."""
    n = 12
    h = 1.0 / n
    x = centres(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    phi = X * X + 3 * Y * Z
    g = oracle.gravity(phi, h, FIXED)
    s = (slice(1, -1),) * 3
    assert np.max(np.abs(g[0][s] + 2 * X[s])) < 1e-12
    assert np.max(np.abs(g[1][s] + 3 * Z[s])) < 1e-12
    assert np.max(np.abs(g[2][s] + 3 * Y[s])) < 1e-12


def test_linear_field_with_its_face_values():
    """A linear potential with fixed faces holding its surface values: the ghost 2b - phi is
    the linear extrapolation, so g = -grad phi exactly in every cell and on every face,
    the boundary faces included (Sec. 2.3.6: the surface value equals b)."""
    n = 8
    h = 1.0 / n
    x = centres(n)
    a = (0.7, -1.3, 2.1)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    phi = 0.4 + a[0] * X + a[1] * Y + a[2] * Z
    faces = []
    for face in range(6):
        axis, side = face // 2, face % 2
        coords = [None, None, None]
        coords[axis] = 0.0 if side == 0 else 1.0
        t = [q for q in range(3) if q != axis]
        coords[t[0]] = x[None, :]
        coords[t[1]] = x[:, None]
        faces.append(oracle.extend_face(np.broadcast_to(0.4 + sum(a[q] * coords[q] for q in range(3)), (n, n))))
    g, (fx, fy, fz) = oracle.gravity(phi, h, FIXED, faces, faces=True)
    for axis in range(3):
        assert np.max(np.abs(g[axis] + a[axis])) < 1e-12
        assert np.max(np.abs((fx, fy, fz)[axis] + a[axis])) < 1e-12


@pytest.mark.parametrize("kinds", KIND_SETS)
def test_divergence_of_faces_is_minus_laplacian(kinds):
    """Discrete divergence theorem: sum over axes of (g_high - g_low)/h = -L_h phi in every
    cell, with L_h phi taken from the defect operator (d = 0 - L_h phi), whose stencil and
    ghost rules are pinned on their own.  Catches a sign, a swapped face or a wrong ghost."""
    n = 16
    h = 1.0 / n
    rng = np.random.default_rng(11)
    phi = rng.uniform(-1, 1, (n, n, n))
    bext = random_faces(n, 12)
    g, (fx, fy, fz) = oracle.gravity(phi, h, kinds, bext, faces=True)
    div = (fx[:, :, 1:] - fx[:, :, :-1] + fy[:, 1:, :] - fy[:, :-1, :] + fz[1:] - fz[:-1]) / h
    d = oracle.defect(phi, np.zeros_like(phi), h, kinds, bext)
    assert np.max(np.abs(div - d)) < 1e-10 * np.max(np.abs(d))
    # cell values are the mean of their two faces
    assert np.array_equal(g[0], 0.5 * (fx[:, :, :-1] + fx[:, :, 1:]))
    assert np.array_equal(g[1], 0.5 * (fy[:, :-1, :] + fy[:, 1:, :]))
    assert np.array_equal(g[2], 0.5 * (fz[:-1] + fz[1:]))


def test_face_field_is_curl_free():
    """Face differences of one potential: the circulation around every interior cell edge
    vanishes, (gx(j+1) - gx(j)) - (gy(i+1) - gy(i)) = 0 (same for the other pairs).  Catches
    axis mix-ups that the divergence alone does not see."""
    n = 10
    h = 0.1
    phi = np.random.default_rng(3).normal(size=(n, n, n))
    _, (fx, fy, fz) = oracle.gravity(phi, h, PERIODIC, faces=True)
    cxy = (fx[:, 1:, 1:n] - fx[:, :-1, 1:n]) - (fy[:, 1:n, 1:] - fy[:, 1:n, :-1])
    cxz = (fx[1:, :, 1:n] - fx[:-1, :, 1:n]) - (fz[1:n, :, 1:] - fz[1:n, :, :-1])
    cyz = (fy[1:, 1:n, :] - fy[:-1, 1:n, :]) - (fz[1:n, 1:, :] - fz[1:n, :-1, :])
    for c in (cxy, cxz, cyz):
        assert np.max(np.abs(c)) < 1e-12 / h


def test_boundary_faces():
    """Zero-gradient faces carry no acceleration; periodic ones repeat the opposite face; a
    fixed face gives -(phi_0 - b)/(h/2) (the surface value b reached over half a cell)."""
    n = 8
    h = 1.0 / n
    rng = np.random.default_rng(5)
    phi = rng.normal(size=(n, n, n))
    _, (fx, fy, fz) = oracle.gravity(phi, h, ZERO_GRADIENT, faces=True)
    for f in (fx[:, :, 0], fx[:, :, n], fy[:, 0, :], fy[:, n, :], fz[0], fz[n]):
        assert np.max(np.abs(f)) == 0.0
    _, (fx, fy, fz) = oracle.gravity(phi, h, PERIODIC, faces=True)
    assert np.array_equal(fx[:, :, 0], fx[:, :, n])
    assert np.array_equal(fy[:, 0, :], fy[:, n, :])
    assert np.array_equal(fz[0], fz[n])
    b = rng.normal(size=(n, n))
    bext = [oracle.extend_face(b)] * 6
    _, (fx, fy, fz) = oracle.gravity(phi, h, FIXED, bext, faces=True)
    assert np.allclose(fx[:, :, 0], -(phi[:, :, 0] - b) / (h / 2), rtol=1e-13, atol=1e-12)
    assert np.allclose(fx[:, :, n], -(b - phi[:, :, n - 1]) / (h / 2), rtol=1e-13, atol=1e-12)
    assert np.allclose(fy[:, 0, :], -(phi[:, 0, :] - b) / (h / 2), rtol=1e-13, atol=1e-12)
    assert np.allclose(fz[n], -(b - phi[n - 1]) / (h / 2), rtol=1e-13, atol=1e-12)


def test_momentum_source_is_rho_g():
    n = 8
    rng = np.random.default_rng(9)
    phi, rho = rng.normal(size=(n, n, n)), rng.uniform(0, 2, (n, n, n))
    g, rg = oracle.gravity(phi, 1.0 / n, PERIODIC, rho=rho)
    assert np.array_equal(rg, rho[None] * g)


def test_uniform_sphere_field():
    """Self-gravity of a uniform sphere with multipole faces (Appendix A): outside the sphere
    g = -G M r / |r|^3, inside g = -(4 pi / 3) G rho r (Sec. 4.2's analytic solution), to the
    discretisation error of the surface-averaged density on a 64^3 grid."""
    n = 64
    h = 1.0 / n
    radius = 0.25
    rho, c = wl.uniform_sphere(n, 4, radius=radius)
    mass = float(rho.sum()) * h ** 3
    phi, hist, st = oracle.solve(rho, h, MULTIPOLE, tol=1e-10)
    assert st in (0, 2)
    s = oracle.State(rho, h, MULTIPOLE)
    bext = [s.face(s.levels(), f) for f in range(6)]
    g = oracle.gravity(phi, h, [FIXED] * 6, bext)
    x = centres(n)
    Z, Y, X = np.meshgrid(x - c[2], x - c[1], x - c[0], indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    rr = np.maximum(r, 1e-12) ** 3
    scale = np.where(r >= radius, -mass / rr, -(4 * math.pi / 3) * 1.0)
    want = [scale * X, scale * Y, scale * Z]
    gmax = mass / radius ** 2
    for sel in (r > radius + 4 * h, r < radius - 4 * h):
        err = max(np.max(np.abs(g[a][sel] - want[a][sel])) for a in range(3))
        assert err < 0.03 * gmax, err
