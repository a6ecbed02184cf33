"""Pins of the oracle's single operators against facts that do not come from the oracle:
discrete eigenvectors, exactness on polynomials, the paper's printed weights, and
algebraic properties of the RB-SOR update.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from oracle import FIXED, MULTIPOLE, PERIODIC, ZERO_GRADIENT
from oracle import exact as ex

KIND_SETS = [
    [PERIODIC] * 6,
    [FIXED] * 6,
    [ZERO_GRADIENT] * 6,
    [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, ZERO_GRADIENT],
    [FIXED, ZERO_GRADIENT, PERIODIC, PERIODIC, ZERO_GRADIENT, FIXED],
]


def centres(n):
    return (np.arange(n) + 0.5) / n


def axis_mode(kind, k, x):
    """Discrete eigenvector along one axis for the given (paired) boundary kind."""
    if kind == PERIODIC:
        return np.sin(2 * math.pi * k * x + 0.3), 2 * math.pi * k / len(x)
    if kind == FIXED:
        return np.sin(math.pi * k * x), math.pi * k / len(x)
    return np.cos(math.pi * k * x), math.pi * k / len(x)


@pytest.mark.parametrize("kinds", [[PERIODIC] * 6, [FIXED] * 6, [ZERO_GRADIENT] * 6,
                                   [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, ZERO_GRADIENT]])
def test_laplacian_eigenvectors(kinds):
    """Textbook eigenpairs of the 7-point operator (eq. discretized2) under each ghost rule:
    L u = -(4/h^2) sum_d sin^2(theta_d/2) u.  Pins the stencil and the ghost rules."""
    n = 16
    h = 1.0 / n
    x = centres(n)
    ks = (3, 2, 5)
    mx, tx = axis_mode(kinds[0], ks[0], x)
    my, ty = axis_mode(kinds[2], ks[1], x)
    mz, tz = axis_mode(kinds[4], ks[2], x)
    u = mz[:, None, None] * my[None, :, None] * mx[None, None, :]
    lam = -(4 / h ** 2) * (math.sin(tx / 2) ** 2 + math.sin(ty / 2) ** 2 + math.sin(tz / 2) ** 2)
    d = oracle.defect(u, np.zeros_like(u), h, kinds)       # d = -L u
    assert np.max(np.abs(-d - lam * u)) <= 1e-11 * abs(lam)


def test_fixed_faces_exact_on_linear_fields():
    """With ghost = 2b - u and b the face value of a linear field, the ghost equals the
    field's linear extrapolation, so L u = 0 exactly (Sec. 2.3.6: surface value = b)."""
    n = 8
    h = 1.0 / n
    x = centres(n)
    a = (0.7, -1.3, 2.1)
    u = 0.4 + a[0] * x[None, None, :] + a[1] * x[None, :, None] + a[2] * x[:, None, None]
    u = np.broadcast_to(u, (n, n, n)).copy()
    faces = []
    for face in range(6):
        axis, side = face // 2, face % 2
        pos = 0.0 if side == 0 else 1.0
        t = [q for q in range(3) if q != axis]
        coords = [None, None, None]
        coords[axis] = pos
        coords[t[0]] = x[None, :]
        coords[t[1]] = x[:, None]
        faces.append(np.broadcast_to(0.4 + sum(a[q] * coords[q] for q in range(3)), (n, n)).copy())
    bext = [oracle.extend_face(b) for b in faces]
    d = oracle.defect(u, np.zeros_like(u), h, [FIXED] * 6, bext)
    assert np.max(np.abs(d)) < 1e-10


def test_restriction_weights(golden):
    """eq. restriction: each child weighs 1/8; constants and the total are preserved."""
    w = golden["restriction_weight"]["value"]
    rng = np.random.default_rng(1)
    uf = rng.standard_normal((8, 8, 8))
    uc = oracle.restrict(uf)
    assert np.isclose(uc.sum() * 8, uf.sum(), rtol=1e-13)
    assert np.allclose(oracle.restrict(np.full((4, 4, 4), 3.25)), 3.25, rtol=0, atol=1e-15)
    delta = np.zeros((4, 4, 4))
    delta[3, 2, 1] = 1.0                      # child (1,2,3) -> parent (0,1,1)
    uc = oracle.restrict(delta)
    assert uc[1, 1, 0] == w and np.count_nonzero(uc) == 1


@pytest.mark.parametrize("cubic", [0, 1])
def test_prolongation_weights_match_paper(cubic, golden):
    """A coarse delta prolongs to the tensor product of the printed 1-D weights."""
    nc = 4
    uc = np.zeros((nc,) * 3)
    uc[2, 1, 2] = 1.0
    kinds = [PERIODIC] * 6
    if cubic:
        uf = oracle.prolong_fmg(uc, kinds)
        lo, up = golden["tricubic_lower"]["value"], golden["tricubic_upper"]["value"]
    else:
        uf = oracle.prolong_add(uc, np.zeros((2 * nc,) * 3), kinds)
        lo, up = golden["trilinear_lower"]["value"], golden["trilinear_upper"]["value"]

    def w1(i, I):
        # weight of coarse cell I for fine cell i
        off = I - (i >> 1)
        if off not in (-1, 0, 1):
            return 0.0
        return (up if i & 1 else lo)[off + 1]

    expect = np.zeros((2 * nc,) * 3)
    for k in range(2 * nc):
        for j in range(2 * nc):
            for i in range(2 * nc):
                expect[k, j, i] = w1(i, 2) * w1(j, 1) * w1(k, 2)
    assert np.allclose(uf, expect, rtol=0, atol=1e-16)


def _linear_with_faces(nc, a, c0):
    """Linear field on an nc grid plus exact extended face values (ring included)."""
    x = centres(nc)
    u = c0 + a[0] * x[None, None, :] + a[1] * x[None, :, None] + a[2] * x[:, None, None]
    u = np.broadcast_to(u, (nc,) * 3).copy()
    xe = (np.arange(-1, nc + 1) + 0.5) / nc
    bext = []
    for face in range(6):
        axis, side = face // 2, face % 2
        t = [q for q in range(3) if q != axis]
        coords = [None, None, None]
        coords[axis] = 0.0 if side == 0 else 1.0
        coords[t[0]] = xe[None, :]
        coords[t[1]] = xe[:, None]
        bext.append(np.broadcast_to(c0 + sum(a[q] * coords[q] for q in range(3)), (nc + 2, nc + 2)).copy())
    return u, bext


@pytest.mark.parametrize("cubic", [0, 1])
def test_prolongation_exact_on_linear_fields(cubic):
    """Both prolongations reproduce a linear field exactly, ghosts and edges included
    (the fixed ghost rule extrapolates linear fields exactly)."""
    nc = 4
    a, c0 = (0.9, -0.4, 1.7), 0.25
    uc, bext = _linear_with_faces(nc, a, c0)
    uf_exact, _ = _linear_with_faces(2 * nc, a, c0)
    if cubic:
        uf = oracle.prolong_fmg(uc, [FIXED] * 6, bext)
    else:
        uf = oracle.prolong_add(uc, np.zeros((2 * nc,) * 3), [FIXED] * 6, bext)
    assert np.max(np.abs(uf - uf_exact)) < 1e-13


def test_tricubic_exact_on_quadratics():
    """The FMG weights are 3-point Lagrange interpolation at -+1/4 of a coarse cell, so
    quadratics are reproduced exactly wherever the stencil stays inside the grid."""
    nc = 8
    xc = centres(nc)
    xf = centres(2 * nc)

    def q(x, y, z):
        return 0.3 + x * x - 2 * y * z + 0.5 * z * z + x * y - y

    uc = q(xc[None, None, :], xc[None, :, None], xc[:, None, None])
    uf = oracle.prolong_fmg(uc, [PERIODIC] * 6)
    ref = q(xf[None, None, :], xf[None, :, None], xf[:, None, None])
    s = slice(2, 2 * nc - 2)
    assert np.max(np.abs(uf[s, s, s] - ref[s, s, s])) < 1e-13
    # weights sum to one: a constant is reproduced everywhere under periodic ghosts
    assert np.allclose(oracle.prolong_fmg(np.full((nc,) * 3, 2.5), [PERIODIC] * 6), 2.5, atol=1e-14)


@pytest.mark.parametrize("kinds", KIND_SETS)
@pytest.mark.parametrize("omega", [1.0, 1.15])
def test_half_sweep_defect_contraction(kinds, omega):
    """After one colour of the RB-SOR update the defect on the updated cells is (1-omega)
    times its previous value, and the other colour is untouched (eqs. rbsor1-2).
    Boundary cells of non-periodic faces are excluded here (their ghost moves with them);
    the fixed-point test below covers them."""
    n = 8
    h = 1.0 / n
    rng = np.random.default_rng(7)
    u = rng.standard_normal((n,) * 3)
    f = rng.standard_normal((n,) * 3)
    bext = [oracle.extend_face(rng.standard_normal((n, n))) for _ in range(6)]
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    interior = np.ones((n,) * 3, dtype=bool)
    for face, kind in enumerate(kinds):
        if kind == PERIODIC:
            continue
        axis, side = face // 2, face % 2
        idx = (i, j, k)[axis]
        interior &= idx != (0 if side == 0 else n - 1)
    for colour in (0, 1):
        mask = ((i + j + k) % 2) == colour
        d0 = oracle.defect(u, f, h, kinds, bext)
        u1 = oracle.half_sweep(u, f, h, omega, colour, kinds, bext)
        d1 = oracle.defect(u1, f, h, kinds, bext)
        assert np.array_equal(u1[~mask], u[~mask])
        sel = mask & interior
        assert np.max(np.abs(d1[sel] - (1 - omega) * d0[sel])) <= 1e-10 * np.max(np.abs(d0))
        u = u1


@pytest.mark.parametrize("kinds", KIND_SETS)
def test_sweep_fixed_point_is_discrete_solution(kinds):
    """The exact discrete solution (dense direct solve) is a fixed point of a full
    smoothing sweep for every boundary kind, boundary cells included."""
    n = 4
    h = 1.0 / n
    rng = np.random.default_rng(11)
    f = rng.standard_normal((n,) * 3)
    faces = [rng.standard_normal((n, n)) for _ in range(6)]
    if all(kd in (PERIODIC, ZERO_GRADIENT) for kd in kinds):
        f -= f.mean()
    u = ex.dense_solve(f, h, kinds, faces)
    bext = [oracle.extend_face(b) for b in faces]
    u2 = oracle.smooth(u, f, h, 1.15, kinds, bext)
    assert np.max(np.abs(u2 - u)) <= 1e-12 * np.max(np.abs(u))


def test_fill_edges_follow_axis_order():
    """Edges/corners: x ghosts first, then y over the x ghosts, then z (Sec. 2.3.6 applied
    axis by axis); checked by hand for zero-fixed on all faces."""
    n = 2
    u = np.arange(1.0, 9.0).reshape(2, 2, 2)
    g = oracle.fill(u, [FIXED] * 6)
    # x-ghost of (0,0,0) is -u000; the edge (-1,-1,0) is -(x-ghost of (-1,0,0)) = u000
    assert g[1, 1, 0] == -u[0, 0, 0]
    assert g[1, 0, 0] == u[0, 0, 0]
    assert g[0, 0, 0] == -u[0, 0, 0]
    gp = oracle.fill(u, [PERIODIC] * 6)
    assert gp[0, 0, 0] == u[1, 1, 1] and gp[3, 3, 3] == u[0, 0, 0]
    gz = oracle.fill(u, [ZERO_GRADIENT] * 6)
    assert gz[0, 0, 0] == u[0, 0, 0] and gz[3, 0, 3] == u[1, 0, 1]


def test_coarsest_closed_forms():
    """Single-cell solve (Sec. 2.3.2): fixed faces give u = (2 sum b - h^2 f) / (6 + #fixed)
    ... / (6 - sum alpha); the result has zero defect with its own ghosts."""
    h = 0.5
    f = 1.7
    b = [0.3, -0.2, 0.5, 0.1, -0.4, 0.25]
    bext = [np.full((3, 3), v) for v in b]
    u = oracle.coarsest(h, f, [FIXED] * 6, bext)
    assert math.isclose(u, (2 * sum(b) - h * h * f) / 12.0, rel_tol=1e-15)
    kinds = [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, FIXED]
    u = oracle.coarsest(h, f, kinds, bext)
    sb = 2 * (b[2] + b[3] + b[5])
    assert math.isclose(u, (sb - h * h * f) / (6.0 - (1 + 1 - 1 - 1 + 1 - 1)), rel_tol=1e-15)
    d = oracle.defect(np.full((1, 1, 1), u), np.full((1, 1, 1), f), h, kinds, bext)
    assert abs(d[0, 0, 0]) < 1e-13
    assert oracle.coarsest(h, 0.0, [PERIODIC] * 6) == 0.0
