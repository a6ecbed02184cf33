"""Exact discrete solutions phi*_h = L_h^-1 f_h computed without multigrid.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Multigrid converges to the exact solution of the discretised problem (eq. discretized3,
Sec. 2.1); these routines compute that solution by other means so the iteration oracle
and the HIP path can be pinned to it:

* per-axis spectral solves (periodic -> FFT, fixed with ghost = 2b - u -> DST-II,
  zero-gradient with ghost = u -> DCT-II), the discrete eigenvalues of the 7-point
  operator being  lambda = -(4/h^2) sum_d sin^2(theta_d / 2);
* a dense direct solve for grids up to 8^3 and any mix of boundary kinds;
* closed forms for the product-of-sines problem of Sec. 4.1.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft

PERIODIC, ZERO_GRADIENT, FIXED, MULTIPOLE = 0, 1, 2, 3


def _axis_kind(kinds, axis):
    a, b = kinds[2 * axis], kinds[2 * axis + 1]
    if a == MULTIPOLE:
        a = FIXED
    if b == MULTIPOLE:
        b = FIXED
    if a != b:
        raise ValueError("spectral solve needs the same kind on both faces of an axis")
    return a


def boundary_rhs(n, h, kinds, faces):
    """Contribution of fixed face values moved to the right-hand side.

    With ghost = 2b - u the boundary cell's stencil gains 2b/h^2, so
    L_0 u = f - 2b/h^2 on boundary cells, L_0 having ghost = -u.
    ``faces``: six (n, n) arrays [t2][t1] (or None = 0)."""
    r = np.zeros((n, n, n))
    for face in range(6):
        if kinds[face] not in (FIXED, MULTIPOLE) or faces is None or faces[face] is None:
            continue
        b = np.asarray(faces[face], dtype=np.float64)
        axis, side = face // 2, face % 2
        idx = 0 if side == 0 else n - 1
        if axis == 0:
            r[:, :, idx] += 2.0 * b / (h * h)          # b[z][y]
        elif axis == 1:
            r[:, idx, :] += 2.0 * b / (h * h)          # b[z][x]
        else:
            r[idx, :, :] += 2.0 * b / (h * h)          # b[y][x]
    return r


def spectral_solve(f, h, kinds, faces=None):
    """Exact discrete solution with per-axis FFT / DST-II / DCT-II.

    f: (n,n,n) source (already mean-free when no face is fixed).  kinds: 6 face kinds,
    identical on the two faces of each axis.  Returns phi with mean zero when no face
    fixes the zero point."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    kinds = [int(k) for k in kinds]
    ak = [_axis_kind(kinds, a) for a in range(3)]
    rhs = f - boundary_rhs(n, h, kinds, faces)
    # numpy axes: 0 = z, 1 = y, 2 = x
    lam = np.zeros((n, n, n))
    spec = rhs.astype(np.complex128) if PERIODIC in ak else rhs.copy()
    for a in range(3):
        ax = 2 - a
        if ak[a] == PERIODIC:
            spec = sfft.fft(spec, axis=ax, workers=-1)
            theta = 2.0 * math.pi * np.arange(n) / n
        elif ak[a] == FIXED:
            spec = sfft.dst(spec, type=2, axis=ax, workers=-1)
            theta = math.pi * (np.arange(n) + 1) / n
        else:
            spec = sfft.dct(spec, type=2, axis=ax, workers=-1)
            theta = math.pi * np.arange(n) / n
        l1 = -(4.0 / (h * h)) * np.sin(theta / 2.0) ** 2
        shape = [1, 1, 1]
        shape[ax] = n
        lam = lam + l1.reshape(shape)
    zero = lam == 0.0
    lam[zero] = 1.0
    spec = spec / lam
    spec[zero] = 0.0
    for a in range(3):
        ax = 2 - a
        if ak[a] == PERIODIC:
            spec = sfft.ifft(spec, axis=ax, workers=-1)
        elif ak[a] == FIXED:
            spec = sfft.idst(spec, type=2, axis=ax, workers=-1)
        else:
            spec = sfft.idct(spec, type=2, axis=ax, workers=-1)
    return np.real(spec) if np.iscomplexobj(spec) else spec


def dense_matrix(n, h, kinds, faces=None):
    """Dense matrix of the 7-point operator with ghost rules, and the boundary shift.

    Returns (A, g) with L_h u = A u + g for every u (g from fixed face values)."""
    N = n ** 3
    A = np.zeros((N, N))
    g = np.zeros(N)
    ih2 = 1.0 / (h * h)

    def lin(i, j, k):
        return (k * n + j) * n + i

    for k in range(n):
        for j in range(n):
            for i in range(n):
                c = lin(i, j, k)
                A[c, c] -= 6.0 * ih2
                for axis in range(3):
                    for side in (0, 1):
                        p = [i, j, k]
                        p[axis] += -1 if side == 0 else 1
                        if 0 <= p[axis] < n:
                            A[c, lin(*p)] += ih2
                            continue
                        face = 2 * axis + side
                        kind = kinds[face]
                        if kind == PERIODIC:
                            p[axis] %= n
                            A[c, lin(*p)] += ih2
                        elif kind == ZERO_GRADIENT:
                            A[c, c] += ih2
                        else:
                            A[c, c] -= ih2
                            if faces is not None and faces[face] is not None:
                                t = [q for q in range(3) if q != axis]
                                b = faces[face][[i, j, k][t[1]], [i, j, k][t[0]]]
                                g[c] += 2.0 * b * ih2
    return A, g


def dense_solve(f, h, kinds, faces=None):
    """Direct solve of L_h u = f on a small grid (bordered by sum u = 0 when singular)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    kinds = [int(k) for k in kinds]
    A, g = dense_matrix(n, h, kinds, faces)
    rhs = f.ravel() - g
    gauge_free = all(k in (PERIODIC, ZERO_GRADIENT) for k in kinds)
    if gauge_free:
        N = n ** 3
        B = np.zeros((N + 1, N + 1))
        B[:N, :N] = A
        B[:N, N] = 1.0
        B[N, :N] = 1.0
        sol = np.linalg.solve(B, np.concatenate([rhs, [0.0]]))
        return sol[:N].reshape(n, n, n)
    return np.linalg.solve(A, rhs).reshape(n, n, n)


def sine_modes_exact(n, modes, four_pi_g=4.0 * math.pi, length=1.0):
    """Exact discrete solution for rho = sum_m A_m prod_d sin(2 pi k_d x_d): every
    product-of-sines mode is an eigenvector of the periodic 7-point operator."""
    h = length / n
    x = (np.arange(n) + 0.5) * h
    phi = np.zeros((n, n, n))
    for (kx, ky, kz), a in modes:
        lam = -(4.0 / (h * h)) * sum(math.sin(math.pi * kk / n) ** 2 for kk in (kx, ky, kz))
        sx = np.sin(2 * math.pi * kx * x / length)
        sy = np.sin(2 * math.pi * ky * x / length)
        sz = np.sin(2 * math.pi * kz * x / length)
        phi += four_pi_g * a / lam * sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    return phi


def sine_modes_continuum(n, modes, four_pi_g=4.0 * math.pi, length=1.0):
    """Continuum solution of the same problem (Sec. 4.1 analytic form)."""
    h = length / n
    x = (np.arange(n) + 0.5) * h
    phi = np.zeros((n, n, n))
    for (kx, ky, kz), a in modes:
        kk2 = (2 * math.pi / length) ** 2 * (kx * kx + ky * ky + kz * kz)
        sx = np.sin(2 * math.pi * kx * x / length)
        sy = np.sin(2 * math.pi * ky * x / length)
        sz = np.sin(2 * math.pi * kz * x / length)
        phi += -four_pi_g * a / kk2 * sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    return phi


def rel_residual(phi, f, h, kinds, faces=None):
    """RMS(f - L phi) / RMS(f) computed with the explicit matrix-free ghost rules."""
    n = phi.shape[0]
    kinds = [int(k) for k in kinds]
    pad = np.zeros((n + 2,) * 3)
    pad[1:-1, 1:-1, 1:-1] = phi
    # fill per axis x, y, z (numpy axes 2, 1, 0), each covering earlier ghosts
    for axis in range(3):
        ax = 2 - axis
        for side in (0, 1):
            face = 2 * axis + side
            g = 0 if side == 0 else n + 1
            a = 1 if side == 0 else n
            o = n if side == 0 else 1
            sl_g = [slice(None)] * 3
            sl_a = [slice(None)] * 3
            sl_o = [slice(None)] * 3
            sl_g[ax], sl_a[ax], sl_o[ax] = g, a, o
            kind = kinds[face]
            if kind == PERIODIC:
                pad[tuple(sl_g)] = pad[tuple(sl_o)]
            elif kind == ZERO_GRADIENT:
                pad[tuple(sl_g)] = pad[tuple(sl_a)]
            else:
                bb = 0.0
                if faces is not None and faces[face] is not None:
                    bb = np.pad(np.asarray(faces[face]), 1, mode="edge")
                pad[tuple(sl_g)] = 2.0 * bb - pad[tuple(sl_a)]
    lap = (pad[1:-1, 1:-1, :-2] + pad[1:-1, 1:-1, 2:] + pad[1:-1, :-2, 1:-1] + pad[1:-1, 2:, 1:-1] +
           pad[:-2, 1:-1, 1:-1] + pad[2:, 1:-1, 1:-1] - 6.0 * phi) / (h * h)
    d = f - lap
    rf = math.sqrt(np.mean(f * f))
    rd = math.sqrt(np.mean(d * d))
    return rd / rf if rf > 0 else rd
