"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only *generates inputs*: densities, boundary values and request traces.
It holds none of the multigrid arithmetic, and neither the HIP path nor the oracle
is imported here.  Every generator is deterministic in its seed
(``numpy.random.default_rng``) and returns C-ordered float64 arrays indexed
``[z][y][x]`` (x fastest), on the unit cube by default, with cell ``(i, j, k)``
centred at ``((i + 1/2) h, (j + 1/2) h, (k + 1/2) h)``.

Recipes (the paper's test problems, Sec. 4.1 and Sec. 4.2, at the sizes the
benchmark uses):

* ``sine_modes``      -- sum of product-of-sines modes in a periodic box (Sec. 4.1).
* ``gaussian_clumps`` -- background plus Gaussian clumps with lognormal amplitudes.
* ``uniform_sphere``  -- uniform sphere sampled by volume fraction with 10^3 sub-cells
                         on cells cut by the surface (the sampling of Sec. 4.2).
* ``lognormal_grf``   -- exp of a Gaussian random field with P(k) ~ k^-4.
* ``sphere_potential``-- closed-form potential of a uniform sphere (Sec. 4.2), used to
                         make fixed boundary values and as an analytic reference.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "cell_centres",
    "random_field",
    "sine_modes",
    "gaussian_clumps",
    "uniform_sphere",
    "sphere_potential",
    "sphere_face_values",
    "lognormal_grf",
    "serving_trace",
]


def cell_centres(n: int, length: float = 1.0) -> np.ndarray:
    """1-D cell-centre coordinates of an n-cell axis of the given length."""
    h = length / n
    return (np.arange(n, dtype=np.float64) + 0.5) * h


def random_field(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Uniform random float64 array (used for operator-level checks)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape).astype(np.float64)


def sine_modes(n: int, seed: int, n_modes: int = 8, kmax: int = 4, length: float = 1.0):
    """Sum of ``n_modes`` product-of-sines modes with distinct integer wave vectors.

    rho = sum_m A_m sin(2 pi kx x / L) sin(2 pi ky y / L) sin(2 pi kz z / L),
    k drawn without replacement from {1..kmax}^3, A_m ~ N(0, 1).  This is the
    periodic sinusoidal problem of Sec. 4.1 with several modes; its mean is zero
    to round-off and is removed exactly.

    Returns ``(rho, modes)`` where ``modes`` is a list of ``((kx, ky, kz), A)``.
    """
    rng = np.random.default_rng(seed)
    all_k = [(a, b, c) for c in range(1, kmax + 1) for b in range(1, kmax + 1) for a in range(1, kmax + 1)]
    pick = rng.choice(len(all_k), size=n_modes, replace=False)
    amps = rng.standard_normal(n_modes)
    x = cell_centres(n, length)
    rho = np.zeros((n, n, n), dtype=np.float64)
    modes = []
    for idx, a in zip(pick, amps):
        kx, ky, kz = all_k[int(idx)]
        sx = np.sin(2.0 * math.pi * kx * x / length)
        sy = np.sin(2.0 * math.pi * ky * x / length)
        sz = np.sin(2.0 * math.pi * kz * x / length)
        rho += float(a) * sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
        modes.append(((kx, ky, kz), float(a)))
    rho -= rho.mean()
    return rho, modes


def _periodic_gauss_1d(x: np.ndarray, c: float, w: float, length: float) -> np.ndarray:
    d = np.abs(x - c)
    d = np.minimum(d, length - d)          # minimum-image distance
    return np.exp(-0.5 * (d / w) ** 2)


def gaussian_clumps(n: int, seed: int, n_clumps: int = 64, background: float = 1.0,
                    wmin: float = 0.01, wmax: float = 0.05, sigma_ln: float = 1.0,
                    remove_mean: bool = True, length: float = 1.0) -> np.ndarray:
    """rho = background + sum_c A_c prod_d exp(-D_d^2 / (2 w_c^2)).

    Centres uniform in the box, widths w_c ~ U[wmin, wmax] (Gaussian sigma),
    amplitudes A_c ~ LogNormal(0, sigma_ln), D_d the periodic minimum-image
    distance along axis d.  The field is a sum of rank-one tensors, evaluated as
    one matrix product: (z profiles scaled by A_c) x (y profile (x) x profile).
    The mean is removed when ``remove_mean`` (periodic problems).
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, length, size=(n_clumps, 3))
    widths = rng.uniform(wmin, wmax, size=n_clumps)
    amps = rng.lognormal(0.0, sigma_ln, size=n_clumps)
    x = cell_centres(n, length)
    gx = np.stack([_periodic_gauss_1d(x, float(centres[c, 0]), float(widths[c]), length) for c in range(n_clumps)])
    gy = np.stack([_periodic_gauss_1d(x, float(centres[c, 1]), float(widths[c]), length) for c in range(n_clumps)])
    gz = np.stack([_periodic_gauss_1d(x, float(centres[c, 2]), float(widths[c]), length) for c in range(n_clumps)])
    zc = (gz * amps[:, None]).T                                   # (n, C)
    yx = (gy[:, :, None] * gx[:, None, :]).reshape(n_clumps, n * n)  # (C, n*n)
    rho = zc @ yx
    rho += background
    rho = rho.reshape(n, n, n)
    if remove_mean:
        rho -= rho.mean()
    return rho


# The unequal-mass binary of the refined-mesh test (Sec. 4.3): two uniform spheres of radius
# 6/1024, masses 2 and 1, on the x axis at +6/1024 and -12/1024 from the centre of the box
# (the paper's [-0.5, 0.5]^3 shifted to the unit cube).
BINARY_R = 6.0 / 1024.0
BINARY_STARS = ((2.0, (0.5 + 6.0 / 1024.0, 0.5, 0.5)), (1.0, (0.5 - 12.0 / 1024.0, 0.5, 0.5)))


def binary_density_on_axes(xs, ys, zs, h: float, subcells: int = 10) -> np.ndarray:
    """Density of the binary on the tensor grid of cell-centre axes (cells of width h): each
    star a uniform sphere of density M / (4/3 pi R^3); cells the surface cuts take the mean
    over subcells^3 sub-cell centres (the paper's smoothing).  Indexed [z][y][x]."""
    xs, ys, zs = (np.asarray(a, dtype=np.float64) for a in (xs, ys, zs))
    rho = np.zeros((len(zs), len(ys), len(xs)))
    half_diag = 0.5 * math.sqrt(3.0) * h
    s = (np.arange(subcells) + 0.5) / subcells - 0.5
    oz, oy, ox = (a.ravel() * h for a in np.meshgrid(s, s, s, indexing="ij"))
    for M, c in BINARY_STARS:
        dens = M / (4.0 / 3.0 * math.pi * BINARY_R ** 3)
        dz = (zs - c[2])[:, None, None]
        dy = (ys - c[1])[None, :, None]
        dx = (xs - c[0])[None, None, :]
        r = np.sqrt(dx * dx + dy * dy + dz * dz)
        rho += np.where(r <= BINARY_R - half_diag, dens, 0.0)
        cut = np.argwhere(np.abs(r - BINARY_R) < half_diag)
        for s0 in range(0, cut.shape[0], 4096):
            cc = cut[s0:s0 + 4096]
            pz = zs[cc[:, 0]][:, None] + oz[None, :] - c[2]
            py = ys[cc[:, 1]][:, None] + oy[None, :] - c[1]
            px = xs[cc[:, 2]][:, None] + ox[None, :] - c[0]
            frac = ((px * px + py * py + pz * pz) < BINARY_R * BINARY_R).mean(axis=1)
            rho[cc[:, 0], cc[:, 1], cc[:, 2]] += dens * frac
    return rho


def binary_potential(x, y, z, G: float = 1.0):
    """The binary's analytic potential: the sum of the two uniform-sphere potentials."""
    out = 0.0
    for M, c in BINARY_STARS:
        out = out + sphere_potential(x, y, z, c, BINARY_R, M, G)
    return out


def binary_mesh_boxes(NB: int, levels: int = 4):
    """Nested refinement boxes of the binary test: level l covers [-0.5^(l+1), 0.5^(l+1)] around
    the centre at 2^l times the root resolution, in level-(l-1) block units (NB root blocks
    per side, NB >= 4 a power of two)."""
    boxes = []
    for l in range(1, levels + 1):
        nblk = NB << (l - 1)          # level-(l-1) blocks per side of the whole domain
        lo = nblk // 2 - NB // 4      # half-width 0.5^(l+1) is NB/4 level-(l-1) blocks
        boxes.append(((lo,) * 3, (nblk - lo,) * 3))
    return boxes


def uniform_sphere(n: int, seed: int, radius: float = 0.25, max_offset: float = 0.05,
                   density: float = 1.0, subcells: int = 10, length: float = 1.0):
    """Uniform sphere of the given radius centred at (L/2 + delta) with |delta| <= max_offset.

    Cells entirely inside get ``density``, entirely outside 0; cells the surface cuts
    get ``density`` times the fraction of their ``subcells^3`` sub-cell centres that
    lie inside (the sub-cell averaging of Sec. 4.2).

    Returns ``(rho, centre)``.
    """
    rng = np.random.default_rng(seed)
    while True:
        delta = rng.uniform(-max_offset, max_offset, size=3)
        if float(np.dot(delta, delta)) <= max_offset * max_offset:
            break
    centre = np.full(3, 0.5 * length) + delta
    h = length / n
    x = cell_centres(n, length)
    dz = (x - centre[2])[:, None, None]
    dy = (x - centre[1])[None, :, None]
    dx = (x - centre[0])[None, None, :]
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    half_diag = 0.5 * math.sqrt(3.0) * h
    rho = np.where(r <= radius - half_diag, density, 0.0).astype(np.float64)
    cut = np.argwhere(np.abs(r - radius) < half_diag)
    if cut.size:
        s = (np.arange(subcells, dtype=np.float64) + 0.5) / subcells - 0.5   # sub-cell offsets in units of h
        oz, oy, ox = np.meshgrid(s, s, s, indexing="ij")
        oz = oz.ravel()[None, :] * h
        oy = oy.ravel()[None, :] * h
        ox = ox.ravel()[None, :] * h
        chunk = 8192
        for s0 in range(0, cut.shape[0], chunk):
            cc = cut[s0:s0 + chunk]
            pz = x[cc[:, 0]][:, None] + oz - centre[2]
            py = x[cc[:, 1]][:, None] + oy - centre[1]
            px = x[cc[:, 2]][:, None] + ox - centre[0]
            inside = (px * px + py * py + pz * pz) < radius * radius
            frac = inside.mean(axis=1)
            rho[cc[:, 0], cc[:, 1], cc[:, 2]] = density * frac
    return rho, centre


def sphere_potential(px, py, pz, centre, radius: float, mass: float, G: float = 1.0):
    """Closed-form potential of a uniform sphere (Sec. 4.2): -GM/r outside,
    -GM (3R^2 - r^2) / (2 R^3) inside."""
    dx = np.asarray(px, dtype=np.float64) - centre[0]
    dy = np.asarray(py, dtype=np.float64) - centre[1]
    dz = np.asarray(pz, dtype=np.float64) - centre[2]
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    rs = np.maximum(r, 1e-300)
    outside = -G * mass / rs
    inside = -G * mass * (3.0 * radius * radius - r * r) / (2.0 * radius ** 3)
    return np.where(r >= radius, outside, inside)


def sphere_face_values(n: int, centre, radius: float, mass: float, G: float = 1.0,
                       length: float = 1.0):
    """Analytic sphere potential at the face centres of the six domain faces.

    Returns a list of six (n, n) arrays for faces -x,+x,-y,+y,-z,+z.  Each array
    is indexed [t2][t1] where (t1, t2) are the face's two transverse axes in
    increasing axis order (x-faces: (y, z); y-faces: (x, z); z-faces: (x, y)).
    """
    c = cell_centres(n, length)
    t1 = c[None, :]
    t2 = c[:, None]
    faces = []
    for axis in range(3):
        for side in range(2):
            pos = 0.0 if side == 0 else length
            if axis == 0:
                v = sphere_potential(pos, t1, t2, centre, radius, mass, G)
            elif axis == 1:
                v = sphere_potential(t1, pos, t2, centre, radius, mass, G)
            else:
                v = sphere_potential(t1, t2, pos, centre, radius, mass, G)
            faces.append(np.ascontiguousarray(np.broadcast_to(v, (n, n)), dtype=np.float64))
    return faces


def lognormal_grf(n: int, seed: int, slope: float = -4.0, sigma: float = 1.0,
                  remove_mean: bool = True) -> np.ndarray:
    """rho = exp(g), g a Gaussian random field with power spectrum P(k) ~ k^slope.

    White N(0,1) noise -> FFT -> multiply by |k|^(slope/2) (k = 0 zeroed, integer
    wave numbers) -> inverse FFT -> scale to standard deviation ``sigma``.
    """
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(white)
    k = np.fft.fftfreq(n, d=1.0 / n)
    kr = np.fft.rfftfreq(n, d=1.0 / n)
    kk = np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + kr[None, None, :] ** 2)
    amp = np.zeros_like(kk)
    nz = kk > 0
    amp[nz] = kk[nz] ** (0.5 * slope)
    g = np.fft.irfftn(wk * amp, s=(n, n, n), axes=(0, 1, 2))
    g *= sigma / g.std()
    rho = np.exp(g)
    if remove_mean:
        rho -= rho.mean()
    return np.ascontiguousarray(rho)


def serving_trace(n_requests: int, seed: int, rate: float,
                  sizes=(64, 128, 256, 512), bcs=("periodic", "fixed", "multipole")):
    """Poisson-arrival request trace: list of dicts with arrival time, size, bc and seed."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    ns = rng.choice(np.asarray(sizes), size=n_requests)
    bi = rng.integers(0, len(bcs), size=n_requests)
    seeds = rng.integers(0, 2 ** 31 - 1, size=n_requests)
    return [
        {"id": i, "t": float(t[i]), "n": int(ns[i]), "bc": bcs[int(bi[i])], "seed": int(seeds[i])}
        for i in range(n_requests)
    ]
