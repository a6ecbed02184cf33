"""Pins of the refined-mesh oracle (Sec. 3.3; level boundaries eqs. masscons-lbext; FAS V-cycle
on MeshBlock, Octet and root levels) against facts that do not come from it: the composite
operator is exact for linear fields and conserves mass (the paper's reason for the
conservative formulation), equals the uniform 7-point operator away from level boundaries,
the multigrid iteration converges to the dense direct solve of the composite system (whose
solution is a fixed point of one V-cycle), and the refined solution of a smooth density is
second-order accurate against the analytic potential, well ahead of the uniform coarse grid.
CPU only."""
import math

import numpy as np
import pytest

import oracle
from oracle import amr

FPG = 4 * math.pi


def grids(m, k=None):
    out = []
    for l in range(m.Lam + 1):
        x, y, z = m.centres(l, k)
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        out.append((X, Y, Z))
    return out


MESHES = {
    "one level": lambda: amr.AmrMesh(4, 4, [((1, 1, 1), (3, 3, 3))]),
    "two levels": lambda: amr.AmrMesh(4, 4, [((1, 1, 1), (3, 3, 3)), ((3, 3, 3), (5, 5, 5))]),
    "off-centre box": lambda: amr.AmrMesh(4, 2, [((1, 2, 1), (3, 3, 2))]),
}


@pytest.mark.parametrize("name", list(MESHES))
def test_linear_fields_are_exact(name):
    """Linear phi with fixed faces holding its values: every ghost (physical, fine-side
    interpolation, coarse-side extrapolation) is exact, so L phi = 0 in every active cell,
    on both sides of every level boundary."""
    m = MESHES[name]()
    a = (0.7, -1.3, 2.1)
    lin = lambda x, y, z: 0.4 + a[0] * x + a[1] * y + a[2] * z
    phi = [lin(X, Y, Z) for X, Y, Z in grids(m)]
    L = amr.composite_laplacian(m, phi, [amr.FIXED] * 6, lin)
    hmin = m.patches[m.Lam][m.K].h
    assert max(np.abs(x).max() for x in L) < 1e-10 / hmin ** 2 * 1e-3


@pytest.mark.parametrize("name", list(MESHES))
def test_mass_conservation(name):
    """Periodic domain, arbitrary phi: the volume integral of the composite Laplacian vanishes
    (the fluxes through every coarse face equal the mean of the four fine fluxes, eq. masscons,
    so they telescope).  A non-conservative level boundary leaves a residue of order
    h^2 |L phi|."""
    m = MESHES[name]()
    rng = np.random.default_rng(1)
    phi = [rng.normal(size=m.patches[l][m.K].n[::-1]) for l in range(m.Lam + 1)]
    L = amr.composite_laplacian(m, phi, [amr.PERIODIC] * 6)
    tot = sum(m.patches[l][m.K].h ** 3 * L[l].sum() for l in range(m.Lam + 1))
    scale = sum(m.patches[l][m.K].h ** 3 * np.abs(L[l]).sum() for l in range(m.Lam + 1))
    assert abs(tot) < 1e-13 * scale


def test_uniform_operator_away_from_level_boundaries():
    """Cells whose six neighbours are in their own patch see the plain 7-point operator: the
    uniform oracle's defect on the root patch agrees there (to rounding)."""
    m = MESHES["one level"]()
    rng = np.random.default_rng(2)
    phi = [rng.normal(size=m.patches[l][m.K].n[::-1]) for l in range(m.Lam + 1)]
    L = amr.composite_laplacian(m, phi, [amr.PERIODIC] * 6)
    p0 = m.patches[0][m.K]
    d = oracle.defect(phi[0], np.zeros_like(phi[0]), p0.h, oracle.PERIODIC)     # -L phi
    (x0, y0, z0), (x1, y1, z1) = p0.hole
    far = np.ones_like(phi[0], dtype=bool)
    far[z0 - 1:z1 + 1, y0 - 1:y1 + 1, x0 - 1:x1 + 1] = False
    assert np.max(np.abs(L[0][far] + d[far])) < 1e-12 * np.abs(d).max()


def dense_composite_solve(m, rho, kinds, bfun):
    """Assemble the composite operator column by column (unit potentials on the active cells)
    and solve L phi = f directly."""
    act = [m.patches[l][m.K].active() for l in range(m.Lam + 1)]
    sizes = [int(a.sum()) for a in act]
    N = sum(sizes)

    def unpack(v):
        out, o = [], 0
        for l in range(m.Lam + 1):
            a = np.zeros(act[l].shape)
            a[act[l]] = v[o:o + sizes[l]]
            out.append(a)
            o += sizes[l]
        return out

    def pack(arrs):
        return np.concatenate([arrs[l][act[l]] for l in range(m.Lam + 1)])

    g = pack(amr.composite_laplacian(m, unpack(np.zeros(N)), kinds, bfun))
    A = np.zeros((N, N))
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        A[:, c] = pack(amr.composite_laplacian(m, unpack(e), kinds, None))
    f = pack([FPG * r for r in rho])
    return unpack(np.linalg.solve(A, f - g))


@pytest.mark.parametrize("name", ["one level", "off-centre box"])
def test_converges_to_dense_composite_solve(name):
    m = amr.AmrMesh(4, 2, [((1, 1, 1), (3, 3, 3))]) if name == "one level" else MESHES[name]()
    rng = np.random.default_rng(3)
    rho = [rng.uniform(0, 1, m.patches[l][m.K].n[::-1]) for l in range(m.Lam + 1)]
    bfun = lambda x, y, z: 0.1 * x - 0.2 * y * z
    ref = dense_composite_solve(m, rho, [amr.FIXED] * 6, bfun)
    phi, hist = amr.solve(m, rho, [amr.FIXED] * 6, bfun, tol=1e-13)
    assert hist[-1] <= 1e-13
    num = math.sqrt(sum(np.sum((phi[l] - ref[l]) ** 2) for l in range(m.Lam + 1)))
    den = math.sqrt(sum(np.sum(ref[l] ** 2) for l in range(m.Lam + 1)))
    assert num / den < 1e-11
    # the exact composite solution is a fixed point of one V-cycle
    phi1, h1 = amr.solve(m, rho, [amr.FIXED] * 6, bfun, phi0=ref, cycles=1)
    assert h1[0] < 1e-12 and h1[1] < 1e-12
    assert max(np.abs(phi1[l] - ref[l]).max() for l in range(m.Lam + 1)) < 1e-12 * max(np.abs(r).max() for r in ref)


@pytest.mark.parametrize("name", list(MESHES))
def test_vcycle_contracts(name):
    """FAS V(2,2) on the refined mesh reduces the composite residual by at least 5x per cycle
    (measured ~15x), from zero to below 1e-10 within 12 cycles."""
    m = MESHES[name]()
    rho = []
    for X, Y, Z in grids(m):
        r = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2)
        rho.append(np.where(r < 0.2, 1.0, 0.0))
    phi, hist = amr.solve(m, rho, [amr.PERIODIC] * 6, cycles=12)
    assert hist[-1] < 1e-10
    for a, b in zip(hist[1:6], hist[2:7]):
        assert b < 0.2 * a


def _gaussian_case(NB, nb):
    """Gaussian density (sigma = 0.04, centred in the refined box) with its analytic potential
    -M erf(r / (sqrt(2) sigma)) / r on the domain faces; returns (refined-region error,
    error of the uniform root-resolution solve in the same region)."""
    from scipy.special import erf
    sig, c = 0.04, np.array([0.5, 0.5, 0.5])
    M = (2 * math.pi * sig * sig) ** 1.5

    def exact(x, y, z):
        r = np.maximum(np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2), 1e-12)
        return -M * erf(r / (math.sqrt(2) * sig)) / r

    def dens(X, Y, Z):
        return np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / (2 * sig * sig))

    m = amr.AmrMesh(NB, nb, [((1, 1, 1), (3, 3, 3))])
    gs = grids(m)
    phi, hist = amr.solve(m, [dens(*g) for g in gs], [amr.FIXED] * 6, exact, tol=1e-11)
    err_fine = np.abs(phi[1] - exact(*gs[1])).max()
    n = NB * nb
    x = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    faces = []
    for face in range(6):
        axis, side = face // 2, face % 2
        t = [q for q in range(3) if q != axis]
        co = [None, None, None]
        co[axis] = np.array(0.0 if side == 0 else 1.0)
        co[t[0]] = x[None, :]
        co[t[1]] = x[:, None]
        faces.append(np.ascontiguousarray(np.broadcast_to(exact(*co), (n, n))))
    phi_u, _, _ = oracle.solve(dens(X, Y, Z), 1.0 / n, [oracle.FIXED] * 6, fixed_b=faces, tol=1e-11)
    lo, hi = m.patches[0][m.K].hole
    sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
    return err_fine, np.abs(phi_u - exact(X, Y, Z))[sl].max()


def test_refinement_accuracy_against_analytic():
    """Second-order accuracy through the level boundary: in the refined region the error
    against the analytic potential is about a quarter of the uniform coarse grid's (measured
    0.30), and it falls about fourfold when the resolution doubles (measured 3.9x)."""
    e4, _ = _gaussian_case(4, 4)
    e8, u8 = _gaussian_case(4, 8)
    assert e8 < 0.35 * u8, (e8, u8)
    assert e8 < 0.3 * e4, (e4, e8)


def test_face_arrays_match_point_values_for_linear_b():
    """Fixed faces given as arrays (area means on coarser levels) equal the pointwise face
    function when b is linear along the face (its area mean is its centre value): the two
    solves agree to rounding."""
    m = MESHES["one level"]()
    N = m.NB * m.nb
    bfun = lambda x, y, z: 0.3 + 0.1 * x - 0.2 * y + 0.05 * z
    x = (np.arange(N) + 0.5) / N
    faces = []
    for face in range(6):
        axis, side = face // 2, face % 2
        t = [q for q in range(3) if q != axis]
        co = [None, None, None]
        co[axis] = np.array(0.0 if side == 0 else 1.0)
        co[t[0]] = x[None, :]
        co[t[1]] = x[:, None]
        faces.append(np.ascontiguousarray(np.broadcast_to(bfun(*co), (N, N))))
    rng = np.random.default_rng(4)
    rho = [rng.uniform(0, 1, m.patches[l][m.K].n[::-1]) for l in range(m.Lam + 1)]
    a, ha = amr.solve(m, rho, [amr.FIXED] * 6, bfun, cycles=4)
    b, hb = amr.solve(m, rho, [amr.FIXED] * 6, amr.FaceArrays(faces), cycles=4)
    assert np.allclose(ha, hb, rtol=1e-9)
    assert max(np.abs(a[l] - b[l]).max() for l in range(m.Lam + 1)) < 1e-12


def test_fmg_converges_to_dense_composite_solve():
    """FMG (Alg. 2 with FAS) on the refined hierarchy followed by V-cycles reaches the dense
    direct solution of the composite system, from a far better start than zero."""
    m = amr.AmrMesh(4, 2, [((1, 1, 1), (3, 3, 3))])
    rng = np.random.default_rng(6)
    rho = [rng.uniform(0, 1, m.patches[l][m.K].n[::-1]) for l in range(m.Lam + 1)]
    bfun = lambda x, y, z: 0.1 * x - 0.2 * y * z
    ref = dense_composite_solve(m, rho, [amr.FIXED] * 6, bfun)
    phi, hist = amr.solve(m, rho, [amr.FIXED] * 6, bfun, tol=1e-13, mode="fmg")
    assert hist[0] < 0.1 and hist[-1] <= 1e-13
    num = math.sqrt(sum(np.sum((phi[l] - ref[l]) ** 2) for l in range(m.Lam + 1)))
    den = math.sqrt(sum(np.sum(ref[l] ** 2) for l in range(m.Lam + 1)))
    assert num / den < 1e-11


def test_fmg_reaches_truncation_error():
    """One FMG sweep already has an error against the analytic potential of the order of the
    discretisation error (Sec. 2.3.4): within 1.5x of the converged solution's, on the
    Gaussian of the accuracy test (two refinement levels)."""
    from scipy.special import erf
    sig, c = 0.04, np.array([0.5, 0.5, 0.5])
    M = (2 * math.pi * sig * sig) ** 1.5

    def exact(x, y, z):
        r = np.maximum(np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2), 1e-12)
        return -M * erf(r / (math.sqrt(2) * sig)) / r

    m = amr.AmrMesh(4, 4, [((1, 1, 1), (3, 3, 3)), ((3, 3, 3), (5, 5, 5))])
    gs = grids(m)
    rho = [np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2) / (2 * sig * sig)) for X, Y, Z in gs]
    f0, _ = amr.solve(m, rho, [amr.FIXED] * 6, exact, mode="fmg", cycles=0)
    fc, _ = amr.solve(m, rho, [amr.FIXED] * 6, exact, mode="fmg", tol=1e-11)
    act = [m.patches[l][m.K].active() for l in range(m.Lam + 1)]
    e0 = max(np.abs(f0[l] - exact(*gs[l]))[act[l]].max() for l in range(m.Lam + 1))
    ec = max(np.abs(fc[l] - exact(*gs[l]))[act[l]].max() for l in range(m.Lam + 1))
    assert e0 < 1.5 * ec, (e0, ec)


TWO_SMALL = (4, 2, [((1, 1, 1), (3, 3, 3)), ((3, 3, 3), (5, 5, 5))])


def test_fmg_sources_are_volume_means():
    """Alg. 2 step 1 on the refined hierarchy: every Octet-level cell's source is the volume
    mean of the finest composite source over the cell (a covered cell averages the finer
    patches inside it), computed here directly from cell positions."""
    NB, nb, boxes = TWO_SMALL
    m = amr.AmrMesh(NB, nb, boxes)
    rng = np.random.default_rng(8)
    rho = [rng.uniform(0, 1, m.patches[l][m.K].n[::-1]) for l in range(m.Lam + 1)]
    st = amr.AmrState(m, rho, [amr.FIXED] * 6)
    st.fmg_sources()
    for t in range(m.Lam + 1):
        pt = m.patches[t][0]
        acc = np.zeros(pt.n[::-1])
        vol = np.zeros(pt.n[::-1])
        B = pt.h
        for l in range(t, m.Lam + 1):
            p = m.patches[l][m.K]
            act = p.active()
            x, y, z = m.centres(l)
            Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
            ix = np.floor(X / B).astype(int) - pt.origin[0]
            iy = np.floor(Y / B).astype(int) - pt.origin[1]
            iz = np.floor(Z / B).astype(int) - pt.origin[2]
            sel = act & (ix >= 0) & (ix < pt.n[0]) & (iy >= 0) & (iy < pt.n[1]) & (iz >= 0) & (iz < pt.n[2])
            np.add.at(acc, (iz[sel], iy[sel], ix[sel]), p.h ** 3 * FPG * rho[l][sel])
            np.add.at(vol, (iz[sel], iy[sel], ix[sel]), p.h ** 3)
        want = acc / vol
        got = st.fsrc[t][1:-1, 1:-1, 1:-1] if t > 0 else st.rfsrc[NB][1:-1, 1:-1, 1:-1]
        assert np.allclose(got, want, rtol=1e-13, atol=1e-12), t


@pytest.mark.parametrize("lam", [1, 2])
def test_octet_cycle_fixed_point(lam):
    """A V-cycle started on Octet level lam leaves the exact solution of that level's composite
    problem unchanged.  That problem is the composite operator of the same boxes at one cell
    per MeshBlock (a mesh with nb = 1), solved here densely with the FMG sources; the uncovered
    cells of the coarser patches must enter the cycle with their defect in this problem."""
    NB, nb, boxes = TWO_SMALL
    m = amr.AmrMesh(NB, nb, boxes)
    rng = np.random.default_rng(9)
    rho = [rng.uniform(0, 1, m.patches[l][m.K].n[::-1]) for l in range(m.Lam + 1)]
    bfun = lambda x, y, z: 0.2 + 0.1 * x - 0.3 * z
    st = amr.AmrState(m, rho, [amr.FIXED] * 6, bfun)
    st.fmg_sources()
    m1 = amr.AmrMesh(NB, 1, boxes[:lam])
    srcs = [st.rfsrc[NB][1:-1, 1:-1, 1:-1]] + [st.fsrc[l][1:-1, 1:-1, 1:-1] for l in range(1, lam + 1)]
    exact = dense_composite_solve(m1, [s / FPG for s in srcs], [amr.FIXED] * 6, bfun)
    for l in range(lam + 1):
        st.u[l][0][1:-1, 1:-1, 1:-1] = exact[l]
    st.vcycle(("oct", lam))
    act1 = [m1.patches[l][0].active() for l in range(lam + 1)]
    scale = max(np.abs(e).max() for e in exact)
    for l in range(lam + 1):
        got = st.u[l][0][1:-1, 1:-1, 1:-1]
        assert np.max(np.abs(got - exact[l])[act1[l]]) < 1e-11 * scale, l


@pytest.mark.parametrize("name", list(MESHES))
def test_fmg_exact_for_linear_potentials(name):
    """f = 0 with fixed faces holding a linear field: the composite problem's solution is that
    field, and every FMG stage reproduces it exactly (the tricubic and trilinear
    prolongations, the physical ghosts and the normal level boundary are exact for linear
    fields, and V-cycles leave an exact solution alone), so one FMG sweep alone returns it."""
    m = MESHES[name]()
    a = (0.7, -1.3, 2.1)
    lin = lambda x, y, z: 0.4 + a[0] * x + a[1] * y + a[2] * z
    rho = [np.zeros(m.patches[l][m.K].n[::-1]) for l in range(m.Lam + 1)]
    phi, hist = amr.solve(m, rho, [amr.FIXED] * 6, lin, mode="fmg", cycles=0)
    for l, (X, Y, Z) in enumerate(grids(m)):
        act = m.patches[l][m.K].active()
        assert np.max(np.abs(phi[l] - lin(X, Y, Z))[act]) < 1e-12, l


def _binary(NB, nb, **kw):
    import workloads as wl
    m = amr.AmrMesh(NB, nb, wl.binary_mesh_boxes(NB))
    gs = grids(m)
    rho = [wl.binary_density_on_axes(*m.centres(l), m.patches[l][m.K].h) for l in range(m.Lam + 1)]
    phi, hist = amr.solve(m, rho, [amr.FIXED] * 6, wl.binary_potential, mode="fmg", **kw)
    err = []
    for l in range(m.Lam + 1):
        ex = wl.binary_potential(*gs[l])
        err.append(((phi[l] - ex) / ex)[m.patches[l][m.K].active()])
    e = np.concatenate(err)
    return math.sqrt(np.mean(e * e)), hist


def test_binary_potential_second_order():
    """The paper's refined-mesh test (Sec. 4.3): the unequal-mass binary on four nested levels
    of refinement (16x the root resolution at the stars), analytic potential on the faces.
    The normalised error against the analytic potential is small and falls about fourfold per
    doubling of the root resolution (measured 3.0x from h = 1/32 to 1/64, where the stars
    span a few fine cells); FMG reaches that error within a few V-cycles (saturation:
    measured 12x, 3.7x, 1.5x, 1.07x of it after 0, 1, 2, 3 cycles)."""
    e8, h8 = _binary(4, 8, tol=1e-10)
    e16, h16 = _binary(4, 16, tol=1e-10)
    assert h16[-1] <= 1e-10 and len(h16) - 1 <= 12
    assert e16 < 1e-3
    assert e8 / e16 > 2.5, (e8, e16)
    f16, _ = _binary(4, 16, cycles=3)
    assert f16 < 1.2 * e16, (f16, e16)


# ------------------------------------------------------------------ multipole faces (Appendix A)

def _legendre_expansion(px, py, pz, mass, origin, lmax, r):
    """-G sum_c m_c sum_{l<=lmax} |r_c|^l / |r|^(l+1) P_l(cos gamma_c) (G = 1): the same
    truncated expansion written through the addition theorem, independent of any harmonic table."""
    from numpy.polynomial import legendre
    rc = np.stack([px, py, pz], axis=1) - origin
    rv = np.asarray(r, dtype=np.float64) - origin
    a, b = np.linalg.norm(rc, axis=1), np.linalg.norm(rv)
    cosg = np.where(a > 0, rc @ rv / np.maximum(a, 1e-300) / b, 0.0)
    tot = 0.0
    for l in range(lmax + 1):
        pl = legendre.legval(cosg, [0.0] * l + [1.0])
        tot += np.sum(mass * a ** l * pl) / b ** (l + 1)
    return -tot


def test_composite_multipole_matches_point_mass_sum():
    """Composite moments over the active cells only (a mass put under the refined box is
    ignored; the refined cells count at their own centres and volumes), checked through the
    Legendre form of the expansion at points on the domain faces, for both origins."""
    m = amr.AmrMesh(4, 4, [((1, 1, 1), (3, 3, 3))])
    rng = np.random.default_rng(7)
    rho = [np.zeros(m.patches[l][m.K].n[::-1]) for l in range(m.Lam + 1)]
    # coarse active cells, one covered coarse cell, refined cells
    for (z, y, x) in [(1, 2, 3), (14, 3, 9), (8, 12, 2)]:
        rho[0][z, y, x] = rng.uniform(1, 3)
    rho[0][6, 7, 8] = 100.0                       # under the box: covered, ignored
    assert not m.patches[0][m.K].active()[6, 7, 8]
    for (z, y, x) in [(0, 0, 0), (15, 4, 11), (7, 8, 9), (3, 14, 5)]:
        rho[1][z, y, x] = rng.uniform(1, 3)
    px, py, pz, pm = [], [], [], []
    for l in range(m.Lam + 1):
        p = m.patches[l][m.K]
        cx, cy, cz = m.centres(l)
        for (z, y, x) in zip(*np.nonzero(rho[l] * p.active())):
            px.append(cx[x]); py.append(cy[y]); pz.append(cz[z]); pm.append(rho[l][z, y, x] * p.h ** 3)
    px, py, pz, pm = (np.array(v) for v in (px, py, pz, pm))
    for given in (None, np.array([0.5, 0.5, 0.5])):
        o, q = amr.composite_moments(m, rho, 4, given)
        if given is None:
            com = np.array([np.sum(pm * px), np.sum(pm * py), np.sum(pm * pz)]) / np.sum(pm)
            np.testing.assert_allclose(o, com, rtol=0, atol=1e-15)
            np.testing.assert_allclose(q[1:4], 0.0, atol=1e-15)   # no dipole about the centre of mass
        np.testing.assert_allclose(q[0], np.sum(pm), rtol=1e-14)
        for lmax in (0, 2, 4):
            for r in [(0.0, 0.3, 0.6), (1.0, 0.55, 0.1), (0.2, 1.0, 0.9), (0.7, 0.4, 0.0)]:
                want = _legendre_expansion(px, py, pz, pm, o, lmax, r)
                got = oracle.multipole_potential_points(*(np.array([c]) for c in r), q, o, lmax)[0]
                assert abs(got - want) <= 1e-13 * abs(want), (lmax, r, got, want)


def test_multipole_faces_per_root_level():
    """Face values sit at each root level's face centres: the one-cell level holds the
    expansion at the six face midpoints, and at every level a face's values are the expansion
    at ((t1 + 1/2)/n, (t2 + 1/2)/n) on that face (indexed [t2][t1], transverse axes ascending)."""
    o = np.array([0.45, 0.52, 0.5])
    q = np.zeros(25)
    q[0], q[6], q[20] = 1.5, 0.01, -0.002
    mf = amr.MultipoleFaces(8, q, o, 4)
    # monopole + quadrupole + hexadecapole along z: compare against a direct point evaluation
    for n in (8, 4, 2, 1):
        for face in range(6):
            axis = face // 2
            arr = mf.at(n)[face]
            assert arr.shape == (n, n)
            t2, t1 = n - 1, 0
            c = [(t1 + 0.5) / n, (t2 + 0.5) / n]
            pt = c[:axis] + [1.0 if face & 1 else 0.0] + c[axis:]
            rv = np.array(pt) - o
            r = np.linalg.norm(rv)
            mu = rv[2] / r
            p2 = 0.5 * (3 * mu * mu - 1)
            p4 = (35 * mu ** 4 - 30 * mu ** 2 + 3) / 8
            want = -(q[0] / r + q[6] * p2 / r ** 3 + q[20] * p4 / r ** 5)
            assert abs(arr[t2, t1] - want) <= 1e-13 * abs(want), (n, face)


def _binary_mp(NB, nb):
    import workloads as wl
    m = amr.AmrMesh(NB, nb, wl.binary_mesh_boxes(NB))
    rho = [wl.binary_density_on_axes(*m.centres(l), m.patches[l][m.K].h) for l in range(m.Lam + 1)]
    mp = amr.multipole_faces(m, rho, 4)
    phi_mp, h_mp = amr.solve(m, rho, [amr.FIXED] * 6, mp, mode="fmg", tol=1e-10)
    # the analytic potential scaled to the discretised mass (cell-averaged spheres)
    s = amr.composite_moments(m, rho, 0)[1][0] / 3.0
    phi_an, _ = amr.solve(m, rho, [amr.FIXED] * 6, lambda x, y, z: s * wl.binary_potential(x, y, z),
                          mode="fmg", tol=1e-10)
    return m, rho, mp, phi_mp, phi_an, h_mp


def test_binary_multipole_faces_match_analytic_faces():
    """The paper's binary test with its open boundaries (hexadecapole expansion about the
    centre of mass): the stars are 18/1024 apart and the faces at least 1/2 away, so the
    truncated expansion matches the analytic potential on the faces to about (18/512)^5 of
    it, and the solution with multipole faces matches the one with analytic faces as
    closely once both carry the discretised mass (the cell-averaged spheres hold 3 (1 + 6e-5)
    at this resolution); the centre of mass is the domain centre."""
    import workloads as wl
    m, rho, mp, phi_mp, phi_an, h_mp = _binary_mp(4, 8)
    assert h_mp[-1] <= 1e-10
    o, q = amr.composite_moments(m, rho, 4)
    assert abs(q[0] / 3.0 - 1.0) < 1e-4
    assert np.max(np.abs(o - 0.5)) < 1e-12       # 2 (+6/1024) + 1 (-12/1024) = 0 about the centre
    N = m.NB * m.nb
    t = (np.arange(N) + 0.5) / N
    T2, T1 = np.meshgrid(t, t, indexing="ij")
    ex = wl.binary_potential(np.zeros_like(T1), T1, T2)
    assert np.max(np.abs(mp.at(N)[0] - q[0] / 3.0 * ex) / np.abs(ex)) < 1e-6
    num = sum(np.sum((a - b) ** 2) for a, b in zip(phi_mp, phi_an))
    den = sum(np.sum(b ** 2) for b in phi_an)
    rel = math.sqrt(num / den)
    assert rel < 1e-8, rel          # measured 9e-12


def test_composite_multipole_zero_mass():
    """No mass: the origin falls back to the domain centre and every moment and face value is 0."""
    m = amr.AmrMesh(4, 2, [((1, 1, 1), (3, 3, 3))])
    rho = [np.zeros(m.patches[l][m.K].n[::-1]) for l in range(m.Lam + 1)]
    o, q = amr.composite_moments(m, rho, 4)
    assert np.all(o == 0.5) and np.all(q == 0.0)
    mf = amr.multipole_faces(m, rho, 4)
    assert all(np.all(a == 0.0) for n in (8, 4, 2, 1) for a in mf.at(n))
