"""Oracle of the multigrid solver on a statically refined mesh (Sec. 3.3 of Tomida & Stone,
arXiv:2302.13903): FAS V-cycles (Alg. 3) over the MeshBlock levels, the Octet levels and the
root grid, with the conservative level boundary (eqs. masscons, transgrad, piint, lbint,
lbext) before smoothing and defect computation, and the normal level boundary (restriction
and trilinear prolongation) before the prolongation of corrections.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's CPU baseline may
use it; the product never imports it.  Plain FP64 numpy, written for clarity: every operator
fills ghosts first, then applies its formula to whole arrays.

Mesh model (a nested special case of the octree of MeshBlocks):
  - the root grid is NB^3 MeshBlocks of nb^3 cells (nb a power of two) on the unit cube;
  - refinement level lam = 1..Lam is one box of level-(lam-1) MeshBlocks, each refined into
    2 x 2 x 2 level-lam MeshBlocks; box lam lies inside box lam-1 (inside the root domain for
    lam = 1) with at least one level-(lam-1) MeshBlock between the two boundaries (the 2:1
    balance of neighbouring blocks);
  - on MG level k (2^k cells per MeshBlock side, k = K..0 with nb = 2^K) refinement level lam
    is one dense patch P[lam][k] covering its box, with one ghost layer; the cells of P[lam]
    under box lam+1 are covered (not active).
Readings of the paper taken here (and in the GPU path):
  - transverse gradient of eq. transgrad: the centred coarse difference over two coarse cells,
    (phi_{J+1} - phi_{J-1}) / (2 H) with H the coarse spacing; with the +-h/2 offsets of
    eq. piint (h the fine spacing) the interpolation is then exact for linear fields and the
    four points average to the coarse value, as the paper states;
  - a coarse active cell next to a covered cell takes one ghost per face (eq. lbext), so a
    cell facing the refined region on two faces sees two different ghost values;
  - the Octet levels are the patches of each refinement level at k = 0 (one cell per
    MeshBlock), smoothed finest first with the conservative ghosts from the next coarser
    patch held fixed, then restricted into the covered cells of that patch; the root grid
    (P[0][0], NB^3 cells) is then solved by a uniform FAS V-cycle;
  - the FAS coarse source of a patch at level k-1 (and of the Octet and root levels) is the
    restricted defect plus the level's own operator applied to the restricted potential;
    corrections psi - phibar are prolongated with the normal level boundary and homogeneous
    physical conditions;
  - domain faces are periodic, zero-gradient or fixed (b given as a function of position,
    evaluated at every level's face points, as the multipole values of the uniform solver);
  - multipole faces (Appendix A) take their moments over the composite grid: every active cell
    of every patch at the finest MG level, at its centre with mass rho h^3 (covered cells
    excluded, since the finer patch holds that mass); the truncated expansion is evaluated at
    the face centres of every root level (N, N/2, .., 1 cells per side), not area-averaged.
Parity unpinned parts: none beyond the pins of tests/test_oracle_amr.py.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

PERIODIC, ZERO_GRADIENT, FIXED = 0, 1, 2
FOUR_PI_G = 4.0 * math.pi

Box = Tuple[Tuple[int, int, int], Tuple[int, int, int]]   # (lo, hi) in parent-block units, (x, y, z)


@dataclass
class Patch:
    lam: int
    k: int
    origin: Tuple[int, int, int]      # global index of local cell 0 (x, y, z) at (lam, k)
    n: Tuple[int, int, int]           # cells per side (x, y, z)
    h: float
    hole: Optional[Tuple[Tuple[int, int, int], Tuple[int, int, int]]] = None   # local [lo, hi) of covered cells

    def shape(self):
        nx, ny, nz = self.n
        return (nz + 2, ny + 2, nx + 2)

    def active(self) -> np.ndarray:
        nx, ny, nz = self.n
        a = np.ones((nz, ny, nx), dtype=bool)
        if self.hole is not None:
            (x0, y0, z0), (x1, y1, z1) = self.hole
            a[z0:z1, y0:y1, x0:x1] = False
        return a


def interior(a):
    return a[1:-1, 1:-1, 1:-1]


class AmrMesh:
    """Static nested refinement: NB^3 root blocks of nb^3 cells; boxes[lam-1] = (lo, hi) of
    refinement level lam in level-(lam-1) block units."""

    def __init__(self, NB: int, nb: int, boxes: Sequence[Box]):
        assert nb >= 1 and nb & (nb - 1) == 0     # nb = 1: operators at one cell per block only
        self.NB, self.nb = NB, nb
        self.K = int(round(math.log2(nb)))
        self.boxes = [tuple(tuple(int(v) for v in c) for c in b) for b in boxes]
        self.Lam = len(self.boxes)
        # validate nesting with a one-block margin
        for lam, (lo, hi) in enumerate(self.boxes, start=1):
            parent_n = NB if lam == 1 else 2 * (self.boxes[lam - 2][1][0] - self.boxes[lam - 2][0][0])
            for a in range(3):
                if lam == 1:
                    plo, phi_ = 0, NB
                else:
                    plo, phi_ = 2 * self.boxes[lam - 2][0][a], 2 * self.boxes[lam - 2][1][a]
                if not (plo + 1 <= lo[a] < hi[a] <= phi_ - 1):
                    raise ValueError(f"box {lam} must lie inside its parent with a one-block margin")
            del parent_n
        self.patches = [[self._patch(lam, k) for k in range(self.K + 1)] for lam in range(self.Lam + 1)]

    def block_origin(self, lam: int) -> Tuple[int, int, int]:
        """Global index (level-lam block units) of the first block of patch lam."""
        if lam == 0:
            return (0, 0, 0)
        lo = self.boxes[lam - 1][0]
        return tuple(2 * v for v in lo)

    def block_count(self, lam: int) -> Tuple[int, int, int]:
        if lam == 0:
            return (self.NB,) * 3
        lo, hi = self.boxes[lam - 1]
        return tuple(2 * (hi[a] - lo[a]) for a in range(3))

    def _patch(self, lam: int, k: int) -> Patch:
        c = 1 << k
        bo, bn = self.block_origin(lam), self.block_count(lam)
        origin = tuple(bo[a] * c for a in range(3))
        n = tuple(bn[a] * c for a in range(3))
        h = 1.0 / (self.NB * (1 << lam) * c)
        hole = None
        if lam < self.Lam:
            lo, hi = self.boxes[lam]          # level-lam block units (global)
            hole = (tuple(lo[a] * c - origin[a] for a in range(3)), tuple(hi[a] * c - origin[a] for a in range(3)))
        return Patch(lam, k, origin, n, h, hole)

    def centres(self, lam: int, k: int = None):
        """Cell-centre coordinates (x, y, z) 1-D arrays of patch lam at MG level k (default K)."""
        k = self.K if k is None else k
        p = self.patches[lam][k]
        return tuple((p.origin[a] + np.arange(p.n[a]) + 0.5) * p.h for a in range(3))


# ------------------------------------------------------------------ physical ghosts (root patch)

def fill_physical(u: np.ndarray, p: Patch, kinds, bfun: Optional[Callable], homogeneous: bool):
    """Sec. 2.3.6 ghost rules on the domain faces of the root patch, axis by axis (x, y, z),
    each pass covering the ghosts already filled.  Fixed faces: ghost = 2 b - u with b the
    face value at the level's face point (0 when homogeneous)."""
    nz, ny, nx = u.shape[0] - 2, u.shape[1] - 2, u.shape[2] - 2
    h = p.h
    for axis in range(3):
        for side in range(2):
            face = 2 * axis + side
            kd = kinds[face]
            # index expressions along the axis (array axis = 2 - axis)
            ax = 2 - axis
            n_ax = (nx, ny, nz)[axis]
            g = 0 if side == 0 else n_ax + 1
            a = 1 if side == 0 else n_ax
            o = n_ax if side == 0 else 1
            # transverse ranges: axes filled earlier include their ghosts
            sl = [slice(1, -1)] * 3
            for t in range(3):
                if t != axis and t < axis:
                    sl[2 - t] = slice(None)
            sg, sa, so = list(sl), list(sl), list(sl)
            sg[ax], sa[ax], so[ax] = g, a, o
            sg, sa, so = tuple(sg), tuple(sa), tuple(so)
            if kd == PERIODIC:
                u[sg] = u[so]
            elif kd == ZERO_GRADIENT:
                u[sg] = u[sa]
            else:
                if homogeneous or bfun is None:
                    b = 0.0
                elif isinstance(bfun, FaceArrays):
                    # arrays at this level's resolution, the ring repeating the nearest value
                    arr = bfun.at(nx if axis != 0 else ny)[face]
                    t = _transverse(axis)
                    m1, m2 = (nx, ny, nz)[t[0]], (nx, ny, nz)[t[1]]
                    i1 = np.arange(m1 + 2) - 1 if t[0] < axis else np.arange(m1)
                    i2 = np.arange(m2 + 2) - 1 if t[1] < axis else np.arange(m2)
                    b = arr[np.clip(i2, 0, m2 - 1)[:, None], np.clip(i1, 0, m1 - 1)[None, :]]
                else:
                    # face points: the transverse cell centres (ghost positions included)
                    coords = []
                    for t in range(3):
                        if t == axis:
                            coords.append(np.array([0.0 if side == 0 else 1.0]))
                        else:
                            m = (nx, ny, nz)[t]
                            idx = np.arange(m + 2) - 1 if t < axis else np.arange(m)
                            coords.append((idx + 0.5) * h)
                    X, Y, Z = np.meshgrid(coords[0], coords[1], coords[2], indexing="ij")
                    b = np.transpose(bfun(X, Y, Z), (2, 1, 0))     # -> [z][y][x]
                    b = np.squeeze(b, axis=ax)
                u[sg] = 2.0 * b - u[sa]


class FaceArrays:
    """Fixed-face values given as six (N, N) arrays at the finest root resolution (indexed
    [t2][t1], the transverse axes in increasing order); coarser levels take 2 x 2 area means,
    as the uniform solver does."""

    def __init__(self, faces):
        self.levels = {}
        cur = [np.asarray(b, dtype=np.float64) if b is not None else None for b in faces]
        n = next(b.shape[0] for b in cur if b is not None)
        while True:
            self.levels[n] = [np.zeros((n, n)) if b is None else b for b in cur]
            if n == 1:
                break
            cur = [0.25 * (b[0::2, 0::2] + b[0::2, 1::2] + b[1::2, 0::2] + b[1::2, 1::2]) if b is not None else None
                   for b in self.levels[n]]
            n //= 2

    def at(self, n):
        return self.levels[n]

    def point(self, face):
        return float(self.levels[1][face][0, 0])


def composite_moments(mesh: "AmrMesh", rho, lmax: int = 4, origin=None):
    """Appendix A on the refined mesh: origin (composite centre of mass unless given) and the
    25 moments Q_lm, summed over the active cells of every patch at the finest MG level (each
    cell at its centre, mass rho h^3); rho[lam] is indexed [z][y][x], covered cells ignored."""
    from . import multipole_moments_points
    xs, ys, zs, ms = [], [], [], []
    for lam in range(mesh.Lam + 1):
        p = mesh.patches[lam][mesh.K]
        cx, cy, cz = mesh.centres(lam)
        Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
        a = p.active()
        xs.append(X[a])
        ys.append(Y[a])
        zs.append(Z[a])
        ms.append(np.asarray(rho[lam], dtype=np.float64)[a] * p.h ** 3)
    return multipole_moments_points(np.concatenate(xs), np.concatenate(ys), np.concatenate(zs),
                                    np.concatenate(ms), lmax, origin)


class MultipoleFaces(FaceArrays):
    """Multipole faces (Appendix A) of the unit cube: the truncated expansion with moments q
    about `origin`, evaluated at the face centres of each root level of n = N, N/2, .., 1
    cells per side (arrays [t2][t1] like FaceArrays)."""

    def __init__(self, N: int, q, origin, lmax: int = 4, G: float = 1.0):
        from . import multipole_potential_points
        self.levels = {}
        n = N
        while n >= 1:
            t = (np.arange(n) + 0.5) / n
            T2, T1 = np.meshgrid(t, t, indexing="ij")
            faces = []
            for face in range(6):
                axis, P = face // 2, np.full_like(T1, 1.0 if face & 1 else 0.0)
                x, y, z = (P, T1, T2) if axis == 0 else (T1, P, T2) if axis == 1 else (T1, T2, P)
                faces.append(multipole_potential_points(x, y, z, q, origin, lmax, G))
            self.levels[n] = faces
            n //= 2


def multipole_faces(mesh: "AmrMesh", rho, lmax: int = 4, origin=None, G: float = 1.0) -> MultipoleFaces:
    """Open (multipole) boundary values for the refined mesh from its composite moments."""
    o, q = composite_moments(mesh, rho, lmax, origin)
    return MultipoleFaces(mesh.NB * mesh.nb, q, o, lmax, G)


# ------------------------------------------------------------------ conservative level boundary

def _slab(arr, axis, idx):
    """arr[..] at index idx along physical axis (0 = x) of a [z][y][x] array."""
    s = [slice(None)] * 3
    s[2 - axis] = idx
    return arr[tuple(s)]


def _transverse(axis):
    return [t for t in range(3) if t != axis]


def conservative_ghosts(fine: Patch, uf: np.ndarray, coarse: Patch, uc: np.ndarray):
    """Ghost layer of the fine patch (faces only) from the coarse patch (eqs. transgrad, piint,
    lbint), and the coarse ghost arrays for the six faces of its hole (eq. lbext).

    uf, uc are ghost-layered arrays holding the current values.  Returns the dict
    {face: array} of coarse ghosts, each indexed [t2][t1] over the hole face (the two
    transverse axes in increasing order); the fine ghosts are written into uf."""
    (h0x, h0y, h0z), (h1x, h1y, h1z) = coarse.hole
    hlo, hhi = (h0x, h0y, h0z), (h1x, h1y, h1z)
    cg = {}
    for axis in range(3):
        t1, t2 = _transverse(axis)
        nf_t1, nf_t2 = fine.n[t1], fine.n[t2]
        for side in range(2):
            face = 2 * axis + side
            # coarse layer outside the hole on this side (local coarse index, ghosted +1)
            cl = (hlo[axis] - 1) if side == 0 else hhi[axis]
            C = _slab(uc, axis, cl + 1)                     # 2-D [..][..] over the other two array axes
            # C is indexed by the two transverse array axes in array order (t2 slower, t1 faster)
            # coarse transverse range of the box, with one neighbour each side
            c1 = slice(hlo[t1] + 1 - 1, hhi[t1] + 1 + 1)
            c2 = slice(hlo[t2] + 1 - 1, hhi[t2] + 1 + 1)
            Cb = C[c2, c1]                                  # (m2 + 2, m1 + 2)
            phiC = Cb[1:-1, 1:-1]
            d1 = Cb[1:-1, 2:] - Cb[1:-1, :-2]               # phi_{J+1} - phi_{J-1} along t1
            d2 = Cb[2:, 1:-1] - Cb[:-2, 1:-1]               # along t2
            # fine first active layer on this side
            fl = 1 if side == 0 else fine.n[axis]
            F = _slab(uf, axis, fl)[1:-1, 1:-1]             # (nf_t2, nf_t1)
            # crosses: coarse value at the fine transverse centres, offsets -+ h/2 -> -+ D/8
            s1 = np.where(np.arange(nf_t1) % 2 == 0, -1.0, 1.0)[None, :]
            s2 = np.where(np.arange(nf_t2) % 2 == 0, -1.0, 1.0)[:, None]
            rep = lambda a: np.repeat(np.repeat(a, 2, axis=0), 2, axis=1)
            cross = rep(phiC) + s1 * rep(d1 * 0.125) + s2 * rep(d2 * 0.125)
            ghost = (1.0 / 3.0) * F + (2.0 / 3.0) * cross                       # eq. lbint
            gl = 0 if side == 0 else fine.n[axis] + 1
            tgt = _slab(uf, axis, gl)
            tgt[1:-1, 1:-1] = ghost
            # coarse ghost (eq. lbext): restricted fine first cells (area mean) and the coarse cell
            fr = 0.25 * (F[0::2, 0::2] + F[0::2, 1::2] + F[1::2, 0::2] + F[1::2, 1::2])
            cg[face] = (4.0 / 3.0) * fr - (1.0 / 3.0) * phiC
    return cg


def neighbour_sum(p: Patch, u: np.ndarray, cghost=None) -> np.ndarray:
    """Sum of the six face neighbours of every cell of patch p (ghost-filled u).  Active cells
    next to the hole take the per-face coarse ghosts (eq. lbext) instead of the covered cell."""
    nb = (u[1:-1, 1:-1, :-2] + u[1:-1, 1:-1, 2:]) + u[1:-1, :-2, 1:-1]
    nb = nb + u[1:-1, 2:, 1:-1]
    nb = nb + u[:-2, 1:-1, 1:-1]
    nb = nb + u[2:, 1:-1, 1:-1]
    if p.hole is not None and cghost is not None:
        lo, hi = p.hole
        for axis in range(3):
            t1, t2 = _transverse(axis)
            for side in range(2):
                face = 2 * axis + side
                # active cells just outside the hole face, and the covered cell they see
                a_idx = lo[axis] - 1 if side == 0 else hi[axis]
                c_idx = lo[axis] if side == 0 else hi[axis] - 1
                sl_a = [slice(None)] * 3
                sl_c = [slice(None)] * 3
                sl_a[2 - t1] = sl_c[2 - t1] = slice(lo[t1], hi[t1])
                sl_a[2 - t2] = sl_c[2 - t2] = slice(lo[t2], hi[t2])
                sl_a[2 - axis] = a_idx
                sl_c[2 - axis] = c_idx
                covered = interior(u)[tuple(sl_c)]
                nb[tuple(sl_a)] = nb[tuple(sl_a)] + (cghost[face] - covered)
    return nb


# ------------------------------------------------------------------ the solver state

class AmrState:
    def __init__(self, mesh: AmrMesh, rho: List[np.ndarray], kinds, bfun=None, npre=2, npost=2, omega=1.15,
                 four_pi_g=FOUR_PI_G):
        self.m = mesh
        self.kinds = [int(k) for k in kinds]
        self.bfun = bfun
        self.npre, self.npost, self.omega = npre, npost, omega
        K, Lam = mesh.K, mesh.Lam
        P = mesh.patches
        self.u = [[np.zeros(P[l][k].shape()) for k in range(K + 1)] for l in range(Lam + 1)]
        self.f = [[np.zeros(P[l][k].shape()) for k in range(K + 1)] for l in range(Lam + 1)]
        self.pbar = [[np.zeros(P[l][k].shape()) for k in range(K + 1)] for l in range(Lam + 1)]
        self.dres = [[np.zeros(P[l][k].shape()) for k in range(K + 1)] for l in range(Lam + 1)]
        self.act = [[P[l][k].active() for k in range(K + 1)] for l in range(Lam + 1)]
        self.gauge_free = all(k in (PERIODIC, ZERO_GRADIENT) for k in self.kinds)
        for l in range(Lam + 1):
            interior(self.f[l][K])[...] = four_pi_g * np.asarray(rho[l], dtype=np.float64)
            interior(self.f[l][K])[~self.act[l][K]] = 0.0
        if self.gauge_free:
            mean = self.volume_mean([interior(self.f[l][K]) for l in range(Lam + 1)], K)
            for l in range(Lam + 1):
                interior(self.f[l][K])[self.act[l][K]] -= mean
        self.rms_f = math.sqrt(self.volume_mean([interior(self.f[l][K]) ** 2 for l in range(Lam + 1)], K))
        # root grid hierarchy (uniform, NB^3 down to 1): potentials below NB, sources at every n
        self.root_L = int(round(math.log2(mesh.NB)))
        assert (1 << self.root_L) == mesh.NB
        self.ru, self.rf, self.rfsrc = {}, {}, {}
        n = mesh.NB
        while n >= 1:
            if n < mesh.NB:
                self.ru[n] = np.zeros((n + 2,) * 3)
            self.rf[n] = np.zeros((n + 2,) * 3)
            n //= 2
        # FMG sources: per patch at k = 0 (the Octet levels, covered cells filled from the
        # finer Octets) and the MeshBlock levels
        self.fsrc = [None] * (Lam + 1)
        self.fsrc_mb = [[f.copy() for f in fl] for fl in self.f]

    # ---- reductions over the composite grid (active cells, volume weighted)
    def volume_mean(self, per_patch, k):
        s = 0.0
        v = 0.0
        for l, a in enumerate(per_patch):
            p = self.m.patches[l][k]
            act = self.act[l][k]
            w = p.h ** 3
            s += w * float(np.sum(a[act]))
            v += w * float(np.count_nonzero(act))
        return s / v

    # ---- composite operators on MG level k (all patches)
    def fill(self, k, arrs, homogeneous=False):
        """Physical ghosts of the root patch, then the conservative level boundary of each
        finer patch; returns the coarse-side per-face ghosts for every patch with a hole."""
        P = self.m.patches
        fill_physical(arrs[0], P[0][k], self.kinds, self.bfun, homogeneous)
        cgs = [None] * (self.m.Lam + 1)
        for l in range(1, self.m.Lam + 1):
            cgs[l - 1] = conservative_ghosts(P[l][k], arrs[l], P[l - 1][k], arrs[l - 1])
        return cgs

    def laplacian_upto(self, k, arrs, top):
        """Composite L of patches 0 .. top-1 at level k, the level boundary to patch `top`
        included (patches finer than `top` ignored)."""
        P = self.m.patches
        fill_physical(arrs[0], P[0][k], self.kinds, self.bfun, False)
        cgs = []
        for l in range(1, top + 1):
            # ghosts of patch l from patch l-1 (patch `top` only lends its first cells)
            tgt = arrs[l] if l < top else arrs[l].copy()
            cgs.append(conservative_ghosts(P[l][k], tgt, P[l - 1][k], arrs[l - 1]))
        out = []
        for l in range(top):
            nb = neighbour_sum(P[l][k], arrs[l], cgs[l])
            out.append((nb - 6.0 * interior(arrs[l])) * (1.0 / (P[l][k].h * P[l][k].h)))
        return out

    def laplacian(self, k, arrs, homogeneous=False):
        cgs = self.fill(k, arrs, homogeneous)
        out = []
        for l in range(self.m.Lam + 1):
            p = self.m.patches[l][k]
            nb = neighbour_sum(p, arrs[l], cgs[l])
            out.append((nb - 6.0 * interior(arrs[l])) * (1.0 / (p.h * p.h)))
        return out

    def defect(self, k):
        L = self.laplacian(k, [self.u[l][k] for l in range(self.m.Lam + 1)])
        return [np.where(self.act[l][k], interior(self.f[l][k]) - L[l], 0.0) for l in range(self.m.Lam + 1)]

    def colour_mask(self, l, k, colour):
        p = self.m.patches[l][k]
        z, y, x = np.meshgrid(*(p.origin[a] + np.arange(p.n[a]) for a in (2, 1, 0)), indexing="ij")
        return (((x + y + z) & 1) == colour) & self.act[l][k]

    def smooth(self, k, sweeps, lams=None, frozen_coarse=None):
        """RB-SOR (eqs. rbsor1-2) on the active cells of the patches `lams` (default: all) at
        level k; ghosts (physical and level boundary) refreshed before each colour."""
        P = self.m.patches
        lams = range(self.m.Lam + 1) if lams is None else lams
        for _ in range(sweeps):
            for colour in (0, 1):
                arrs = [self.u[l][k] for l in range(self.m.Lam + 1)]
                cgs = self.fill(k, arrs)
                new = {}
                for l in lams:
                    p = P[l][k]
                    u = interior(self.u[l][k])
                    nb = neighbour_sum(p, self.u[l][k], cgs[l])
                    upd = u + self.omega * ((nb - p.h * p.h * interior(self.f[l][k])) / 6.0 - u)
                    m = self.colour_mask(l, k, colour)
                    new[l] = np.where(m, upd, u)
                for l, v in new.items():
                    interior(self.u[l][k])[...] = v

    # ---- transfers
    @staticmethod
    def restrict(a):
        """8-cell mean (eq. restriction) of a (n)^3 interior array -> (n/2)^3."""
        s = (a[0::2, 0::2, 0::2] + a[0::2, 0::2, 1::2] + a[0::2, 1::2, 0::2] + a[0::2, 1::2, 1::2] +
             a[1::2, 0::2, 0::2] + a[1::2, 0::2, 1::2] + a[1::2, 1::2, 0::2] + a[1::2, 1::2, 1::2])
        return s / 8.0

    @staticmethod
    def prolong(c):
        """Trilinear prolongation (eq. trilinear) of a ghost-filled coarse array (nc+2)^3 to the
        (2 nc)^3 fine cells: per axis the lower child takes 1/4 c[I-1] + 3/4 c[I], the upper
        3/4 c[I] + 1/4 c[I+1]."""
        def axis_prolong(a, ax):
            lo = 0.25 * np.take(a, range(0, a.shape[ax] - 2), axis=ax) + 0.75 * np.take(a, range(1, a.shape[ax] - 1), axis=ax)
            hi = 0.75 * np.take(a, range(1, a.shape[ax] - 1), axis=ax) + 0.25 * np.take(a, range(2, a.shape[ax]), axis=ax)
            shp = list(lo.shape)
            shp[ax] *= 2
            out = np.empty(shp)
            s_lo = [slice(None)] * 3
            s_hi = [slice(None)] * 3
            s_lo[ax] = slice(0, None, 2)
            s_hi[ax] = slice(1, None, 2)
            out[tuple(s_lo)] = lo
            out[tuple(s_hi)] = hi
            return out
        a = axis_prolong(c, 2)
        a = axis_prolong(a, 1)
        a = axis_prolong(a, 0)
        return a

    def normal_fill(self, k, arrs, homogeneous=True):
        """Normal level boundary for prolongation at level k (homogeneous physical conditions):
        each finer patch is restricted into the covered cells of the coarser one (finest
        first), the root patch gets its physical ghosts, then the ghost shell of each finer
        patch (faces, edges and corners) is the trilinear prolongation of the coarser patch."""
        P = self.m.patches
        Lam = self.m.Lam
        for l in range(Lam, 0, -1):
            lo, hi = P[l - 1][k].hole
            interior(arrs[l - 1])[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = self.restrict(interior(arrs[l]))
        fill_physical(arrs[0], P[0][k], self.kinds, None if homogeneous else self.bfun, homogeneous)
        for l in range(1, Lam + 1):
            lo, hi = P[l - 1][k].hole
            # coarse region: the hole with one coarse cell around, plus one more for the stencil
            reg = arrs[l - 1][lo[2] - 1:hi[2] + 3, lo[1] - 1:hi[1] + 3, lo[0] - 1:hi[0] + 3]
            full = self.prolong(reg)              # fine cells of the hole and one coarse cell around
            # full covers fine local indices -2 .. n+1 (two fine cells each side)
            shell = full[1:-1, 1:-1, 1:-1]        # fine -1 .. n, i.e. the ghosted fine array
            g = arrs[l]
            keep = interior(g).copy()
            g[...] = shell
            interior(g)[...] = keep

    # ---- the FAS V-cycle on the refined mesh
    # ---- the root grid: a uniform hierarchy NB^3 .. 1 with the physical conditions of each
    # level (Sec. 2.3.6); level NB shares the root patch's potential array
    def root_u(self, n):
        return self.u[0][0] if n == self.m.NB else self.ru[n]

    def _root_patch(self, n):
        return Patch(0, 0, (0, 0, 0), (n, n, n), 1.0 / n)

    def root_smooth(self, n, sweeps):
        u, f, p = self.root_u(n), self.rf[n], self._root_patch(n)
        z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        for _ in range(sweeps):
            for colour in (0, 1):
                fill_physical(u, p, self.kinds, self.bfun, False)
                nb = neighbour_sum(p, u)
                c = interior(u)
                upd = c + self.omega * ((nb - p.h * p.h * interior(f)) / 6.0 - c)
                c[...] = np.where(((x + y + z) & 1) == colour, upd, c)

    def root_lap(self, u, n):
        p = self._root_patch(n)
        fill_physical(u, p, self.kinds, self.bfun, False)
        return (neighbour_sum(p, u) - 6.0 * interior(u)) / (p.h * p.h)

    def root_coarsest(self):
        """One cell (Sec. 2.3.2): ghost = alpha u + beta per face; u kept when nothing fixes it."""
        u, f = self.root_u(1), self.rf[1]
        sa, sb = 0.0, 0.0
        for face in range(6):
            if self.kinds[face] in (PERIODIC, ZERO_GRADIENT):
                sa += 1.0
            else:
                axis, side = face // 2, face % 2
                pt = [0.5, 0.5, 0.5]
                pt[axis] = 0.0 if side == 0 else 1.0
                if self.bfun is None:
                    b = 0.0
                elif isinstance(self.bfun, FaceArrays):
                    b = self.bfun.point(face)
                else:
                    b = float(self.bfun(np.array(pt[0]), np.array(pt[1]), np.array(pt[2])))
                sa -= 1.0
                sb += 2.0 * b
        if sa != 6.0:
            h = 1.0                                           # the unit cube's single cell
            u[1, 1, 1] = (sb - h * h * f[1, 1, 1]) / (6.0 - sa)

    def root_cycle(self, n):
        """Uniform FAS V-cycle (Alg. 3) from root level n with its source in rf[n]."""
        if n == 1:
            self.root_coarsest()
            return
        u, f = self.root_u(n), self.rf[n]
        self.root_smooth(n, self.npre)
        d = interior(f) - self.root_lap(u, n)
        nc = n // 2
        uc = self.root_u(nc)
        interior(uc)[...] = self.restrict(interior(u))
        pb = uc.copy()
        interior(self.rf[nc])[...] = self.restrict(d) + self.root_lap(pb, nc)
        self.root_cycle(nc)
        delta = uc - pb
        fill_physical(delta, self._root_patch(nc), self.kinds, None, True)
        interior(u)[...] += self.prolong(delta)
        self.root_smooth(n, self.npost)

    def octet_smooth(self, l, sweeps):
        """RB-SOR on every cell of the Octet patch l (k = 0), the conservative ghosts from the
        coarser patch (held fixed) refreshed before each colour."""
        P = self.m.patches
        fine, coarse = P[l][0], P[l - 1][0]
        full = Patch(l, 0, fine.origin, fine.n, fine.h, None)
        z, y, x = np.meshgrid(*(full.origin[a] + np.arange(full.n[a]) for a in (2, 1, 0)), indexing="ij")
        par = (x + y + z) & 1
        for _ in range(sweeps):
            for colour in (0, 1):
                conservative_ghosts(full, self.u[l][0], coarse, self.u[l - 1][0])
                c = interior(self.u[l][0])
                nb = neighbour_sum(full, self.u[l][0])
                upd = c + self.omega * ((nb - full.h * full.h * interior(self.f[l][0])) / 6.0 - c)
                c[...] = np.where(par == colour, upd, c)

    def vcycle(self, top=None):
        """One FAS V-cycle from `top`: ("mb", k) starts on MeshBlock level k (default: the
        finest), ("oct", lam) on Octet level lam, ("root", n) on root level n.  A cycle from
        an Octet level treats the uncovered cells of the coarser patches as part of their own
        levels: their restricted potential is the current value and their restricted defect
        their own, so their coarse source is their own source."""
        m, K, Lam = self.m, self.m.K, self.m.Lam
        P = m.patches
        all_l = range(Lam + 1)
        kind, level = top if top is not None else ("mb", K)
        if kind == "root":
            self.root_cycle(level)
            return
        kt = level if kind == "mb" else 0
        lam_top = Lam if kind == "mb" else level
        # ---- MeshBlock levels, down
        for k in range(kt, 0, -1):
            self.smooth(k, self.npre)
            d = self.defect(k)
            for l in all_l:
                pb = self.restrict(interior(self.u[l][k]) * self.act[l][k])
                interior(self.pbar[l][k - 1])[...] = pb
                interior(self.u[l][k - 1])[...] = pb
                interior(self.dres[l][k - 1])[...] = self.restrict(d[l])
            if k - 1 >= 1:
                Lc = self.laplacian(k - 1, [self.pbar[l][k - 1] for l in all_l])
                for l in all_l:
                    interior(self.f[l][k - 1])[...] = np.where(self.act[l][k - 1],
                                                               interior(self.dres[l][k - 1]) + Lc[l], 0.0)
        if kind == "oct":
            # the uncovered cells of the coarser patches belong to this Octet level's composite
            # problem: phibar = their current value, restricted defect = their defect in that
            # problem (composite operator at k = 0 over patches 0 .. lam_top, the conservative
            # ghosts from the finer patch included); covered cells are filled from the Octets
            # below as the cycle goes down
            arrs = [self.u[l][0] for l in range(Lam + 1)]
            Lc = self.laplacian_upto(0, arrs, lam_top)
            srcs = [self.rfsrc[m.NB]] + [self.fsrc[l] for l in range(1, lam_top)]
            for l in range(lam_top):
                interior(self.dres[l][0])[...] = np.where(self.act[l][0], interior(srcs[l]) - Lc[l], 0.0)
                self.pbar[l][0][...] = self.u[l][0]
        # ---- Octet levels, finest first (k = 0): smooth, then restrict into the coarser patch
        for l in range(lam_top, 0, -1):
            fine, coarse = P[l][0], P[l - 1][0]
            # the octet operator: the full patch (covered cells hold the restricted finer
            # octets) with the conservative ghosts from the coarser patch
            full = Patch(l, 0, fine.origin, fine.n, fine.h, None)
            if not (kind == "oct" and l == lam_top):
                pb = self.pbar[l][0]
                conservative_ghosts(full, pb, coarse, self.pbar[l - 1][0])
                Lp = (neighbour_sum(full, pb) - 6.0 * interior(pb)) / (full.h * full.h)
                interior(self.f[l][0])[...] = interior(self.dres[l][0]) + Lp
                interior(self.u[l][0])[...] = interior(pb)
            else:
                interior(self.f[l][0])[...] = interior(self.fsrc[l])
            self.octet_smooth(l, self.npre)
            conservative_ghosts(full, self.u[l][0], coarse, self.u[l - 1][0])
            d = interior(self.f[l][0]) - (neighbour_sum(full, self.u[l][0]) - 6.0 * interior(self.u[l][0])) / (full.h * full.h)
            lo, hi = coarse.hole
            sl = (slice(lo[2] + 1, hi[2] + 1), slice(lo[1] + 1, hi[1] + 1), slice(lo[0] + 1, hi[0] + 1))
            rp = self.restrict(interior(self.u[l][0]))
            self.pbar[l - 1][0][sl] = rp
            self.u[l - 1][0][sl] = rp
            self.dres[l - 1][0][sl] = self.restrict(d)
        # ---- root grid: uniform FAS from the restricted potential
        root = P[0][0]
        full0 = Patch(0, 0, root.origin, root.n, root.h, None)
        pb0 = self.pbar[0][0]
        fill_physical(pb0, full0, self.kinds, self.bfun, False)
        L0 = (neighbour_sum(full0, pb0) - 6.0 * interior(pb0)) / (full0.h * full0.h)
        interior(self.rf[m.NB])[...] = interior(self.dres[0][0]) + L0
        interior(self.u[0][0])[...] = interior(pb0)
        self.root_cycle(m.NB)
        # ---- Octet levels, coarsest first: prolongated correction, then post-smoothing
        for l in range(1, lam_top + 1):
            coarse = P[l - 1][0]
            delta = self.u[l - 1][0] - self.pbar[l - 1][0]
            if l - 1 == 0:
                fill_physical(delta, Patch(0, 0, coarse.origin, coarse.n, coarse.h, None), self.kinds, None, True)
            lo, hi = coarse.hole
            reg = delta[lo[2]:hi[2] + 2, lo[1]:hi[1] + 2, lo[0]:hi[0] + 2]
            interior(self.u[l][0])[...] += self.prolong(reg)
            self.octet_smooth(l, self.npost)
        # ---- MeshBlock levels, up
        for k in range(1, kt + 1):
            delta = [self.u[l][k - 1] - self.pbar[l][k - 1] for l in all_l]
            for l in all_l:
                interior(delta[l])[~self.act[l][k - 1]] = 0.0
            self.normal_fill(k - 1, delta)
            for l in all_l:
                interior(self.u[l][k])[...] += np.where(self.act[l][k], self.prolong(delta[l]), 0.0)
            self.smooth(k, self.npost)

    # ---- full multigrid (Alg. 2 with FAS in place of the V-cycle) on the refined hierarchy
    @staticmethod
    def prolong_cubic(c):
        """Tricubic FMG prolongation (Sec. 2.3.1) of a ghost-filled coarse array: per axis the
        lower child (5 c[I-1] + 30 c[I] - 3 c[I+1]) / 32, the upper (-3 c[I-1] + 30 c[I] +
        5 c[I+1]) / 32, applied x, then y, then z."""
        def axis_prolong(a, ax):
            m = np.take(a, range(0, a.shape[ax] - 2), axis=ax)
            c0 = np.take(a, range(1, a.shape[ax] - 1), axis=ax)
            p_ = np.take(a, range(2, a.shape[ax]), axis=ax)
            lo = ((5.0 / 32.0) * m + (30.0 / 32.0) * c0) + (-3.0 / 32.0) * p_
            hi = ((-3.0 / 32.0) * m + (30.0 / 32.0) * c0) + (5.0 / 32.0) * p_
            shp = list(lo.shape)
            shp[ax] *= 2
            out = np.empty(shp)
            s_lo = [slice(None)] * 3
            s_hi = [slice(None)] * 3
            s_lo[ax] = slice(0, None, 2)
            s_hi[ax] = slice(1, None, 2)
            out[tuple(s_lo)] = lo
            out[tuple(s_hi)] = hi
            return out
        a = axis_prolong(c, 2)
        a = axis_prolong(a, 1)
        return axis_prolong(a, 0)

    def fmg_sources(self):
        """Alg. 2 step 1: the source on every MeshBlock level (8-cell means per patch), on every
        Octet level (covered cells: the means of the finer Octet level) and root level."""
        m, K, Lam = self.m, self.m.K, self.m.Lam
        P = m.patches
        all_l = range(Lam + 1)
        for k in range(K, 0, -1):
            for l in all_l:
                interior(self.f[l][k - 1])[...] = self.restrict(interior(self.f[l][k]))
        self.fsrc_mb = [[f.copy() for f in fl] for fl in self.f]
        for l in all_l:
            self.fsrc[l] = self.f[l][0].copy()
        for l in range(Lam, 0, -1):
            lo, hi = P[l - 1][0].hole
            interior(self.fsrc[l - 1])[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = self.restrict(interior(self.fsrc[l]))
        n = m.NB
        self.rfsrc[n] = self.fsrc[0].copy()
        while n > 1:
            self.rfsrc[n // 2] = np.zeros((n // 2 + 2,) * 3)
            interior(self.rfsrc[n // 2])[...] = self.restrict(interior(self.rfsrc[n]))
            n //= 2

    def fmg(self):
        """Alg. 2 on the refined hierarchy: sources restricted to every level; the single root
        cell solved; then root levels 2 .. NB, Octet levels 1 .. Lam and MeshBlock levels
        1 .. K each start from the tricubic prolongation of the solution one level down
        (ghosts: physical conditions on the root patch, the normal level boundary between
        patches) and take one V-cycle from that level."""
        m, K, Lam = self.m, self.m.K, self.m.Lam
        P = m.patches
        all_l = range(Lam + 1)
        self.fmg_sources()
        # root levels
        self.rf[1][...] = self.rfsrc[1]
        self.root_u(1)[...] = 0.0
        self.root_coarsest()
        n = 2
        while n <= m.NB:
            c = self.root_u(n // 2)
            fill_physical(c, self._root_patch(n // 2), self.kinds, self.bfun, False)
            interior(self.root_u(n))[...] = self.prolong_cubic(c)
            self.rf[n][...] = self.rfsrc[n]
            self.root_cycle(n)
            n *= 2
        # Octet levels
        for l in range(1, Lam + 1):
            c = self.u[l - 1][0]
            lo, hi = P[l - 1][0].hole
            reg = c[lo[2]:hi[2] + 2, lo[1]:hi[1] + 2, lo[0]:hi[0] + 2]
            interior(self.u[l][0])[...] = self.prolong_cubic(reg)
            self.vcycle(("oct", l))
        # MeshBlock levels
        for k in range(1, K + 1):
            for l in all_l:
                interior(self.f[l][k])[...] = np.where(self.act[l][k], interior(self.fsrc_mb[l][k]), 0.0)
            self.normal_fill(k - 1, [self.u[l][k - 1] for l in all_l], homogeneous=False)
            for l in all_l:
                interior(self.u[l][k])[...] = np.where(self.act[l][k], self.prolong_cubic(self.u[l][k - 1]), 0.0)
            self.vcycle(("mb", k))

    def residual(self) -> float:
        K = self.m.K
        d = self.defect(K)
        rd = math.sqrt(self.volume_mean([x * x for x in d], K))
        return rd / self.rms_f if self.rms_f > 0 else rd

    def phi(self):
        """Potential of the active cells per patch at the finest MG level (covered cells 0); the
        volume mean is removed when no face fixes the zero point."""
        K = self.m.K
        out = [np.where(self.act[l][K], interior(self.u[l][K]), 0.0) for l in range(self.m.Lam + 1)]
        if self.gauge_free:
            mean = self.volume_mean(out, K)
            out = [np.where(self.act[l][K], o - mean, 0.0) for l, o in enumerate(out)]
        return out

    def set_phi(self, phi):
        K = self.m.K
        for l in range(self.m.Lam + 1):
            interior(self.u[l][K])[...] = np.where(self.act[l][K], phi[l], 0.0)


def solve(mesh: AmrMesh, rho, kinds, bfun=None, phi0=None, cycles=None, tol=1e-10, max_cycles=60, mode="mgi",
          **kw):
    """FMG (mode "fmg") or V-cycles from phi0 (zero by default), then V-cycles until the
    relative composite residual is <= tol (or `cycles` exactly).  Returns (phi per patch,
    residual history)."""
    st = AmrState(mesh, rho, kinds, bfun, **kw)
    if mode == "fmg":
        st.fmg()
    elif phi0 is not None:
        st.set_phi(phi0)
    hist = [st.residual()]
    n = cycles if cycles is not None else max_cycles
    for _ in range(n):
        if cycles is None and hist[-1] <= tol:
            break
        st.vcycle()
        hist.append(st.residual())
    return st.phi(), hist


def composite_laplacian(mesh: AmrMesh, phi, kinds, bfun=None):
    """L_h phi on the composite grid (active cells of every patch at the finest level)."""
    st = AmrState(mesh, [np.zeros(mesh.patches[l][mesh.K].n[::-1]) for l in range(mesh.Lam + 1)], kinds, bfun)
    arrs = []
    for l in range(mesh.Lam + 1):
        a = np.zeros(mesh.patches[l][mesh.K].shape())
        interior(a)[...] = phi[l]
        arrs.append(a)
    L = st.laplacian(mesh.K, arrs)
    return [np.where(st.act[l][mesh.K], L[l], 0.0) for l in range(mesh.Lam + 1)]
