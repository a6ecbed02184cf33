"""CPU oracle for the uniform-grid FMG / V-cycle multigrid Poisson solver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package.  It shares no code with the HIP
path and never imports it.

Two layers (the method is an iteration, so both are needed):

* ``oracle.exact``   -- the *result definition*: the exact discrete solution
  phi*_h = L_h^-1 f_h computed without multigrid (FFT / DST-II / DCT-II per axis, or a
  dense direct solve on small grids), plus closed forms.
* this module        -- the *iteration definition*: a ctypes binding to the plain C
  FP64 implementation in ``mg_oracle.c`` of Algorithms 1 and 2 of the paper
  (V-cycle correction scheme and full multigrid) with the RB-SOR smoother.

Face order everywhere: -x, +x, -y, +y, -z, +z.  Face kinds: ``PERIODIC``,
``ZERO_GRADIENT``, ``FIXED``, ``MULTIPOLE``.  Arrays are float64, C-ordered [z][y][x].
Extended face arrays are ((n+2), (n+2)) indexed [t2+1][t1+1] over the two transverse
axes in increasing axis order.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

PERIODIC, ZERO_GRADIENT, FIXED, MULTIPOLE = 0, 1, 2, 3
KIND_NAMES = {"periodic": PERIODIC, "zero_gradient": ZERO_GRADIENT, "fixed": FIXED, "multipole": MULTIPOLE}
OK, NOT_CONVERGED, STALLED = 0, 1, 2
ERR_INVALID, ERR_NONFINITE = -1, -5
FOUR_PI_G = 4.0 * math.pi        # G = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp = ctypes.c_void_p
    lib.oracle_solve.restype = ctypes.c_int
    lib.oracle_solve.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _ip,
                                 ctypes.POINTER(_dp), ctypes.c_int, ctypes.c_int, _dp,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp, _dp, _ip]
    lib.oracle_set_scheme.argtypes = [vp, ctypes.c_int]
    lib.oracle_set_coarse_rule.argtypes = [vp, ctypes.c_int]
    lib.oracle_state_create.restype = vp
    lib.oracle_state_create.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _ip,
                                        ctypes.POINTER(_dp), ctypes.c_int, ctypes.c_int, _dp,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_double, _ip]
    lib.oracle_state_destroy.argtypes = [vp]
    lib.oracle_fmg.argtypes = [vp]
    lib.oracle_vcycle.argtypes = [vp]
    lib.oracle_vcycle.restype = ctypes.c_double
    lib.oracle_residual.argtypes = [vp]
    lib.oracle_residual.restype = ctypes.c_double
    lib.oracle_set_phi.argtypes = [vp, _dp]
    lib.oracle_get_phi.argtypes = [vp, _dp]
    lib.oracle_get_origin_moments.argtypes = [vp, _dp, _dp]
    lib.oracle_state_levels.argtypes = [vp]
    lib.oracle_state_levels.restype = ctypes.c_int
    lib.oracle_state_face.argtypes = [vp, ctypes.c_int, ctypes.c_int, _dp]
    lib.oracle_state_source.argtypes = [vp, ctypes.c_int, _dp]
    lib.oracle_op_fill.argtypes = [ctypes.c_int, _dp, _ip, ctypes.POINTER(_dp), _dp]
    lib.oracle_op_half_sweep.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                         _dp, _dp, _ip, ctypes.POINTER(_dp)]
    lib.oracle_op_defect.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _ip, ctypes.POINTER(_dp)]
    lib.oracle_op_restrict.argtypes = [ctypes.c_int, _dp, _dp]
    lib.oracle_op_prolong.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, _ip, ctypes.POINTER(_dp)]
    lib.oracle_op_coarsest.argtypes = [ctypes.c_double, _dp, _dp, _ip, ctypes.POINTER(_dp)]
    lib.oracle_multipole_moments.argtypes = [ctypes.c_int, ctypes.c_double, _dp, ctypes.c_int, ctypes.c_int,
                                             _dp, _dp, _dp]
    lib.oracle_multipole_potential.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp,
                                               ctypes.c_int, _dp, ctypes.c_double]
    lib.oracle_multipole_potential.restype = ctypes.c_double
    lib.oracle_multipole_moments_points.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int,
                                                    _dp, _dp, _dp]
    lib.oracle_multipole_potential_points.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_int, _dp,
                                                      ctypes.c_double, _dp]
    lib.oracle_gravity.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _ip, ctypes.POINTER(_dp), _dp, _dp,
                                   _dp]
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _kinds(kinds) -> np.ndarray:
    if isinstance(kinds, (str, int)):
        kinds = [kinds] * 6
    out = [KIND_NAMES[k] if isinstance(k, str) else int(k) for k in kinds]
    assert len(out) == 6
    return np.asarray(out, dtype=np.int32)


def _face_ptrs(faces, keep):
    arr = (_dp * 6)()
    for f in range(6):
        b = None if faces is None else faces[f]
        if b is None:
            arr[f] = _dp()
        else:
            b = _f64(b)
            keep.append(b)
            arr[f] = _ptr(b)
    return arr


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_threads(t: int) -> None:
    _load().oracle_set_threads(int(t))


# ------------------------------------------------------------------ whole solve

def solve(rho, dx, kinds, fixed_b=None, lmax=4, origin=None, npre=2, npost=2, omega=1.15,
          mode="fmg", phi0=None, tol=1e-10, max_cycles=50, fixed_cycles=0, four_pi_g=FOUR_PI_G,
          scheme="cs"):
    """Oracle solve of nabla^2 phi = 4 pi G rho (eq. poisson).

    ``fixed_b``: six (n, n) face-centre arrays (or None) for FIXED faces.
    ``scheme``: "cs" (correction scheme, Alg. 1) or "fas" (Alg. 3) for the iterations.
    Returns ``(phi, hist, status)``.
    """
    lib = _load()
    rho = _f64(rho)
    n = rho.shape[0]
    k = _kinds(kinds)
    keep = []
    bp = _face_ptrs(fixed_b, keep)
    org = _f64(origin if origin is not None else np.zeros(3))
    phi = np.zeros_like(rho) if phi0 is None else _f64(phi0).copy()
    cap = max(max_cycles, fixed_cycles) + 2
    hist = np.zeros(cap, dtype=np.float64)
    nh = ctypes.c_int(0)
    st = lib.oracle_solve(n, float(dx), float(four_pi_g), _ptr(rho), k.ctypes.data_as(_ip), bp,
                          int(lmax), int(origin is not None), _ptr(org), int(npre), int(npost),
                          float(omega), 0 if mode == "fmg" else 1, 1 if scheme == "fas" else 0,
                          float(tol), int(max_cycles),
                          int(fixed_cycles), _ptr(phi), _ptr(hist), ctypes.byref(nh))
    return phi, hist[: nh.value].copy(), st


class State:
    """Step-by-step access to the oracle iteration (set-up, FMG, single V-cycles)."""

    def __init__(self, rho, dx, kinds, fixed_b=None, lmax=4, origin=None, npre=2, npost=2,
                 omega=1.15, four_pi_g=FOUR_PI_G, scheme="cs"):
        self._lib = _load()
        self.rho = _f64(rho)
        self.n = self.rho.shape[0]
        k = _kinds(kinds)
        self._keep = []
        bp = _face_ptrs(fixed_b, self._keep)
        org = _f64(origin if origin is not None else np.zeros(3))
        err = ctypes.c_int(0)
        self._s = self._lib.oracle_state_create(self.n, float(dx), float(four_pi_g), _ptr(self.rho),
                                                k.ctypes.data_as(_ip), bp, int(lmax),
                                                int(origin is not None), _ptr(org), int(npre),
                                                int(npost), float(omega), ctypes.byref(err))
        if not self._s:
            raise ValueError(f"oracle set-up failed with status {err.value}")
        self._lib.oracle_set_scheme(self._s, 1 if scheme == "fas" else 0)

    def __del__(self):
        if getattr(self, "_s", None):
            self._lib.oracle_state_destroy(self._s)
            self._s = None

    def set_coarse_rule(self, rule: str):
        """Conditions of the coarse-level corrections: "homogeneous" (the default: each face's
        homogeneous counterpart) or "literal" (Sec. 2.3.6 word for word: zero-fixed unless
        periodic)."""
        if rule not in ("homogeneous", "literal"):
            raise ValueError(rule)
        self._lib.oracle_set_coarse_rule(self._s, 1 if rule == "literal" else 0)

    def fmg(self):
        self._lib.oracle_fmg(self._s)

    def vcycle(self) -> float:
        return self._lib.oracle_vcycle(self._s)

    def residual(self) -> float:
        return self._lib.oracle_residual(self._s)

    def set_phi(self, phi):
        phi = _f64(phi)
        self._lib.oracle_set_phi(self._s, _ptr(phi))

    def phi(self):
        out = np.empty((self.n,) * 3, dtype=np.float64)
        self._lib.oracle_get_phi(self._s, _ptr(out))
        return out

    def levels(self) -> int:
        return self._lib.oracle_state_levels(self._s)

    def face(self, level, face):
        nl = 1 << level
        out = np.empty((nl + 2, nl + 2), dtype=np.float64)
        self._lib.oracle_state_face(self._s, level, face, _ptr(out))
        return out

    def source(self, level):
        nl = 1 << level
        out = np.empty((nl,) * 3, dtype=np.float64)
        self._lib.oracle_state_source(self._s, level, _ptr(out))
        return out

    def origin_moments(self):
        o = np.zeros(3)
        q = np.zeros(25)
        self._lib.oracle_get_origin_moments(self._s, _ptr(o), _ptr(q))
        return o, q


# ------------------------------------------------------------ single operators

def fill(u, kinds, bext=None):
    """Ghost-filled copy ((n+2)^3) of u under the given boundary description."""
    lib = _load()
    u = _f64(u)
    n = u.shape[0]
    out = np.zeros((n + 2,) * 3, dtype=np.float64)
    keep = []
    lib.oracle_op_fill(n, _ptr(u), _kinds(kinds).ctypes.data_as(_ip), _face_ptrs(bext, keep), _ptr(out))
    return out


def half_sweep(u, f, h, omega, colour, kinds, bext=None):
    """One colour (0 red, 1 black) of the RB-SOR smoother (eqs. rbsor1-2); returns new u."""
    lib = _load()
    u = _f64(u).copy()
    f = _f64(f)
    keep = []
    lib.oracle_op_half_sweep(u.shape[0], float(h), float(omega), int(colour), _ptr(u), _ptr(f),
                             _kinds(kinds).ctypes.data_as(_ip), _face_ptrs(bext, keep))
    return u


def smooth(u, f, h, omega, kinds, bext=None):
    u = half_sweep(u, f, h, omega, 0, kinds, bext)
    return half_sweep(u, f, h, omega, 1, kinds, bext)


def defect(u, f, h, kinds, bext=None):
    """d = f - L_h u (eq. defect)."""
    lib = _load()
    u = _f64(u)
    f = _f64(f)
    d = np.zeros_like(u)
    keep = []
    lib.oracle_op_defect(u.shape[0], float(h), _ptr(u), _ptr(f), _ptr(d),
                         _kinds(kinds).ctypes.data_as(_ip), _face_ptrs(bext, keep))
    return d


def restrict(uf):
    """8-cell volume-weighted restriction (eq. restriction)."""
    lib = _load()
    uf = _f64(uf)
    nc = uf.shape[0] // 2
    uc = np.zeros((nc,) * 3, dtype=np.float64)
    lib.oracle_op_restrict(nc, _ptr(uf), _ptr(uc))
    return uc


def prolong_add(uc, uf, kinds, bext=None):
    """uf + trilinear(uc) (eq. trilinear); ghosts of uc from the boundary description."""
    lib = _load()
    uc = _f64(uc)
    out = _f64(uf).copy()
    keep = []
    lib.oracle_op_prolong(uc.shape[0], _ptr(uc), _ptr(out), 0, _kinds(kinds).ctypes.data_as(_ip),
                          _face_ptrs(bext, keep))
    return out


def prolong_fmg(uc, kinds, bext=None):
    """tricubic FMG prolongation of uc (Sec. 2.3.1)."""
    lib = _load()
    uc = _f64(uc)
    nc = uc.shape[0]
    out = np.zeros((2 * nc,) * 3, dtype=np.float64)
    keep = []
    lib.oracle_op_prolong(nc, _ptr(uc), _ptr(out), 1, _kinds(kinds).ctypes.data_as(_ip),
                          _face_ptrs(bext, keep))
    return out


def coarsest(h, f, kinds, bext=None):
    """Exact one-cell solve (Sec. 2.3.2); f is a scalar; bext are 3x3 extended arrays."""
    lib = _load()
    u = np.zeros(1)
    ff = np.asarray([float(f)])
    keep = []
    lib.oracle_op_coarsest(float(h), _ptr(u), _ptr(ff), _kinds(kinds).ctypes.data_as(_ip),
                           _face_ptrs(bext, keep))
    return float(u[0])


def gravity(phi, h, kinds, bext=None, rho=None, faces=False):
    """g = -grad phi in the cell-centred scheme of Sec. 2.4 (eq. acceleration): returns
    g (3, n, n, n); with rho also rho*g (3, n, n, n); with faces=True also the face values
    (gx (n, n, n+1), gy (n, n+1, n), gz (n+1, n, n)), each indexed [k][j][i]."""
    lib = _load()
    phi = _f64(phi)
    n = phi.shape[0]
    g = np.zeros((3, n, n, n))
    rg = np.zeros((3, n, n, n)) if rho is not None else None
    gf = np.zeros(3 * n * n * (n + 1)) if faces else None
    rho_a = _f64(rho) if rho is not None else None
    keep = []
    lib.oracle_gravity(n, float(h), _ptr(phi), _ptr(rho_a) if rho_a is not None else None,
                       _kinds(kinds).ctypes.data_as(_ip), _face_ptrs(bext, keep), _ptr(g),
                       _ptr(rg) if rg is not None else None, _ptr(gf) if gf is not None else None)
    out = [g]
    if rho is not None:
        out.append(rg)
    if faces:
        m = n * n * (n + 1)
        out.append((gf[:m].reshape(n, n, n + 1), gf[m:2 * m].reshape(n, n + 1, n), gf[2 * m:].reshape(n + 1, n, n)))
    return out[0] if len(out) == 1 else tuple(out)


def multipole_moments(rho, dx, lmax=4, origin=None):
    """Origin (centre of mass unless given) and the 25 moments Q_lm (Appendix A)."""
    lib = _load()
    rho = _f64(rho)
    org = _f64(origin if origin is not None else np.zeros(3))
    out_o = np.zeros(3)
    q = np.zeros(25)
    lib.oracle_multipole_moments(rho.shape[0], float(dx), _ptr(rho), int(lmax), int(origin is not None),
                                 _ptr(org), _ptr(out_o), _ptr(q))
    return out_o, q


def multipole_potential(x, y, z, q, origin, lmax=4, G=1.0):
    lib = _load()
    q = _f64(q)
    o = _f64(origin)
    return lib.oracle_multipole_potential(float(x), float(y), float(z), _ptr(q), int(lmax), _ptr(o), float(G))


def multipole_moments_points(x, y, z, mass, lmax=4, origin=None):
    """Origin (centre of mass of the points unless given, 0.5 each for zero mass) and the 25
    moments Q_lm of point masses (Appendix A summed over cells given as points)."""
    lib = _load()
    x, y, z, mass = (_f64(np.ravel(a)) for a in (x, y, z, mass))
    org = _f64(origin if origin is not None else np.zeros(3))
    out_o = np.zeros(3)
    q = np.zeros(25)
    lib.oracle_multipole_moments_points(x.size, _ptr(x), _ptr(y), _ptr(z), _ptr(mass), int(lmax),
                                        int(origin is not None), _ptr(org), _ptr(out_o), _ptr(q))
    return out_o, q


def multipole_potential_points(x, y, z, q, origin, lmax=4, G=1.0):
    """The truncated expansion (Appendix A) at arrays of points; returns an array of their shape."""
    lib = _load()
    shape = np.shape(x)
    x, y, z = (_f64(np.ravel(a)) for a in np.broadcast_arrays(x, y, z))
    q, o = _f64(q), _f64(origin)
    out = np.zeros(x.size)
    lib.oracle_multipole_potential_points(x.size, _ptr(x), _ptr(y), _ptr(z), _ptr(q), int(lmax), _ptr(o),
                                          float(G), _ptr(out))
    return out.reshape(shape)


def extend_face(b):
    """(n, n) face-centre array -> ((n+2), (n+2)) with the ring copying the nearest value."""
    b = _f64(b)
    return np.pad(b, 1, mode="edge")
