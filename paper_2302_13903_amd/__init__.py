"""MI355X-native geometric multigrid Poisson solver (Tomida & Stone, arXiv:2302.13903).

Thin Python binding of the C ABI in ``include/mg355.h``: every step of a solve runs in the
HIP kernels of ``libmg355.so``; this module only marshals torch device tensors (memory and
streams) into the C calls, under the same names.  There is no CPU fallback: without the
built library every entry point raises.

Quick use::

    import torch, paper_2302_13903_amd as mg
    phi, hist, status = mg.solve(rho_cuda_f64, dx=1/256, bc="periodic", tol=1e-10)
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field
from typing import Optional, Sequence

from . import _abi
from ._abi import (MG_BC_FIXED, MG_BC_MULTIPOLE, MG_BC_PERIODIC, MG_BC_ZERO_GRADIENT, MG_LAYOUT_BLOCKS,
                   MG_LAYOUT_DENSE, MG_MODE_FMG, MG_MODE_MGI, MG_PREC_FP64, MG_PREC_MIXED, MG_NOT_CONVERGED,
                   MG_OK, MG_STALLED, MgError, STATUS_NAMES)

__all__ = ["Context", "solve", "to_blocks", "from_blocks", "morton_order", "mg_solve", "mg_solve_noalloc", "mg_footprint_bytes", "params", "boundary", "level_bc",
           "mg_solve_simple", "mg_op_fill", "mg_op_half_sweep", "mg_op_smooth", "mg_op_defect", "mg_op_restrict", "mg_op_prolong_add",
           "mg_op_prolong_fmg", "mg_op_coarsest", "mg_op_down", "mg_op_up", "mg_op_smooth_f32", "mg_op_down_f32",
           "mg_op_up_f32", "mg_op_sweep_input_norm", "mg_op_mixed_update", "mg_multipole_moments",
           "gravity", "mg_gravity", "mg_gravity_kernel_name", "amr_mesh", "amr_patch_dims", "amr_solve",
           "mg_amr_solve", "MgError", "KINDS"]

KINDS = {"periodic": MG_BC_PERIODIC, "zero_gradient": MG_BC_ZERO_GRADIENT, "fixed": MG_BC_FIXED,
         "multipole": MG_BC_MULTIPOLE}


def _kinds(k) -> list:
    if isinstance(k, (str, int)):
        k = [k] * 6
    out = [KINDS[x] if isinstance(x, str) else int(x) for x in k]
    if len(out) != 6:
        raise ValueError("six face kinds expected (-x,+x,-y,+y,-z,+z)")
    return out


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("device tensors must be contiguous CUDA/HIP tensors")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Context:
    """Owns an ``mg_ctx`` (pooled device workspace, reused across solves)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        """``hbm_budget``: device bytes the context may hold (0 = no cap); a solve that would
        need more fails with MG_ERR_OOM instead of allocating."""
        self._lib = _abi.lib()
        h = ctypes.c_void_p()
        st = self._lib.mg_ctx_create(ctypes.byref(h), int(device), int(hbm_budget))
        if st != MG_OK:
            raise MgError(f"mg_ctx_create failed: {STATUS_NAMES.get(st, st)}")
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            self._lib.mg_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return self._lib.mg_last_error(self.handle).decode()

    def check(self, st: int, what: str) -> int:
        if st < 0:
            raise MgError(f"{what}: {STATUS_NAMES.get(st, st)}: {self.last_error()}")
        return st

    def last_timing(self, cap: int = 1024):
        setup, fmg = ctypes.c_double(), ctypes.c_double()
        cyc = (ctypes.c_double * cap)()
        n = ctypes.c_int()
        self._lib.mg_last_timing(self.handle, ctypes.byref(setup), ctypes.byref(fmg), cyc, cap, ctypes.byref(n))
        return setup.value, fmg.value, [cyc[i] for i in range(min(n.value, cap))]

    def last_inner(self) -> int:
        """FP32 V-cycles of the last mixed-precision solve (see mg_last_inner)."""
        k = ctypes.c_int()
        self.check(self._lib.mg_last_inner(self.handle, ctypes.byref(k)), "mg_last_inner")
        return k.value

    def set_kernel_timing(self, on: bool):
        self._lib.mg_set_kernel_timing(self.handle, 1 if on else 0)

    def kernel_timing(self):
        """Per-kernel records of the last solve's finest-level passes (see mg_kernel_timing)."""
        out = []
        idx = 0
        while True:
            n, ms, by = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
            name = ctypes.create_string_buffer(256)
            st = self._lib.mg_kernel_timing(self.handle, idx, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by),
                                            name, 256)
            if st != MG_OK:
                return out
            out.append({"launches": n.value, "total_ms": ms.value, "bytes_per_launch": by.value,
                        "name": name.value.decode()})
            idx += 1


    def reserve(self, n: int, precision: str = "fp64", layout: str = "dense", block_n: int = 16):
        p = params(n, 1.0 / n, precision=precision, layout=layout, block_n=block_n)
        self.check(self._lib.mg_ctx_reserve(self.handle, ctypes.byref(p)), "mg_ctx_reserve")

    def autotune(self, n: int, block_n: int = 16, precision: str = "fp64", reps: int = 5,
                 cache: Optional[str] = None, layout: str = "blocks") -> str:
        """Pick the schedules of solves of this shape (see mg_autotune): block-sweep shapes for
        the MeshBlock layout, defect/norm pass fusion for the dense layout.  With ``cache`` (a
        JSON file) a stored result for this device and shape is loaded instead of timing, and
        a new result is stored.  Returns the context's schedule text."""
        import json
        import os
        key = None
        if cache:
            import torch
            key = f"{torch.cuda.get_device_name(self.device)}|n={n}|{layout}|block_n={block_n}|{precision}"
            try:
                with open(cache) as fh:
                    stored = json.load(fh)
            except (OSError, ValueError):
                stored = {}
            if key in stored:
                self.set_tuning(stored[key])
                return stored[key]
        p = params(n, 1.0 / n, precision=precision, layout=layout, block_n=block_n)
        self.check(self._lib.mg_autotune(self.handle, ctypes.byref(p), int(reps)), "mg_autotune")
        text = self.tuning()
        if cache:
            stored[key] = text
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            with open(cache, "w") as fh:
                json.dump(stored, fh, indent=1)
        return text

    def tuning(self) -> str:
        need = self._lib.mg_tuning_get(self.handle, None, 0)
        buf = ctypes.create_string_buffer(max(need, 1))
        self._lib.mg_tuning_get(self.handle, buf, len(buf))
        return buf.value.decode()

    def set_tuning(self, text: str):
        self.check(self._lib.mg_tuning_set(self.handle, text.encode()), "mg_tuning_set")


def morton_order(nb: int):
    """Row-major (bz, by, bx) block numbers listed in Morton order (x bit lowest): element q is
    the row-major number of the block stored q-th in the MeshBlock layout."""
    import numpy as np
    lb = max(nb - 1, 0).bit_length()
    q = np.arange(nb ** 3, dtype=np.int64)
    c = [np.zeros_like(q) for _ in range(3)]
    for bit in range(lb):
        for a in range(3):
            c[a] |= ((q >> (3 * bit + a)) & 1) << bit
    bx, by, bz = c
    return (bz * nb + by) * nb + bx


def to_blocks(x, block_n: int):
    """Dense (n, n, n) [z][y][x] tensor -> MeshBlock layout (flat, blocks in Morton order)."""
    import torch
    n, m = x.shape[0], block_n
    nb = n // m
    b = x.reshape(nb, m, nb, m, nb, m).permute(0, 2, 4, 1, 3, 5).reshape(nb ** 3, m ** 3)
    idx = torch.as_tensor(morton_order(nb), device=x.device)
    return b.index_select(0, idx).reshape(-1).contiguous()


def from_blocks(xb, n: int, block_n: int):
    """Inverse of to_blocks."""
    import torch
    m = block_n
    nb = n // m
    idx = torch.as_tensor(morton_order(nb), device=xb.device)
    rows = torch.empty((nb ** 3, m ** 3), dtype=xb.dtype, device=xb.device)
    rows[idx] = xb.reshape(nb ** 3, m ** 3)
    return rows.reshape(nb, nb, nb, m, m, m).permute(0, 3, 1, 4, 2, 5).reshape(n, n, n).contiguous()


_default_ctx = {}


def default_context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def params(n: int, dx: float, **kw) -> _abi.MgParams:
    p = _abi.MgParams()
    _abi.lib().mg_default_params(ctypes.byref(p))
    p.n = int(n)
    p.dx = float(dx)
    for k, v in kw.items():
        if k == "mode" and isinstance(v, str):
            v = {"fmg": MG_MODE_FMG, "mgi": MG_MODE_MGI}[v]
        if k == "precision" and isinstance(v, str):
            v = {"fp64": MG_PREC_FP64, "mixed": MG_PREC_MIXED}[v]
        if k == "layout" and isinstance(v, str):
            v = {"dense": MG_LAYOUT_DENSE, "blocks": MG_LAYOUT_BLOCKS}[v]
        if k == "scheme" and isinstance(v, str):
            v = {"cs": _abi.MG_SCHEME_CS, "fas": _abi.MG_SCHEME_FAS}[v]
        setattr(p, k, v)
    return p


def boundary(kinds, fixed_b: Optional[Sequence] = None, lmax: int = 4, origin=None) -> _abi.MgBC:
    b = _abi.MgBC()
    for f, k in enumerate(_kinds(kinds)):
        b.kind[f] = k
        b.fixed_b[f] = _ptr(fixed_b[f]) if fixed_b is not None and fixed_b[f] is not None else None
    b.lmax = int(lmax)
    b.use_origin = 0 if origin is None else 1
    if origin is not None:
        for a in range(3):
            b.origin[a] = float(origin[a])
    return b


def level_bc(kinds, bext: Optional[Sequence] = None) -> _abi.MgLevelBC:
    b = _abi.MgLevelBC()
    for f, k in enumerate(_kinds(kinds)):
        b.kind[f] = k
        b.b[f] = _ptr(bext[f]) if bext is not None and bext[f] is not None else None
    return b


def mg_footprint_bytes(p: _abi.MgParams) -> int:
    return int(_abi.lib().mg_footprint_bytes(ctypes.byref(p)))


def mg_solve(ctx: Context, p: _abi.MgParams, bc: _abi.MgBC, rho, phi, stream=None):
    """Raw ``mg_solve``: returns (status, hist list)."""
    cap = max(p.max_cycles, p.fixed_cycles) + 1
    hist = (ctypes.c_double * cap)()
    nh = ctypes.c_int(0)
    st = ctx._lib.mg_solve(ctx.handle, ctypes.byref(p), ctypes.byref(bc), _ptr(rho), _ptr(phi), hist,
                           ctypes.byref(nh), _stream(stream))
    ctx.check(st, "mg_solve")
    return st, [hist[i] for i in range(nh.value)]


def mg_solve_noalloc(ctx: Context, p: _abi.MgParams, bc: _abi.MgBC, rho, phi, stream=None):
    """Raw ``mg_solve_noalloc`` (the solve in the library's static scratch, no allocation):
    returns (status, hist list)."""
    cap = max(p.max_cycles, p.fixed_cycles) + 1
    hist = (ctypes.c_double * cap)()
    nh = ctypes.c_int(0)
    st = ctx._lib.mg_solve_noalloc(ctx.handle, ctypes.byref(p), ctypes.byref(bc), _ptr(rho), _ptr(phi), hist,
                                   ctypes.byref(nh), _stream(stream))
    ctx.check(st, "mg_solve_noalloc")
    return st, [hist[i] for i in range(nh.value)]


def solve(rho, dx: float, bc="periodic", fixed_b=None, lmax: int = 4, origin=None, tol: float = 1e-10,
          max_cycles: int = 50, fixed_cycles: int = 0, npre: int = 2, npost: int = 2, omega: float = 1.15,
          mode: str = "fmg", precision: str = "fp64", layout: str = "dense", block_n: int = 16, phi=None,
          four_pi_g: float = 4.0 * math.pi, scheme: str = "cs", ctx: Optional[Context] = None, stream=None):
    """Solve nabla^2 phi = 4 pi G rho on the device.  ``rho``: contiguous float64 (n, n, n) tensor
    on the GPU.  ``scheme``: "cs" (correction-scheme V-cycles) or "fas" (Full Approximation
    Scheme).  Returns ``(phi, hist, status)``."""
    import torch
    if layout == "blocks":
        # MeshBlock layout: rho is flat (n^3,) in Morton block order (see to_blocks)
        if rho.dtype != torch.float64 or rho.dim() != 1:
            raise ValueError("rho must be a flat float64 tensor in the MeshBlock layout")
        n = round(rho.numel() ** (1.0 / 3.0))
        if n ** 3 != rho.numel():
            raise ValueError("rho must hold n^3 values")
    else:
        if rho.dtype != torch.float64 or rho.dim() != 3:
            raise ValueError("rho must be a float64 (n, n, n) tensor")
        n = rho.shape[0]
    ctx = ctx or default_context(rho.device.index or 0)
    p = params(n, dx, tol=tol, max_cycles=max_cycles, fixed_cycles=fixed_cycles, npre=npre, npost=npost,
               omega=omega, mode=mode, precision=precision, layout=layout, block_n=block_n, four_pi_g=four_pi_g,
               scheme=scheme)
    b = boundary(bc, fixed_b, lmax, origin)
    if phi is None:
        phi = torch.zeros_like(rho)
    st, hist = mg_solve(ctx, p, b, rho, phi, stream)
    return phi, hist, st


def mg_gravity(ctx: Context, p: _abi.MgParams, bc: _abi.MgBC, phi, rho=None, g=None, rhog=None, gface=None,
               stream=None) -> int:
    """Raw ``mg_gravity``: writes the given outputs, asynchronously on the stream."""
    st = ctx._lib.mg_gravity(ctx.handle, ctypes.byref(p), ctypes.byref(bc), _ptr(phi), _ptr(rho), _ptr(g),
                             _ptr(rhog), _ptr(gface), _stream(stream))
    return ctx.check(st, "mg_gravity")


def mg_gravity_kernel_name(p: _abi.MgParams, g=True, rhog=False, gface=False) -> str:
    buf = ctypes.create_string_buffer(256)
    _abi.lib().mg_gravity_kernel_name(ctypes.byref(p), int(g), int(rhog), int(gface), buf, 256)
    return buf.value.decode()


def gravity(phi, dx: float, bc="periodic", rho=None, fixed_b=None, lmax: int = 4, origin=None,
            want_g: bool = True, want_rhog: bool = False, want_faces: bool = False, layout: str = "dense",
            block_n: int = 16, four_pi_g: float = 4.0 * math.pi, ctx: Optional[Context] = None, stream=None):
    """Gravitational acceleration g = -grad phi of a solved potential (cell-centred scheme of
    the paper's Sec. 2.4).  Returns a dict with "g" (3, n, n, n) [or (3, n^3) in the MeshBlock
    layout], "rhog" like g, and "faces" = (gx (n, n, n+1), gy (n, n+1, n), gz (n+1, n, n))
    for the outputs asked for."""
    import torch
    if phi.dtype != torch.float64:
        raise ValueError("phi must be float64")
    n = phi.shape[0] if layout == "dense" else round(phi.numel() ** (1.0 / 3.0))
    ctx = ctx or default_context(phi.device.index or 0)
    p = params(n, dx, layout=layout, block_n=block_n, four_pi_g=four_pi_g)
    b = boundary(bc, fixed_b, lmax, origin)
    shape = (3, n, n, n) if layout == "dense" else (3, n ** 3)
    out = {}
    g = torch.empty(shape, dtype=torch.float64, device=phi.device) if want_g else None
    rg = torch.empty(shape, dtype=torch.float64, device=phi.device) if want_rhog else None
    gf = torch.empty(3 * n * n * (n + 1), dtype=torch.float64, device=phi.device) if want_faces else None
    mg_gravity(ctx, p, b, phi, rho, g, rg, gf, stream)
    if want_g:
        out["g"] = g
    if want_rhog:
        out["rhog"] = rg
    if want_faces:
        m = n * n * (n + 1)
        out["faces"] = (gf[:m].view(n, n, n + 1), gf[m:2 * m].view(n, n + 1, n), gf[2 * m:].view(n + 1, n, n))
    return out


# ------------------------------------------------------------------ refined mesh

def amr_mesh(NB: int, nb: int, boxes) -> _abi.MgAmrMesh:
    """Refined-mesh description: NB^3 root blocks of nb^3 cells; boxes[lam-1] = ((lo), (hi)) of
    refinement level lam in level-(lam-1) block units, (x, y, z)."""
    m = _abi.MgAmrMesh()
    m.NB, m.nb, m.levels = int(NB), int(nb), len(boxes)
    for q, (lo, hi) in enumerate(boxes):
        for a in range(3):
            m.box_lo[q][a] = int(lo[a])
            m.box_hi[q][a] = int(hi[a])
    return m


def amr_patch_dims(mesh: _abi.MgAmrMesh, lam: int):
    """(nx, ny, nz) of patch lam at the finest level."""
    d = (ctypes.c_int * 3)()
    st = _abi.lib().mg_amr_patch_dims(ctypes.byref(mesh), int(lam), d)
    if st < 0:
        raise MgError(f"mg_amr_patch_dims: {STATUS_NAMES.get(st, st)}")
    return tuple(d)


def mg_amr_solve(ctx: Context, p: _abi.MgParams, mesh: _abi.MgAmrMesh, bc: _abi.MgBC, rho, phi, stream=None):
    """Raw ``mg_amr_solve``: rho and phi are lists of device tensors (one per patch, shape
    (nz, ny, nx)); returns (status, hist list)."""
    n = mesh.levels + 1
    rp = (_abi._vp * n)(*[_ptr(r) for r in rho])
    pp = (_abi._vp * n)(*[_ptr(q) for q in phi])
    cap = max(p.max_cycles, p.fixed_cycles) + 1
    hist = (ctypes.c_double * cap)()
    nh = ctypes.c_int(0)
    st = ctx._lib.mg_amr_solve(ctx.handle, ctypes.byref(p), ctypes.byref(mesh), ctypes.byref(bc), rp, pp, hist,
                               ctypes.byref(nh), _stream(stream))
    ctx.check(st, "mg_amr_solve")
    return st, [hist[i] for i in range(nh.value)]


def amr_solve(mesh: _abi.MgAmrMesh, rho, bc="periodic", fixed_b=None, phi=None, tol: float = 1e-10,
              max_cycles: int = 50, fixed_cycles: int = 0, npre: int = 2, npost: int = 2, omega: float = 1.15,
              mode: str = "mgi", four_pi_g: float = 4.0 * math.pi, lmax: int = 4, origin=None,
              ctx: Optional[Context] = None, stream=None):
    """Solve on a statically refined mesh: FMG (mode "fmg") or V-cycles from phi (zero by
    default).  rho: list of float64 device tensors, one per patch (shape (nz, ny, nx) from
    amr_patch_dims).  Multipole faces expand the composite density about its centre of mass
    (or `origin`) up to lmax.  Returns (phi list, hist, status)."""
    import torch
    ctx = ctx or default_context(rho[0].device.index or 0)
    N = mesh.NB * mesh.nb
    p = params(N, 1.0 / N, tol=tol, max_cycles=max_cycles, fixed_cycles=fixed_cycles, npre=npre, npost=npost,
               omega=omega, mode=mode, four_pi_g=four_pi_g)
    b = boundary(bc, fixed_b, lmax, origin)
    if phi is None:
        phi = [torch.zeros_like(r) for r in rho]
    st, hist = mg_amr_solve(ctx, p, mesh, b, rho, phi, stream)
    return phi, hist, st


# ------------------------------------------------------------------ operator entry points

def _ctx(ctx):
    return ctx or default_context()


def mg_op_half_sweep(u, f, h, omega, colour, kinds, bext=None, ctx=None, stream=None):
    c = _ctx(ctx)
    return c.check(c._lib.mg_op_half_sweep(c.handle, u.shape[0], float(h), float(omega), int(colour),
                                           ctypes.byref(level_bc(kinds, bext)), _ptr(u), _ptr(f), _stream(stream)),
                   "mg_op_half_sweep")


def mg_op_smooth(u, f, h, omega, sweeps, kinds, bext=None, ctx=None, stream=None):
    c = _ctx(ctx)
    return c.check(c._lib.mg_op_smooth(c.handle, u.shape[0], float(h), float(omega), int(sweeps),
                                       ctypes.byref(level_bc(kinds, bext)), _ptr(u), _ptr(f), _stream(stream)),
                   "mg_op_smooth")


def mg_op_fill(u, out, kinds, bext=None, ctx=None, stream=None):
    c = _ctx(ctx)
    return c.check(c._lib.mg_op_fill(c.handle, u.shape[0], ctypes.byref(level_bc(kinds, bext)), _ptr(u), _ptr(out),
                                     _stream(stream)), "mg_op_fill")


def mg_solve_simple(rho, bc_kind, dx, tol, phi, ctx=None, stream=None):
    """The short form of mg_solve (defaults; one kind on all six faces); returns (hist, status)."""
    c = _ctx(ctx)
    kind = KINDS[bc_kind] if isinstance(bc_kind, str) else int(bc_kind)
    hist = (ctypes.c_double * 51)()
    nh = ctypes.c_int()
    st = c.check(c._lib.mg_solve_simple(c.handle, rho.shape[0], _ptr(rho), kind, float(dx), float(tol), _ptr(phi),
                                        hist, ctypes.byref(nh), _stream(stream)), "mg_solve_simple")
    return [hist[i] for i in range(nh.value)], st


def mg_op_defect(u, f, d, h, kinds, bext=None, ctx=None, stream=None):
    c = _ctx(ctx)
    return c.check(c._lib.mg_op_defect(c.handle, u.shape[0], float(h), ctypes.byref(level_bc(kinds, bext)),
                                       _ptr(u), _ptr(f), _ptr(d), _stream(stream)), "mg_op_defect")


def mg_op_restrict(uf, uc, ctx=None, stream=None):
    c = _ctx(ctx)
    return c.check(c._lib.mg_op_restrict(c.handle, uc.shape[0], _ptr(uf), _ptr(uc), _stream(stream)),
                   "mg_op_restrict")


def mg_op_prolong_add(uc, uf, kinds, bext=None, ctx=None, stream=None):
    c = _ctx(ctx)
    return c.check(c._lib.mg_op_prolong_add(c.handle, uc.shape[0], ctypes.byref(level_bc(kinds, bext)), _ptr(uc),
                                            _ptr(uf), _stream(stream)), "mg_op_prolong_add")


def mg_op_prolong_fmg(uc, uf, kinds, bext=None, ctx=None, stream=None):
    c = _ctx(ctx)
    return c.check(c._lib.mg_op_prolong_fmg(c.handle, uc.shape[0], ctypes.byref(level_bc(kinds, bext)), _ptr(uc),
                                            _ptr(uf), _stream(stream)), "mg_op_prolong_fmg")


def mg_op_coarsest(u, f, h, kinds, bext=None, ctx=None, stream=None):
    c = _ctx(ctx)
    return c.check(c._lib.mg_op_coarsest(c.handle, float(h), ctypes.byref(level_bc(kinds, bext)), _ptr(u), _ptr(f),
                                         _stream(stream)), "mg_op_coarsest")


def mg_op_down(u, f, fc, uc, h, omega, npre, kinds, bext=None, ctx=None, stream=None):
    c = _ctx(ctx)
    return c.check(c._lib.mg_op_down(c.handle, u.shape[0], float(h), float(omega), int(npre),
                                     ctypes.byref(level_bc(kinds, bext)), _ptr(u), _ptr(f), _ptr(fc), _ptr(uc),
                                     _stream(stream)), "mg_op_down")


def mg_op_up(u, f, uc, h, omega, npost, kinds, bext=None, kinds_coarse=None, ctx=None, stream=None):
    c = _ctx(ctx)
    kc = kinds_coarse if kinds_coarse is not None else kinds
    return c.check(c._lib.mg_op_up(c.handle, u.shape[0], float(h), float(omega), int(npost),
                                   ctypes.byref(level_bc(kinds, bext)), ctypes.byref(level_bc(kc, None)), _ptr(u),
                                   _ptr(f), _ptr(uc), _stream(stream)), "mg_op_up")


def mg_op_smooth_f32(u, f, h, omega, sweeps, kinds, bext=None, zero_in=False, ctx=None, stream=None):
    c = _ctx(ctx)
    return c.check(c._lib.mg_op_smooth_f32(c.handle, u.shape[0], float(h), float(omega), int(sweeps),
                                           1 if zero_in else 0, ctypes.byref(level_bc(kinds, bext)), _ptr(u), _ptr(f),
                                           _stream(stream)), "mg_op_smooth_f32")


def mg_op_down_f32(u, f, fc, uc, h, omega, npre, kinds, bext=None, ctx=None, stream=None):
    c = _ctx(ctx)
    return c.check(c._lib.mg_op_down_f32(c.handle, u.shape[0], float(h), float(omega), int(npre),
                                         ctypes.byref(level_bc(kinds, bext)), _ptr(u), _ptr(f), _ptr(fc), _ptr(uc),
                                         _stream(stream)), "mg_op_down_f32")


def mg_op_up_f32(u, f, uc, h, omega, npost, kinds, bext=None, kinds_coarse=None, ctx=None, stream=None):
    c = _ctx(ctx)
    kc = kinds_coarse if kinds_coarse is not None else kinds
    return c.check(c._lib.mg_op_up_f32(c.handle, u.shape[0], float(h), float(omega), int(npost),
                                       ctypes.byref(level_bc(kinds, bext)), ctypes.byref(level_bc(kc, None)), _ptr(u),
                                       _ptr(f), _ptr(uc), _stream(stream)), "mg_op_up_f32")


def mg_op_sweep_input_norm(u, f, h, omega, kinds, bext=None, ctx=None, stream=None):
    """One sweep of u in place; returns the sum of squared defects of the input u."""
    c = _ctx(ctx)
    out = ctypes.c_double()
    c.check(c._lib.mg_op_sweep_input_norm(c.handle, u.shape[0], float(h), float(omega),
                                          ctypes.byref(level_bc(kinds, bext)), _ptr(u), _ptr(f), ctypes.byref(out),
                                          _stream(stream)), "mg_op_sweep_input_norm")
    return out.value


def mg_op_mixed_update(phi, e, f, r32, h, kinds, bext=None, ctx=None, stream=None):
    """phi += e; r32 = FP32(f - L phi); returns the sum of squared defects."""
    c = _ctx(ctx)
    out = ctypes.c_double()
    c.check(c._lib.mg_op_mixed_update(c.handle, phi.shape[0], float(h), ctypes.byref(level_bc(kinds, bext)),
                                      _ptr(phi), _ptr(e), _ptr(f), _ptr(r32), ctypes.byref(out), _stream(stream)),
            "mg_op_mixed_update")
    return out.value


def mg_multipole_moments(rho, dx, lmax=4, origin=None, ctx=None, stream=None):
    c = _ctx(ctx)
    o_in = (ctypes.c_double * 3)(*(origin if origin is not None else (0.0, 0.0, 0.0)))
    o_out = (ctypes.c_double * 3)()
    q = (ctypes.c_double * 25)()
    c.check(c._lib.mg_multipole_moments(c.handle, rho.shape[0], float(dx), _ptr(rho), int(lmax),
                                        0 if origin is None else 1, o_in, o_out, q, _stream(stream)),
            "mg_multipole_moments")
    return list(o_out), list(q)
