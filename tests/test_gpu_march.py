"""The one-launch V(2,2) legs against the oracle: the two-sweep streaming passes of the large
levels and the region-tile legs of the small ones (32^3 .. 128^3).

Down pass: two sweeps, then the defect restricted to the coarse level (and the coarse
correction cleared); up pass: the trilinear correction added as u is loaded, then two sweeps.
Element by element through mg_op_down / mg_op_up (which run these passes when the context's
"march" setting allows them, as the solver does), FP64 and FP32, on 128^3 (tiles of 52
output cells: ragged), 256^3 and the benchmark's 512^3, periodic (the default schedule) and
every boundary mix (forced with "march ... 2").  Whole solves with the passes on and off: the
same cycles as the oracle, phi to 1e-10 and the residual history (whose entries after each
cycle come from the up pass's norm stage)."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import FIXED, PERIODIC, ZERO_GRADIENT
from parity import rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KIND_SETS = [
    [PERIODIC] * 6,
    [FIXED] * 6,
    [ZERO_GRADIENT] * 6,
    [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, ZERO_GRADIENT],
    [FIXED, ZERO_GRADIENT, ZERO_GRADIENT, FIXED, PERIODIC, PERIODIC],
]
EPS32 = float(np.finfo(np.float32).eps)
TOL64 = 1e-13
OMEGA = 1.15


@pytest.fixture(scope="module")
def mg():
    import paper_2302_13903_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def make(n, seed, kinds, f32):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((n,) * 3)
    f = rng.standard_normal((n,) * 3) * n * n
    bext = [rng.standard_normal((n + 2, n + 2)) if kinds[q] == FIXED else None for q in range(6)]
    if f32:
        u = u.astype(np.float32).astype(np.float64)
        f = f.astype(np.float32).astype(np.float64)
    return u, f, bext


def dbext(bext):
    return [None if b is None else dev(b) for b in bext]


def ctx_for(mg, kinds, prec):
    ctx = mg.Context(0)
    if kinds != [PERIODIC] * 6:
        ctx.set_tuning(f"march {prec} 2\n")
    return ctx


def scale_u(u, ref, f, h, bext):
    bmax = max([0.0] + [float(np.abs(b).max()) for b in bext if b is not None])
    return float(np.abs(u).max() + np.abs(ref).max() + h * h * np.abs(f).max() + 2 * bmax)


CASES = [(128, ks) for ks in range(len(KIND_SETS))] + [(256, 0), (512, 0), (512, 3)]
# region-tile legs: 32^3 (one region per 16 x 16 x 8 block, wrapping halos), 64^3, and 128^3 with
# the streaming passes off
TILE_CASES = [(32, ks) for ks in range(len(KIND_SETS))] + [(64, 0), (64, 4), (128, 3)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,ks", CASES)
def test_march_down(mg, n, ks, prec):
    kinds = KIND_SETS[ks]
    f32 = prec == "fp32"
    print(f"march down n={n} kinds={kinds} {prec}", flush=True)
    u, f, bext = make(n, 100 + n + ks, kinds, f32)
    h = 1.0 / n
    ref = oracle.smooth(oracle.smooth(u, f, h, OMEGA, kinds, bext), f, h, OMEGA, kinds, bext)
    ref_fc = oracle.restrict(oracle.defect(ref, f, h, kinds, bext))
    dt = torch.float32 if f32 else torch.float64
    du = dev(u.astype(np.float32) if f32 else u)
    df = dev(f.astype(np.float32) if f32 else f)
    fc = torch.full((n // 2,) * 3, 7.0, dtype=dt, device="cuda:0")
    uc = torch.full((n // 2,) * 3, 7.0, dtype=dt, device="cuda:0")
    ctx = ctx_for(mg, kinds, prec)
    (mg.mg_op_down_f32 if f32 else mg.mg_op_down)(du, df, fc, uc, h, OMEGA, 2, kinds, dbext(bext), ctx=ctx)
    got, got_fc = host(du).astype(np.float64), host(fc).astype(np.float64)
    s = scale_u(u, ref, f, h, bext)
    ds = float(np.abs(f).max() + 12 * s / h ** 2)
    bu, bf = (40 * EPS32 * s, 40 * EPS32 * ds) if f32 else (TOL64 * s, TOL64 * ds)
    assert float(np.max(np.abs(got - ref))) <= bu, (np.max(np.abs(got - ref)), bu)
    assert float(np.max(np.abs(got_fc - ref_fc))) <= bf, (np.max(np.abs(got_fc - ref_fc)), bf)
    assert float(uc.abs().max()) == 0.0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,ks", CASES)
def test_march_up(mg, n, ks, prec):
    kinds = KIND_SETS[ks]
    hom = [k if k in (PERIODIC, ZERO_GRADIENT) else FIXED for k in kinds]
    f32 = prec == "fp32"
    print(f"march up n={n} kinds={kinds} {prec}", flush=True)
    u, f, bext = make(n, 200 + n + ks, kinds, f32)
    h = 1.0 / n
    rng = np.random.default_rng(300 + n + ks)
    e = rng.standard_normal((n // 2,) * 3)
    if f32:
        e = e.astype(np.float32).astype(np.float64)
    ref = oracle.prolong_add(e, u, hom)
    ref = oracle.smooth(oracle.smooth(ref, f, h, OMEGA, kinds, bext), f, h, OMEGA, kinds, bext)
    du = dev(u.astype(np.float32) if f32 else u)
    df = dev(f.astype(np.float32) if f32 else f)
    de = dev(e.astype(np.float32) if f32 else e)
    ctx = ctx_for(mg, kinds, prec)
    (mg.mg_op_up_f32 if f32 else mg.mg_op_up)(du, df, de, h, OMEGA, 2, kinds, dbext(bext), kinds_coarse=hom, ctx=ctx)
    got = host(du).astype(np.float64)
    s = scale_u(u, ref, f, h, bext) + float(np.abs(e).max())
    bound = 40 * EPS32 * s if f32 else TOL64 * s
    assert float(np.max(np.abs(got - ref))) <= bound, (np.max(np.abs(got - ref)), bound)


def floor_of(phi, rho, gauge_free):
    n = phi.shape[0]
    f = 4 * math.pi * rho
    if gauge_free:
        f = f - f.mean()
    return 12 * np.finfo(float).eps * np.abs(phi).max() * n * n / math.sqrt(np.mean(f * f))


@pytest.mark.parametrize("n,kinds", [(256, "periodic"), (256, [FIXED] * 6),
                                     (256, [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, ZERO_GRADIENT])])
def test_solve_with_march_matches_oracle(mg, n, kinds):
    """Whole FP64 solves with the two-sweep passes on the large levels: phi and the residual
    history cycle by cycle against the oracle, and against the one-sweep passes."""
    print(f"march solve n={n} kinds={kinds}", flush=True)
    gauge_free = kinds == "periodic"
    rho = wl.gaussian_clumps(n, 77, remove_mean=gauge_free)
    faces = None
    if not gauge_free:
        rng = np.random.default_rng(5)
        kk = kinds
        faces = [rng.standard_normal((n, n)) * 0.1 if k == FIXED else None for k in kk]
    ref, rh, _ = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, fixed_cycles=5)
    dfaces = None if faces is None else [None if b is None else dev(b) for b in faces]
    out = {}
    for mode in (2, 0):
        ctx = mg.Context(0)
        ctx.set_tuning(f"march fp64 {mode}\n")
        phi, hist, st = mg.solve(dev(rho), 1.0 / n, kinds, fixed_b=dfaces, fixed_cycles=5, ctx=ctx)
        torch.cuda.synchronize()
        assert st == mg.MG_OK
        out[mode] = (phi.cpu().numpy(), hist)
        assert rel(out[mode][0], ref) < 1e-10, (mode, rel(out[mode][0], ref))
        fl = floor_of(ref, rho, gauge_free)
        for a, b in zip(hist, rh):
            assert abs(a - b) <= 1e-6 * b + 10 * fl, (mode, hist, rh)
    assert rel(out[2][0], out[0][0]) < 1e-12


@pytest.mark.parametrize("n,kinds", [(256, [FIXED] * 6), (512, [ZERO_GRADIENT] * 6),
                                     (256, [FIXED, FIXED, PERIODIC, PERIODIC, FIXED, FIXED])])
def test_split_passes_match_the_single_launch(mg, n, kinds):
    """A level with x or y walls runs its interior tiles and its wall tiles as two concurrent
    launches ("split fp64 1", the default) or as one ("split fp64 0"): the same expressions on
    every cell (the interior tiles in the z-walls form, whose contraction into FMAs may differ),
    so phi agrees to rounding, element-wise; the residual norms too (the cells are grouped into
    per-workgroup partial sums differently)."""
    print(f"split passes n={n} kinds={kinds}", flush=True)
    rho = wl.gaussian_clumps(n, 31, remove_mean=False)
    rng = np.random.default_rng(8)
    faces = [dev(rng.standard_normal((n, n)) * 0.1) if k == FIXED else None for k in kinds]
    out = []
    for split in (1, 0):
        ctx = mg.Context(0)
        ctx.set_tuning(f"split fp64 {split}\n")
        phi, hist, st = mg.solve(dev(rho), 1.0 / n, kinds, fixed_b=faces, fixed_cycles=3, ctx=ctx)
        torch.cuda.synchronize()
        assert st == mg.MG_OK
        out.append((phi.cpu().numpy(), hist))
    assert rel(out[0][0], out[1][0]) < 1e-13
    assert len(out[0][1]) == len(out[1][1])
    # norms of defects of two phi equal to rounding: equal up to the residual's round-off floor
    fl = floor_of(out[1][0], rho, False)
    for a, b in zip(out[0][1], out[1][1]):
        assert abs(a - b) <= 1e-12 * b + fl, (out[0][1], out[1][1], fl)


@pytest.mark.parametrize("n", [256, 512])
def test_tolerance_stop_with_march(mg, n):
    """Stopping by tolerance with the norm taken by the finest up pass: the same cycle count
    and status as the oracle."""
    print(f"march tol stop n={n}", flush=True)
    rho = wl.gaussian_clumps(n, 2)
    ref, rh, rst = oracle.solve(rho, 1.0 / n, "periodic", tol=1e-10)
    phi, hist, st = mg.solve(dev(rho), 1.0 / n, "periodic", tol=1e-10)
    torch.cuda.synchronize()
    assert st == rst == mg.MG_OK and len(hist) == len(rh), (hist, rh)
    assert rel(phi.cpu().numpy(), ref) < 1e-10


def tile_ctx(mg, prec):
    ctx = mg.Context(0)
    ctx.set_tuning(f"march {prec} 0\n")
    return ctx


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,ks", TILE_CASES)
def test_tile_down(mg, n, ks, prec):
    kinds = KIND_SETS[ks]
    f32 = prec == "fp32"
    print(f"tile down n={n} kinds={kinds} {prec}", flush=True)
    u, f, bext = make(n, 400 + n + ks, kinds, f32)
    h = 1.0 / n
    ref = oracle.smooth(oracle.smooth(u, f, h, OMEGA, kinds, bext), f, h, OMEGA, kinds, bext)
    ref_fc = oracle.restrict(oracle.defect(ref, f, h, kinds, bext))
    dt = torch.float32 if f32 else torch.float64
    du = dev(u.astype(np.float32) if f32 else u)
    df = dev(f.astype(np.float32) if f32 else f)
    fc = torch.full((n // 2,) * 3, 7.0, dtype=dt, device="cuda:0")
    uc = torch.full((n // 2,) * 3, 7.0, dtype=dt, device="cuda:0")
    (mg.mg_op_down_f32 if f32 else mg.mg_op_down)(du, df, fc, uc, h, OMEGA, 2, kinds, dbext(bext),
                                                  ctx=tile_ctx(mg, prec))
    got, got_fc = host(du).astype(np.float64), host(fc).astype(np.float64)
    s = scale_u(u, ref, f, h, bext)
    ds = float(np.abs(f).max() + 12 * s / h ** 2)
    bu, bf = (40 * EPS32 * s, 40 * EPS32 * ds) if f32 else (TOL64 * s, TOL64 * ds)
    assert float(np.max(np.abs(got - ref))) <= bu, (np.max(np.abs(got - ref)), bu)
    assert float(np.max(np.abs(got_fc - ref_fc))) <= bf, (np.max(np.abs(got_fc - ref_fc)), bf)
    assert float(uc.abs().max()) == 0.0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,ks", TILE_CASES)
def test_tile_up(mg, n, ks, prec):
    kinds = KIND_SETS[ks]
    hom = [k if k in (PERIODIC, ZERO_GRADIENT) else FIXED for k in kinds]
    f32 = prec == "fp32"
    print(f"tile up n={n} kinds={kinds} {prec}", flush=True)
    u, f, bext = make(n, 500 + n + ks, kinds, f32)
    h = 1.0 / n
    rng = np.random.default_rng(600 + n + ks)
    e = rng.standard_normal((n // 2,) * 3)
    if f32:
        e = e.astype(np.float32).astype(np.float64)
    ref = oracle.prolong_add(e, u, hom)
    ref = oracle.smooth(oracle.smooth(ref, f, h, OMEGA, kinds, bext), f, h, OMEGA, kinds, bext)
    du = dev(u.astype(np.float32) if f32 else u)
    df = dev(f.astype(np.float32) if f32 else f)
    de = dev(e.astype(np.float32) if f32 else e)
    (mg.mg_op_up_f32 if f32 else mg.mg_op_up)(du, df, de, h, OMEGA, 2, kinds, dbext(bext), kinds_coarse=hom,
                                              ctx=tile_ctx(mg, prec))
    got = host(du).astype(np.float64)
    s = scale_u(u, ref, f, h, bext) + float(np.abs(e).max())
    bound = 40 * EPS32 * s if f32 else TOL64 * s
    assert float(np.max(np.abs(got - ref))) <= bound, (np.max(np.abs(got - ref)), bound)


@pytest.mark.parametrize("n,kinds", [(32, "periodic"), (64, [FIXED] * 6), (128, [ZERO_GRADIENT] * 6),
                                     (64, [FIXED, ZERO_GRADIENT, ZERO_GRADIENT, FIXED, PERIODIC, PERIODIC])])
def test_solve_with_tiles_matches_oracle(mg, n, kinds):
    """Whole FP64 solves with the region-tile legs on the levels 32^3 .. 128^3 (the default): phi
    and the residual history (the finest up leg's norm) cycle by cycle against the oracle, and
    against the per-operator launches."""
    print(f"tile solve n={n} kinds={kinds}", flush=True)
    gauge_free = kinds == "periodic" or kinds == [ZERO_GRADIENT] * 6
    rho = wl.gaussian_clumps(n, 99, remove_mean=gauge_free)
    faces = None
    if not gauge_free:
        rng = np.random.default_rng(7)
        faces = [rng.standard_normal((n, n)) * 0.1 if k == FIXED else None for k in kinds]
    ref, rh, _ = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, fixed_cycles=5)
    dfaces = None if faces is None else [None if b is None else dev(b) for b in faces]
    out = {}
    for mode in (1, 0):
        ctx = mg.Context(0)
        ctx.set_tuning(f"tile fp64 {mode}\n")
        phi, hist, st = mg.solve(dev(rho), 1.0 / n, kinds, fixed_b=dfaces, fixed_cycles=5, ctx=ctx)
        torch.cuda.synchronize()
        assert st == mg.MG_OK
        out[mode] = phi.cpu().numpy()
        assert rel(out[mode], ref) < 1e-10, (mode, rel(out[mode], ref))
        fl = floor_of(ref, rho, gauge_free)
        for a, b in zip(hist, rh):
            assert abs(a - b) <= 1e-6 * b + 10 * fl, (mode, hist, rh)
    assert rel(out[1], out[0]) < 1e-12
