"""Every streaming pass of the solver's large levels, element by element against the oracle's
operators, in both precisions, through the C ABI:

  FP64  head pass (one sweep + the defect norm of its input), mixed-precision update
        (phi + e, FP64 defect, its FP32 copy and norm);
  FP32  sweep (also with a zero input that is not read), sweep + restricted defect (the down
        step), prolongation + sweep (the up step) -- the inner cycle of MG_PREC_MIXED.

FP32 results are compared with the FP64 oracle run on the same FP32-rounded inputs, within a
bound of a few FP32 roundings of the operands' magnitude per sweep (a wrong tile, halo or
skipped stage shows up as an O(1) error, far above it).  Sizes: 128^3 (tiles of 56-60
output columns, so the last tile of each row is ragged) for every boundary mix, and 512^3 in
the launch configuration of the benchmark."""
import numpy as np
import pytest

import oracle
from oracle import FIXED, PERIODIC, ZERO_GRADIENT

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


def hom_of(kinds):
    return [k if k in (PERIODIC, ZERO_GRADIENT) else FIXED for k in kinds]


def make(n, seed, kinds, f32):
    """u ~ N(0,1), f ~ N(0,1) n^2 (so h^2 f and u are of one size), face values ~ N(0,1); for
    FP32 runs every input is rounded to FP32 first and the oracle takes the rounded values."""
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


def scale_u(u, ref, f, h, bext):
    bmax = max([0.0] + [float(np.abs(b).max()) for b in bext if b is not None])
    return float(np.abs(u).max() + np.abs(ref).max() + h * h * np.abs(f).max() + 2 * bmax)


def f32dev(a):
    return dev(a.astype(np.float32))


def check_f32(got, ref, bound, what):
    err = float(np.max(np.abs(got.astype(np.float64) - ref)))
    assert err <= bound, (what, err, bound)
    return err


CASES = [(128, ks) for ks in range(len(KIND_SETS))] + [(512, 0), (512, 3)]


@pytest.mark.parametrize("n,ks", CASES)
def test_fp32_sweeps(mg, n, ks):
    kinds = KIND_SETS[ks]
    print(f"fp32 sweeps n={n} kinds={kinds}", flush=True)
    u, f, bext = make(n, 10 + n + ks, kinds, True)
    h = 1.0 / n
    for sweeps in (1, 2):
        ref = u
        for _ in range(sweeps):
            ref = oracle.smooth(ref, f, h, OMEGA, kinds, bext)
        du = f32dev(u)
        mg.mg_op_smooth_f32(du, f32dev(f), h, OMEGA, sweeps, kinds, dbext(bext))
        check_f32(host(du), ref, 20 * sweeps * EPS32 * scale_u(u, ref, f, h, bext), ("sweeps", sweeps))
    # the first sweep of a correction cycle: u = 0 on input, not read (the array holds garbage)
    ref = oracle.smooth(np.zeros_like(u), f, h, OMEGA, kinds, bext)
    du = torch.full((n,) * 3, float("nan"), dtype=torch.float32, device="cuda:0")
    mg.mg_op_smooth_f32(du, f32dev(f), h, OMEGA, 1, kinds, dbext(bext), zero_in=True)
    check_f32(host(du), ref, 20 * EPS32 * scale_u(ref, ref, f, h, bext), "zero input")


@pytest.mark.parametrize("n,ks", CASES)
def test_fp32_down(mg, n, ks):
    """Two sweeps, the last carrying the restricted defect; the coarse correction cleared."""
    kinds = KIND_SETS[ks]
    print(f"fp32 down n={n} kinds={kinds}", flush=True)
    u, f, bext = make(n, 20 + n + ks, kinds, True)
    h = 1.0 / n
    ref = oracle.smooth(oracle.smooth(u, f, h, OMEGA, kinds, bext), f, h, OMEGA, kinds, bext)
    ref_fc = oracle.restrict(oracle.defect(ref, f, h, kinds, bext))
    du = f32dev(u)
    fc = torch.full((n // 2,) * 3, 7.0, dtype=torch.float32, device="cuda:0")
    uc = torch.full((n // 2,) * 3, 7.0, dtype=torch.float32, device="cuda:0")
    mg.mg_op_down_f32(du, f32dev(f), fc, uc, h, OMEGA, 2, kinds, dbext(bext))
    s = scale_u(u, ref, f, h, bext)
    check_f32(host(du), ref, 40 * EPS32 * s, "u")
    check_f32(host(fc), ref_fc, 40 * EPS32 * (np.abs(f).max() + 12 * s / h ** 2), "fc")
    assert float(uc.abs().max()) == 0.0


@pytest.mark.parametrize("n,ks", CASES)
def test_fp32_up(mg, n, ks):
    """The trilinear correction (homogeneous coarse ghosts) entering with the first of two
    sweeps."""
    kinds = KIND_SETS[ks]
    hom = hom_of(kinds)
    print(f"fp32 up n={n} kinds={kinds}", flush=True)
    u, f, bext = make(n, 30 + n + ks, kinds, True)
    h = 1.0 / n
    rng = np.random.default_rng(40 + n + ks)
    e = rng.standard_normal((n // 2,) * 3).astype(np.float32).astype(np.float64)
    ref = oracle.prolong_add(e, u, hom)
    ref = oracle.smooth(oracle.smooth(ref, f, h, OMEGA, kinds, bext), f, h, OMEGA, kinds, bext)
    du = f32dev(u)
    mg.mg_op_up_f32(du, f32dev(f), f32dev(e), h, OMEGA, 2, kinds, dbext(bext), kinds_coarse=hom)
    check_f32(host(du), ref, 40 * EPS32 * (scale_u(u, ref, f, h, bext) + np.abs(e).max()), "u")


@pytest.mark.parametrize("n,ks", CASES)
def test_fp64_head_pass(mg, n, ks):
    """The first pre-sweep of a V-cycle with the residual norm of the iterate it starts from."""
    kinds = KIND_SETS[ks]
    print(f"fp64 head n={n} kinds={kinds}", flush=True)
    u, f, bext = make(n, 50 + n + ks, kinds, False)
    h = 1.0 / n
    ref = oracle.smooth(u, f, h, OMEGA, kinds, bext)
    d = oracle.defect(u, f, h, kinds, bext)
    du = dev(u)
    sumsq = mg.mg_op_sweep_input_norm(du, dev(f), h, OMEGA, kinds, dbext(bext))
    got = host(du)
    assert float(np.max(np.abs(got - ref))) <= TOL64 * float(np.abs(ref).max() + np.abs(u).max())
    want = float(np.sum(d * d))
    assert abs(sumsq - want) <= 1e-12 * want, (sumsq, want)


@pytest.mark.parametrize("n,ks", CASES)
def test_fp64_mixed_update(mg, n, ks):
    """phi + e (FP64 sum of an FP32 correction), the defect of the result, its FP32 copy and
    the sum of its squares, in one pass."""
    kinds = KIND_SETS[ks]
    print(f"mixed update n={n} kinds={kinds}", flush=True)
    phi, f, bext = make(n, 60 + n + ks, kinds, False)
    rng = np.random.default_rng(70 + n + ks)
    e = (rng.standard_normal((n,) * 3) * 1e-3).astype(np.float32)
    h = 1.0 / n
    phi2 = phi + e.astype(np.float64)
    d = oracle.defect(phi2, f, h, kinds, bext)
    dphi = dev(phi)
    r32 = torch.full((n,) * 3, float("nan"), dtype=torch.float32, device="cuda:0")
    sumsq = mg.mg_op_mixed_update(dphi, dev(e), dev(f), r32, h, kinds, dbext(bext))
    assert np.array_equal(host(dphi), phi2)    # one FP64 addition on both sides
    dscale = float(np.abs(f).max() + 12 * np.abs(phi2).max() / h ** 2)
    got_r = host(r32).astype(np.float64)
    assert float(np.max(np.abs(got_r - d) - EPS32 * np.abs(d))) <= TOL64 * dscale
    want = float(np.sum(d * d))
    assert abs(sumsq - want) <= 1e-12 * want, (sumsq, want)
