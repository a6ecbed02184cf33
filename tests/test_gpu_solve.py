"""Whole-solve parity of the HIP path with the oracle (Alg. 1 + Alg. 2 + Sec. 2.3.7), through
mg_solve.  FP64: equal cycle counts, residual histories elementwise and phi to 1e-10 relative
(the bound the method targets; expected ~1e-13).  Mixed precision: phi after refinement to the
FP64 residual floor against the converged oracle."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import FIXED, MULTIPOLE, PERIODIC, ZERO_GRADIENT
from oracle import exact as ex

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mg():
    import paper_2302_13903_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


from parity import rel, rel_l2  # noqa: E402  (relative L2 and element-wise bounds together)


def run_both(mg, rho, kinds, faces=None, cycles=6, **kw):
    n = rho.shape[0]
    ref, rh, rst = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, fixed_cycles=cycles, **kw)
    dfaces = None if faces is None else [None if b is None else dev(b) for b in faces]
    phi, hist, st = mg.solve(dev(rho), 1.0 / n, kinds, fixed_b=dfaces, fixed_cycles=cycles, **kw)
    torch.cuda.synchronize()
    return ref, np.asarray(rh), phi.cpu().numpy(), np.asarray(hist), st


def residual_floor(phi, rho, gauge_free=True):
    """Round-off floor of the relative residual RMS(f - L phi)/RMS(f): each defect carries an
    error of about eps * 12 max|phi| / h^2 (seven terms of size |phi|/h^2)."""
    n = phi.shape[0]
    f = 4 * math.pi * rho
    if gauge_free:
        f = f - f.mean()
    return 12 * np.finfo(float).eps * np.abs(phi).max() * n * n / math.sqrt(np.mean(f * f))


def hist_close(h_gpu, h_ref, floor=1e-13):
    """Residual histories agree elementwise: 1e-6 relative plus ten times the round-off floor
    of the relative residual (FMA contraction and summation order differ between the sides)."""
    assert len(h_gpu) == len(h_ref)
    for a, b in zip(h_gpu, h_ref):
        assert abs(a - b) <= 1e-6 * b + 10 * floor, (h_gpu, h_ref, floor)


@pytest.mark.parametrize("n", [2, 4, 16, 32, 64])
def test_c1_sine_modes(mg, n):
    """Configuration 1 (sum of 8 sine modes, periodic, V(2,2)) and smaller/larger grids."""
    rho, modes = wl.sine_modes(max(n, 8), 1) if n >= 8 else (wl.random_field((n,) * 3, n), None)
    if n < 8:
        rho = rho - rho.mean()
    ref, rh, got, gh, st = run_both(mg, rho, "periodic", cycles=6)
    assert st == mg.MG_OK
    assert rel(got, ref) < 1e-10
    hist_close(gh, rh, residual_floor(ref, rho))


@pytest.mark.parametrize("kinds", [
    [FIXED] * 6,
    [ZERO_GRADIENT] * 6,
    [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, ZERO_GRADIENT],
    [FIXED, ZERO_GRADIENT, ZERO_GRADIENT, FIXED, PERIODIC, PERIODIC],
])
@pytest.mark.parametrize("n", [8, 32, 64])
def test_boundary_kinds(mg, kinds, n):
    rho = wl.gaussian_clumps(n, 11, n_clumps=6, remove_mean=False)
    rng = np.random.default_rng(n)
    faces = [rng.standard_normal((n, n)) * 0.1 if k == FIXED else None for k in kinds]
    ref, rh, got, gh, st = run_both(mg, rho, kinds, faces, cycles=8)
    assert rel(got, ref) < 1e-10, rel(got, ref)
    hist_close(gh, rh, residual_floor(ref, rho, all(k in (PERIODIC, ZERO_GRADIENT) for k in kinds)))


@pytest.mark.parametrize("n", [16, 64])
def test_multipole_sphere(mg, n):
    rho, c = wl.uniform_sphere(n, 2)
    ref, rh, got, gh, st = run_both(mg, rho, [MULTIPOLE] * 6, cycles=8, lmax=4)
    assert rel(got, ref) < 1e-10
    hist_close(gh, rh, residual_floor(ref, rho, False))


@pytest.mark.parametrize("lmax", [0, 1, 2, 3])
def test_multipole_lower_orders(mg, lmax):
    """Expansions truncated below the hexadecapole (each band of the face sum on or off) for an
    off-centre clump field, so that every order carries moments."""
    n = 64
    rho = wl.gaussian_clumps(n, 5)
    ref, rh, got, gh, st = run_both(mg, rho, [MULTIPOLE] * 6, cycles=6, lmax=lmax)
    assert rel(got, ref) < 1e-10
    hist_close(gh, rh, residual_floor(ref, rho, False))


def test_tol_stop_matches_oracle(mg):
    """Stopping by tolerance: same cycle count and status as the oracle."""
    n = 64
    rho = wl.gaussian_clumps(n, 3)
    ref, rh, rst = oracle.solve(rho, 1.0 / n, "periodic", tol=1e-10)
    phi, hist, st = mg.solve(dev(rho), 1.0 / n, "periodic", tol=1e-10)
    assert st == rst == mg.MG_OK and len(hist) == len(rh)
    assert rel(phi.cpu().numpy(), ref) < 1e-10


def test_mgi_mode(mg):
    n = 32
    rho = wl.gaussian_clumps(n, 4)
    guess = wl.random_field((n,) * 3, 9) * 1e-3
    ref, rh, _ = oracle.solve(rho, 1.0 / n, "periodic", mode="mgi", phi0=guess, fixed_cycles=5)
    phi, hist, st = mg.solve(dev(rho), 1.0 / n, "periodic", mode="mgi", phi=dev(guess), fixed_cycles=5)
    assert rel(phi.cpu().numpy(), ref) < 1e-10
    hist_close(np.asarray(hist), rh, residual_floor(ref, rho))


@pytest.mark.parametrize("kinds,n", [("periodic", 64), ("fixed", 64), ("periodic", 128), ("multipole", 128)])
def test_mixed_precision_reaches_fp64(mg, kinds, n):
    """FP32 inner V-cycles inside FP64 defect correction reach the FP64 accuracy: phi agrees
    with the oracle converged to its floor, within 1e-10 relative."""
    if kinds in ("fixed", "multipole"):
        rho, c = wl.uniform_sphere(n, 1)
        faces = wl.sphere_face_values(n, c, 0.25, rho.sum() / n ** 3) if kinds == "fixed" else None
    else:
        rho, faces = wl.gaussian_clumps(n, 2), None
    ref, rh, _ = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, tol=1e-13, max_cycles=40)
    _, rh11, rst11 = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, tol=1e-11, max_cycles=40)
    assert rst11 == oracle.OK
    dfaces = None if faces is None else [dev(b) for b in faces]
    ctx = mg.Context(0)
    phi, hist, st = mg.solve(dev(rho), 1.0 / n, kinds, fixed_b=dfaces, tol=1e-11, precision="mixed", ctx=ctx)
    assert st == mg.MG_OK and hist[-1] <= 1e-11, (st, hist)
    # each outer step runs 1..3 FP32 V-cycles inside FP64 defect correction; each of them
    # contracts like an FP64 V-cycle: in all, at most two more than the FP64 oracle needs for
    # the same tolerance (the last step's count is chosen from the contraction seen so far)
    k = ctx.last_inner()
    assert len(hist) - 1 <= k <= 3 * (len(hist) - 1), (k, hist)
    assert k <= len(rh11) - 1 + 2, (k, hist, rh11)
    for a, b in zip(hist[1:], hist):
        if b > 1e-9:
            assert a <= 0.2 * b, hist
    assert rel(phi.cpu().numpy(), ref) < 1e-10, rel(phi.cpu().numpy(), ref)


def test_mixed_inner_cycles(mg):
    """"inner fp32 k" runs k FP32 V-cycles per outer defect-correction step: the residual
    falls by about k V-cycles' contraction per step, mg_last_inner counts them, and every k
    reaches the oracle's converged phi.  Unset: one per step in a fixed-cycle solve, 1..3 per
    step to a tolerance.  FP64 solves report none."""
    n = 64
    rho = wl.gaussian_clumps(n, 6)
    ref, _, _ = oracle.solve(rho, 1.0 / n, "periodic", tol=1e-13, max_cycles=40)
    steps = {}
    for k in (1, 2, 3):
        ctx = mg.Context(0)
        ctx.set_tuning(f"inner fp32 {k}\n")
        assert f"inner fp32 {k}" in ctx.tuning()
        phi, hist, st = mg.solve(dev(rho), 1.0 / n, "periodic", tol=1e-10, precision="mixed", ctx=ctx)
        assert st == mg.MG_OK and hist[-1] <= 1e-10, (k, st, hist)
        assert ctx.last_inner() == k * (len(hist) - 1), (k, ctx.last_inner(), hist)
        for a, b in zip(hist[1:], hist):
            if b > 1e-8:
                assert a <= 0.2 ** k * b, (k, hist)
        assert rel(phi.cpu().numpy(), ref) < 1e-10
        steps[k] = len(hist) - 1
    assert steps[3] <= steps[2] < steps[1], steps
    ctx = mg.Context(0)
    _, hist, _ = mg.solve(dev(rho), 1.0 / n, "periodic", fixed_cycles=3, precision="mixed", ctx=ctx)
    assert ctx.last_inner() == 3 and len(hist) == 4
    _, hist, st = mg.solve(dev(rho), 1.0 / n, "periodic", tol=1e-10, precision="mixed", ctx=ctx)
    assert st == mg.MG_OK and len(hist) - 1 <= ctx.last_inner() <= 3 * (len(hist) - 1)
    mg.solve(dev(rho), 1.0 / n, "periodic", tol=1e-10, ctx=ctx)
    assert ctx.last_inner() == 0
    for bad in ("inner fp32 0\n", "inner fp32 5\n", "inner fp64 2\n"):
        with pytest.raises(mg.MgError, match="INVALID_ARG"):
            ctx.set_tuning(bad)


def test_deterministic(mg):
    n = 64
    rho = dev(wl.gaussian_clumps(n, 8))
    a, ha, _ = mg.solve(rho, 1.0 / n, "periodic", fixed_cycles=4)
    b, hb, _ = mg.solve(rho, 1.0 / n, "periodic", fixed_cycles=4)
    assert torch.equal(a, b) and ha == hb


def test_status_and_errors(mg):
    n = 16
    rho = wl.gaussian_clumps(n, 1, n_clumps=2)
    bad = rho.copy()
    bad[1, 2, 3] = np.inf
    with pytest.raises(mg.MgError, match="NONFINITE"):
        mg.solve(dev(bad), 1.0 / n, "periodic")
    with pytest.raises(mg.MgError, match="INVALID_ARG"):
        mg.solve(dev(rho), 1.0 / n, ["periodic", "fixed", "periodic", "periodic", "periodic", "periodic"])
    with pytest.raises(mg.MgError, match="INVALID_ARG"):
        mg.solve(dev(np.zeros((12, 12, 12))), 1.0 / 12, "periodic")
    _, hist, st = mg.solve(dev(rho), 1.0 / n, "periodic", tol=1e-30, max_cycles=3)
    assert st in (mg.MG_NOT_CONVERGED, mg.MG_STALLED)
    _, hist, st = mg.solve(dev(rho), 1.0 / n, "periodic", tol=1e-30, max_cycles=100)
    assert st == mg.MG_STALLED


def test_spectral_256(mg):
    """256^3 clumps (configuration 2 at its smaller size): the solve to 1e-10 matches the exact
    discrete solution from the FFT solve to the accuracy the residual implies."""
    n = 256
    rho = wl.gaussian_clumps(n, 2)
    phi, hist, st = mg.solve(dev(rho), 1.0 / n, "periodic", tol=1e-10)
    assert st == mg.MG_OK and hist[-1] <= 1e-10
    f = 4 * math.pi * rho
    f -= f.mean()
    ref = ex.spectral_solve(f, 1.0 / n, [PERIODIC] * 6)
    assert rel(phi.cpu().numpy(), ref) < 1e-9


@pytest.mark.parametrize("kinds", ["periodic", [FIXED] * 6])
def test_pass_fusion_schedules_agree(mg, kinds):
    """The restricted defect and the norm fused into the last smoothing pass or run as their own
    defect-only passes: the same expressions of the same values, so the same result up to
    floating-point contraction, and both equal to the oracle."""
    n = 128
    rho = wl.gaussian_clumps(n, 31, remove_mean=kinds == "periodic")
    ref, rh, _ = oracle.solve(rho, 1.0 / n, kinds, fixed_cycles=4)
    out = {}
    for name, split in (("fused", 0), ("split", 3)):
        ctx = mg.Context(0)
        ctx.set_tuning("fusedmin fp64 64\n" + "".join(f"pass fp64 {l} {split}\n" for l in (6, 7)))
        phi, hist, st = mg.solve(dev(rho), 1.0 / n, kinds, fixed_cycles=4, ctx=ctx)
        out[name] = (phi.cpu().numpy(), hist)
        assert rel(out[name][0], ref) < 1e-10, name
        hist_close(hist, rh, residual_floor(ref, rho, kinds == "periodic"))
    assert rel(out["fused"][0], out["split"][0]) < 1e-13


def test_dense_autotune_sets_pass_schedules(mg):
    ctx = mg.Context(0)
    ctx.set_tuning("fusedmin fp64 64\n")
    text = ctx.autotune(128, precision="fp64", reps=2, layout="dense")
    lines = [l.split() for l in text.strip().splitlines() if l.startswith("pass")]
    assert {int(l[2]) for l in lines} == {6, 7}
    rho = wl.gaussian_clumps(128, 4)
    a, ah, _ = mg.solve(dev(rho), 1.0 / 128, "periodic", fixed_cycles=3, ctx=ctx)
    b, bh, _ = mg.solve(dev(rho), 1.0 / 128, "periodic", fixed_cycles=3)
    assert rel(a.cpu().numpy(), b.cpu().numpy()) < 1e-13


@pytest.mark.parametrize("fusedmin,tail", [(64, 4), (128, 3), (256, 2)])
def test_level_schedules_agree(mg, fusedmin, tail):
    """Where the fused passes start and how many levels the LDS tail holds change only the
    launch structure, not the method: every schedule matches the oracle."""
    n = 256
    rho = wl.gaussian_clumps(n, 41, n_clumps=16, remove_mean=False)
    faces = [np.full((n, n), -0.5)] * 6
    ref, rh, _ = oracle.solve(rho, 1.0 / n, [FIXED] * 6, fixed_b=faces, fixed_cycles=3)
    ctx = mg.Context(0)
    ctx.set_tuning(f"fusedmin fp64 {fusedmin}\ntail fp64 {tail}\n")
    phi, hist, st = mg.solve(dev(rho), 1.0 / n, [FIXED] * 6, fixed_b=[dev(b) for b in faces], fixed_cycles=3,
                             ctx=ctx)
    assert rel(phi.cpu().numpy(), ref) < 1e-10
    hist_close(hist, rh, residual_floor(ref, rho, False))


TB_KINDS = [
    "periodic",
    [FIXED] * 6,
    [ZERO_GRADIENT] * 6,
    [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, ZERO_GRADIENT],
    [FIXED, ZERO_GRADIENT, ZERO_GRADIENT, FIXED, PERIODIC, PERIODIC],
]


@pytest.mark.parametrize("kinds", TB_KINDS)
@pytest.mark.parametrize("n", [64, 128, 256])
def test_temporal_blocking_matches_oracle(mg, kinds, n):
    """Two sweeps per pass (temporally blocked) on every level from 64^3: the same V-cycles."""
    print(f"tb fp64 n={n} kinds={kinds}", flush=True)
    gauge_free = kinds == "periodic" or kinds == [ZERO_GRADIENT] * 6
    rho = wl.gaussian_clumps(n, 50 + n, n_clumps=12, remove_mean=gauge_free)
    faces = None
    if not gauge_free:
        rng = np.random.default_rng(n)
        faces = [rng.normal(size=(n, n)) * 0.2 for _ in range(6)]
    ref, rh, _ = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, fixed_cycles=4)
    ctx = mg.Context(0)
    ctx.set_tuning("tb fp64 1\nfusedmin fp64 64\n")
    dfaces = None if faces is None else [dev(b) for b in faces]
    phi, hist, st = mg.solve(dev(rho), 1.0 / n, kinds, fixed_b=dfaces, fixed_cycles=4, ctx=ctx)
    assert st == mg.MG_OK
    assert rel(phi.cpu().numpy(), ref) < 1e-10
    hist_close(hist, rh, residual_floor(ref, rho, gauge_free))


@pytest.mark.parametrize("kinds", ["periodic", [FIXED] * 6])
def test_temporal_blocking_mixed(mg, kinds):
    print(f"tb mixed kinds={kinds}", flush=True)
    n = 128
    gauge_free = kinds == "periodic"
    rho = wl.gaussian_clumps(n, 77, remove_mean=gauge_free)
    ref, _, _ = oracle.solve(rho, 1.0 / n, kinds, tol=1e-13, max_cycles=40)
    ctx = mg.Context(0)
    ctx.set_tuning("tb fp32 1\nfusedmin fp32 64\n")
    phi, hist, st = mg.solve(dev(rho), 1.0 / n, kinds, precision="mixed", tol=1e-11, max_cycles=40, ctx=ctx)
    assert hist[-1] < 1e-10
    assert rel(phi.cpu().numpy(), ref) < 1e-10


@pytest.mark.parametrize("npre,npost", [(1, 1), (3, 2), (2, 3)])
def test_temporal_blocking_odd_sweep_counts(mg, npre, npost):
    """Sweep counts that are not pairs mix two-sweep and one-sweep passes."""
    n = 64
    rho = wl.gaussian_clumps(n, 9, remove_mean=True)
    ref, rh, _ = oracle.solve(rho, 1.0 / n, "periodic", fixed_cycles=3, npre=npre, npost=npost)
    ctx = mg.Context(0)
    ctx.set_tuning("tb fp64 1\nfusedmin fp64 64\n")
    phi, hist, st = mg.solve(dev(rho), 1.0 / n, "periodic", fixed_cycles=3, npre=npre, npost=npost, ctx=ctx)
    assert rel(phi.cpu().numpy(), ref) < 1e-10
    hist_close(hist, rh, residual_floor(ref, rho, True))


@pytest.mark.parametrize("kinds", ["periodic", [FIXED] * 6])
def test_mixed_zero_start_first_sweep(mg, kinds):
    """The mixed inner V-cycle's first sweep skips reading the (zero) correction: results equal
    those of the path that clears the correction first (one-sweep-per-pass vs blocked)."""
    n = 256
    gauge_free = kinds == "periodic"
    rho = wl.gaussian_clumps(n, 13, remove_mean=gauge_free)
    outs = []
    # the one-sweep passes (the two-sweep passes are off; their zero start is checked below)
    for text in ("march fp32 0\ntb fp32 0\n", "march fp32 0\ntb fp32 1\n"):
        ctx = mg.Context(0)
        ctx.set_tuning(text)
        phi, hist, st = mg.solve(dev(rho), 1.0 / n, kinds, precision="mixed", fixed_cycles=3, ctx=ctx)
        outs.append((phi.cpu().numpy(), hist))
    assert rel(outs[0][0], outs[1][0]) < 1e-12
    assert np.allclose(outs[0][1], outs[1][1], rtol=1e-6)


@pytest.mark.parametrize("kinds", ["periodic", [FIXED] * 6])
def test_mixed_two_sweep_passes_reach_fp64(mg, kinds):
    """Mixed precision with the FP32 inner cycles on the two-sweep streaming passes at 256^3
    (the first down pass starts from a zero correction it does not read): phi against the
    oracle converged to its floor, within 1e-10, in at most one outer step more than FP64."""
    n = 256
    gauge_free = kinds == "periodic"
    rho = wl.gaussian_clumps(n, 13, remove_mean=gauge_free)
    ref, rh, _ = oracle.solve(rho, 1.0 / n, kinds, tol=1e-13, max_cycles=40)
    _, rh11, _ = oracle.solve(rho, 1.0 / n, kinds, tol=1e-11, max_cycles=40)
    ctx = mg.Context(0)
    ctx.set_tuning("march fp32 2\n")
    phi, hist, st = mg.solve(dev(rho), 1.0 / n, kinds, precision="mixed", tol=1e-11, ctx=ctx)
    assert st == mg.MG_OK and hist[-1] <= 1e-11, (st, hist)
    assert len(hist) <= len(rh11) + 1, (hist, rh11)
    assert rel(phi.cpu().numpy(), ref) < 1e-10


@pytest.mark.parametrize("n,kinds,layout,extra", [
    (64, "periodic", "dense", {}),                      # region-tile legs
    (128, "periodic", "dense", {}),                     # two-sweep passes
    (128, [FIXED] * 6, "dense", {}),                    # split passes (interior and wall ring)
    (128, [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, ZERO_GRADIENT], "dense", {}),
    (128, "periodic", "blocks", {}),                    # MeshBlock layout
    (128, "periodic", "dense", {"scheme": "fas"}),
    (128, [FIXED] * 6, "dense", {"precision": "mixed"}),
])
def test_history_is_the_defect_rms_of_phi(mg, n, kinds, layout, extra):
    """Each history entry the device reports (the norm it publishes to the host after a cycle)
    is RMS(f - L phi)/RMS(f) of the phi it returns (Sec. 2.3.7), recomputed on the host with the
    matrix-free ghost rules of oracle.exact: for k = 0..4 cycles after FMG, hist[k] of a k-cycle
    run matches it to 1e-9 relative plus 1 % of the round-off floor (a gauge-free phi is shifted
    to zero mean after the last cycle, which moves its residual by round-off), and every run's
    history is a prefix of the next one's to the same bound."""
    print(f"history pin n={n} kinds={kinds} layout={layout} {extra}", flush=True)
    gauge_free = kinds == "periodic"
    kk = [PERIODIC] * 6 if gauge_free else kinds
    rho = wl.gaussian_clumps(n, 7, remove_mean=False)
    rng = np.random.default_rng(2)
    faces = [rng.standard_normal((n, n)) * 0.1 if k == FIXED else None for k in kk]
    dfaces = None if gauge_free else [None if b is None else dev(b) for b in faces]
    f = 4 * math.pi * rho
    if gauge_free:
        f = f - f.mean()
    x = mg.to_blocks(dev(rho), 16) if layout == "blocks" else dev(rho)
    ctx = mg.Context(0)
    prev = None
    for k in range(5):
        cyc = {"max_cycles": 0} if k == 0 else {"fixed_cycles": k}
        phi, hist, st = mg.solve(x, 1.0 / n, kinds, fixed_b=dfaces, layout=layout, block_n=16, ctx=ctx, **cyc,
                                 **extra)
        torch.cuda.synchronize()
        assert st >= 0, (k, st, hist)
        assert len(hist) == k + 1, (k, hist)
        p = (mg.from_blocks(phi, n, 16) if layout == "blocks" else phi).cpu().numpy()
        r = ex.rel_residual(p, f, 1.0 / n, kk, None if gauge_free else faces)
        floor = residual_floor(p, rho, gauge_free)
        assert hist[-1] > 1e3 * floor or k == 4, (k, hist, floor)
        assert abs(hist[-1] - r) <= 1e-9 * r + 1e-2 * floor, (k, hist[-1], r, floor)
        if prev is not None:
            for a, b in zip(hist[:-1], prev):
                assert abs(a - b) <= 1e-9 * b + 1e-2 * floor, (hist, prev)
        prev = list(hist)
