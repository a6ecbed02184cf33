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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


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
    dfaces = None if faces is None else [dev(b) for b in faces]
    phi, hist, st = mg.solve(dev(rho), 1.0 / n, kinds, fixed_b=dfaces, tol=1e-11, precision="mixed")
    assert st in (mg.MG_OK, mg.MG_STALLED)
    assert hist[-1] <= 1e-11 or st == mg.MG_STALLED
    assert rel(phi.cpu().numpy(), ref) < 1e-10, rel(phi.cpu().numpy(), ref)


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
        ctx.set_tuning("".join(f"pass fp64 {l} {split}\n" for l in (6, 7)))
        phi, hist, st = mg.solve(dev(rho), 1.0 / n, kinds, fixed_cycles=4, ctx=ctx)
        out[name] = (phi.cpu().numpy(), hist)
        assert rel(out[name][0], ref) < 1e-10, name
        hist_close(hist, rh, residual_floor(ref, rho, kinds == "periodic"))
    assert rel(out["fused"][0], out["split"][0]) < 1e-13


def test_dense_autotune_sets_pass_schedules(mg):
    ctx = mg.Context(0)
    text = ctx.autotune(128, precision="fp64", reps=2, layout="dense")
    lines = [l.split() for l in text.strip().splitlines() if l.startswith("pass")]
    assert {int(l[2]) for l in lines} == {6, 7}
    rho = wl.gaussian_clumps(128, 4)
    a, ah, _ = mg.solve(dev(rho), 1.0 / 128, "periodic", fixed_cycles=3, ctx=ctx)
    b, bh, _ = mg.solve(dev(rho), 1.0 / 128, "periodic", fixed_cycles=3)
    assert rel(a.cpu().numpy(), b.cpu().numpy()) < 1e-13
