"""Pins of the oracle's whole iteration (Alg. 1 V-cycle, Alg. 2 FMG) against exact
discrete solutions computed without multigrid, closed forms, and the convergence
behaviour the paper reports.  CPU only."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import FIXED, PERIODIC, ZERO_GRADIENT
from oracle import exact as ex

FPG = 4 * math.pi


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n", [4, 8])
@pytest.mark.parametrize("kinds", [
    [PERIODIC] * 6, [FIXED] * 6, [ZERO_GRADIENT] * 6,
    [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, ZERO_GRADIENT],
    [FIXED, ZERO_GRADIENT, ZERO_GRADIENT, FIXED, PERIODIC, PERIODIC],
])
def test_solve_matches_dense_direct(n, kinds):
    """Converged multigrid equals the dense direct solve of the same discrete system."""
    rng = np.random.default_rng(n + sum(kinds))
    rho = rng.standard_normal((n,) * 3)
    faces = [rng.standard_normal((n, n)) for _ in range(6)]
    gauge_free = all(k in (PERIODIC, ZERO_GRADIENT) for k in kinds)
    phi, hist, st = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, tol=1e-13, max_cycles=300)
    f = FPG * rho
    if gauge_free:
        f = f - f.mean()
    ref = ex.dense_solve(f, 1.0 / n, kinds, faces)
    assert st in (oracle.OK, oracle.STALLED)
    assert _rel(phi, ref) < 1e-11
    if gauge_free:
        assert abs(phi.mean()) < 1e-13 * np.abs(phi).max()


@pytest.mark.parametrize("kinds", [[PERIODIC] * 6, [FIXED] * 6, [ZERO_GRADIENT] * 6])
def test_solve_matches_spectral(kinds):
    """32^3 clump density: multigrid to 1e-11 agrees with the FFT / DST-II / DCT-II
    exact discrete solution."""
    n = 32
    rho = wl.gaussian_clumps(n, 5, n_clumps=8, remove_mean=False)
    faces = [0.01 * np.ones((n, n)) * (f + 1) for f in range(6)] if kinds[0] == FIXED else None
    phi, hist, st = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, tol=1e-11, max_cycles=200)
    f = FPG * rho
    if kinds[0] != FIXED:
        f = f - f.mean()
    ref = ex.spectral_solve(f, 1.0 / n, kinds, faces)
    assert st == oracle.OK
    assert _rel(phi, ref) < 1e-9
    assert ex.rel_residual(phi, f, 1.0 / n, kinds, faces) <= 1e-11


def test_c1_closed_form():
    """The 32^3 sum-of-sines problem: each product-of-sines mode is an eigenvector, so the
    exact discrete solution is closed-form; FMG + V(2,2) to 1e-10 reaches it."""
    n = 32
    rho, modes = wl.sine_modes(n, 1)
    phi, hist, st = oracle.solve(rho, 1.0 / n, "periodic", tol=1e-10)
    ref = ex.sine_modes_exact(n, modes)
    assert st == oracle.OK
    assert hist[-1] <= 1e-10 and len(hist) <= 10
    assert _rel(phi, ref) < 1e-9


def test_vcycle_convergence_factor(golden):
    """Sec. 4.1.1: V(1,1) reduces the defect by CF ~ 0.125 per cycle, independent of h;
    V(2,2) contracts faster still."""
    cf_paper = golden["vcycle_convergence_factor"]["value"]
    cfs = {}
    for n in (16, 32, 64):
        rho = wl.gaussian_clumps(n, 3, n_clumps=16)
        for nu in (1, 2):
            phi, hist, st = oracle.solve(rho, 1.0 / n, "periodic", npre=nu, npost=nu, mode="mgi",
                                         phi0=np.zeros((n,) * 3), fixed_cycles=6)
            ratios = hist[2:6] / hist[1:5]
            cfs[(n, nu)] = float(np.exp(np.mean(np.log(ratios))))
    for n in (16, 32, 64):
        assert cfs[(n, 1)] <= 1.3 * cf_paper, cfs
        assert cfs[(n, 2)] < cfs[(n, 1)], cfs
    # independence of resolution
    assert max(cfs[(n, 1)] for n in (16, 32, 64)) / min(cfs[(n, 1)] for n in (16, 32, 64)) < 2.0


def test_sine_problem_cycles_and_fmg(golden):
    """The paper's sinusoidal problem (rho0 = 2, A = 1, G = 1): V(1,1) reaches the round-off
    floor within the stated 10-15 cycles; one FMG sweep is already at truncation-error level
    against the analytic solution (Sec. 4.1.1)."""
    p = golden["sine_test"]["value"]
    lo, hi = golden["cycles_to_full_convergence"]["value"]
    n = 64
    x = (np.arange(n) + 0.5) / n
    s = np.sin(2 * math.pi * x)
    rho = p["rho0"] + p["A"] * s[:, None, None] * s[None, :, None] * s[None, None, :]
    analytic = -FPG * p["A"] / (3 * (2 * math.pi) ** 2) * s[:, None, None] * s[None, :, None] * s[None, None, :]
    phi0, hist0, _ = oracle.solve(rho, 1.0 / n, "periodic", npre=1, npost=1, fixed_cycles=0)
    phic, hist, _ = oracle.solve(rho, 1.0 / n, "periodic", npre=1, npost=1,
                                 fixed_cycles=golden["fully_converged_cycles_uniform"]["value"])
    floor = hist[-1]
    reached = int(np.argmax(hist <= 3 * floor))
    assert lo - 3 <= reached <= hi, hist
    e_fmg = np.sqrt(np.mean((phi0 - analytic) ** 2))
    e_conv = np.sqrt(np.mean((phic - analytic) ** 2))
    assert e_fmg <= 1.5 * e_conv


def test_second_order_accuracy_sphere():
    """Uniform sphere with fixed boundary values from its analytic potential (Sec. 4.2):
    the converged error against the analytic potential falls ~4x per doubling of N."""
    errs = []
    for n in (16, 32, 64):
        rho, c = wl.uniform_sphere(n, 2)
        mass = rho.sum() / n ** 3
        faces = wl.sphere_face_values(n, c, 0.25, mass)
        phi, hist, st = oracle.solve(rho, 1.0 / n, "fixed", fixed_b=faces, tol=1e-11, max_cycles=60)
        x = (np.arange(n) + 0.5) / n
        ana = wl.sphere_potential(x[None, None, :], x[None, :, None], x[:, None, None], c, 0.25, mass)
        errs.append(np.sqrt(np.mean((phi - ana) ** 2)) / np.sqrt(np.mean(ana ** 2)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 2.5 < r1 < 6 and 2.5 < r2 < 6, errs


def test_gauge_invariance():
    """Periodic: adding a constant to rho does not change phi (mean removal, Sec. 2.3.6)."""
    n = 16
    rho = wl.gaussian_clumps(n, 9, n_clumps=4, remove_mean=False)
    p1, _, _ = oracle.solve(rho, 1.0 / n, "periodic", fixed_cycles=8)
    p2, _, _ = oracle.solve(rho + 5.0, 1.0 / n, "periodic", fixed_cycles=8)
    assert np.max(np.abs(p1 - p2)) < 1e-12 * np.max(np.abs(p1))
    assert abs(p1.mean()) < 1e-14 * np.max(np.abs(p1))


def test_status_codes():
    n = 8
    rho = wl.gaussian_clumps(n, 1, n_clumps=2)
    _, hist, st = oracle.solve(rho, 1.0 / n, "periodic", tol=1e-30, max_cycles=3)
    assert st in (oracle.NOT_CONVERGED, oracle.STALLED) and len(hist) <= 4
    _, hist, st = oracle.solve(rho, 1.0 / n, "periodic", tol=1e-30, max_cycles=200)
    assert st == oracle.STALLED
    bad = rho.copy()
    bad[1, 2, 3] = np.nan
    _, _, st = oracle.solve(bad, 1.0 / n, "periodic")
    assert st == oracle.ERR_NONFINITE
    _, _, st = oracle.solve(np.zeros((6, 6, 6)), 1.0 / 6, "periodic")
    assert st == oracle.ERR_INVALID
    _, _, st = oracle.solve(rho, 1.0 / n, [PERIODIC, FIXED, PERIODIC, PERIODIC, PERIODIC, PERIODIC])
    assert st == oracle.ERR_INVALID


def test_fmg_coarse_boundary_values_are_restricted():
    """Set-up reading: coarser levels take the 2x2 area mean of the finer face values."""
    n = 8
    rng = np.random.default_rng(2)
    faces = [rng.standard_normal((n, n)) for _ in range(6)]
    s = oracle.State(np.zeros((n,) * 3), 1.0 / n, "fixed", fixed_b=faces)
    for face in range(6):
        b3 = s.face(3, face)[1:-1, 1:-1]
        b2 = s.face(2, face)[1:-1, 1:-1]
        assert np.allclose(b3, faces[face])
        assert np.allclose(b2, faces[face].reshape(4, 2, 4, 2).mean(axis=(1, 3)))


@pytest.mark.parametrize("n,kinds", [
    (32, "periodic"),
    (64, [FIXED] * 6),
    (32, [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, ZERO_GRADIENT]),
    (32, [ZERO_GRADIENT] * 6),
])
def test_residual_history_is_the_defect_rms(n, kinds):
    """Every history entry the oracle reports is RMS(f - L phi)/RMS(f) of the iterate it
    returns (Sec. 2.3.7), recomputed with the matrix-free ghost rules of oracle.exact (itself
    pinned: exact discrete solutions have round-off residuals).  For k = 0..4 V-cycles after
    FMG, hist[k] of a k-cycle run matches that recomputation to 1e-12 relative plus 1 % of the
    round-off floor (the returned phi is shifted to zero mean when gauge-free, which moves its
    residual by round-off), and every run's history is a prefix of the next one's."""
    gauge_free = kinds == "periodic" or kinds == [ZERO_GRADIENT] * 6
    kk = [PERIODIC] * 6 if kinds == "periodic" else kinds
    rho = wl.gaussian_clumps(n, 3, remove_mean=False)
    rng = np.random.default_rng(1)
    faces = [rng.standard_normal((n, n)) * 0.1 if k == FIXED else None for k in kk]
    f = FPG * rho
    if gauge_free:
        f = f - f.mean()
    prev = None
    for k in range(5):
        if k == 0:
            phi, hist, st = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, max_cycles=0)
        else:
            phi, hist, st = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, fixed_cycles=k)
        assert len(hist) == k + 1
        r = ex.rel_residual(phi, f, 1.0 / n, kk, faces)
        floor = 12 * np.finfo(float).eps * np.abs(phi).max() * n * n / math.sqrt(np.mean(f * f))
        assert hist[-1] > 1e4 * floor          # every entry is far above the floor here
        assert abs(hist[-1] - r) <= 1e-12 * r + 1e-2 * floor, (k, hist[-1], r, floor)
        if prev is not None:
            assert np.array_equal(hist[:-1], prev)
        prev = hist


def test_coarse_rule_reading():
    """Sec. 2.3.6 taken literally makes the coarse-level corrections of a zero-gradient problem
    zero-fixed: an operator other than the fine level's, and the V-cycle then contracts the
    residual by only about 0.9 per cycle.  The reading followed keeps zero-gradient faces
    zero-gradient on the coarse levels: about 0.1 per cycle or better, as for the other kinds.
    Where no face is zero-gradient the two rules are one rule (equal histories)."""
    n = 32
    rho = wl.gaussian_clumps(n, 3)
    rates, last = {}, {}
    for rule in ("homogeneous", "literal"):
        st = oracle.State(rho, 1.0 / n, [ZERO_GRADIENT] * 6)
        st.set_coarse_rule(rule)
        r0 = st.residual()
        r = [st.vcycle() for _ in range(5)]
        rates[rule] = (r[-1] / r0) ** (1 / 5)
        last[rule] = r[-1] / r[-2]
    assert rates["homogeneous"] < 0.15 and last["homogeneous"] < 0.2, (rates, last)
    # the literal rule slows down cycle after cycle (0.4 in the first, above 0.8 by the fifth)
    assert last["literal"] > 0.7, (rates, last)
    kk = [FIXED, FIXED, PERIODIC, PERIODIC, FIXED, FIXED]
    hs = {}
    for rule in ("homogeneous", "literal"):
        st = oracle.State(rho, 1.0 / n, kk)
        st.set_coarse_rule(rule)
        hs[rule] = [st.vcycle() for _ in range(3)]
    assert hs["homogeneous"] == hs["literal"]
    with pytest.raises(ValueError):
        oracle.State(rho, 1.0 / n, kk).set_coarse_rule("zero")
