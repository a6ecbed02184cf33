"""Pins of the oracle's Full Approximation Scheme iteration (Alg. 3, and FMG with FAS in place
of the V-cycle, Sec. 2.3.5) against facts that do not come from the FAS code: on the linear
Poisson problem FAS is the correction scheme (the paper's equivalence statement; the
correction-scheme oracle is pinned to exact solves on its own), the exact discrete solution is
a fixed point of one FAS iteration, and converged FAS equals the dense direct solve.  CPU only."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import FIXED, MULTIPOLE, PERIODIC, ZERO_GRADIENT
from oracle import exact as ex

FPG = 4 * math.pi

KIND_SETS = [
    [PERIODIC] * 6,
    [FIXED] * 6,
    [ZERO_GRADIENT] * 6,
    [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, ZERO_GRADIENT],
    [FIXED, ZERO_GRADIENT, ZERO_GRADIENT, FIXED, PERIODIC, PERIODIC],
    [MULTIPOLE] * 6,
]


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def problem(n, seed, kinds):
    rng = np.random.default_rng(seed)
    rho = wl.gaussian_clumps(n, seed, n_clumps=6, remove_mean=False)
    faces = [rng.uniform(-0.5, 0.5, (n, n)) if k == FIXED else None for k in kinds]
    return rho, faces


@pytest.mark.parametrize("mode", ["fmg", "mgi"])
@pytest.mark.parametrize("ki", range(len(KIND_SETS)))
def test_fas_equals_correction_scheme(ki, mode):
    """Linear problem: every FAS iterate equals the correction-scheme iterate up to rounding
    (the coarse problem for psi = phibar + delta is the defect equation for delta), so the
    residual histories and the potentials agree to round-off."""
    kinds = KIND_SETS[ki]
    n = 32
    rho, faces = problem(n, 40 + ki, kinds)
    phi0 = np.random.default_rng(1).uniform(-1, 1, (n, n, n)) if mode == "mgi" else None
    a, ha, sa = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, mode=mode, phi0=phi0, fixed_cycles=6)
    b, hb, sb = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, mode=mode, phi0=phi0, fixed_cycles=6,
                             scheme="fas")
    assert len(ha) == len(hb) == 7
    # round-off floor of the relative residual: ~ 16 eps max|phi| / h^2 / RMS(f)
    f = FPG * rho
    if all(k in (PERIODIC, ZERO_GRADIENT) for k in kinds):
        f = f - f.mean()
    floor = 16 * np.finfo(float).eps * np.abs(a).max() * n * n / math.sqrt(np.mean(f * f))
    assert np.allclose(hb, ha, rtol=1e-6, atol=10 * floor), (ha, hb)
    assert _rel(b, a) < 1e-11


@pytest.mark.parametrize("kinds", [[PERIODIC] * 6, [FIXED] * 6, [ZERO_GRADIENT] * 6,
                                   [FIXED, ZERO_GRADIENT, ZERO_GRADIENT, FIXED, PERIODIC, PERIODIC]])
def test_fas_converges_to_dense_solve(kinds):
    n = 8
    rng = np.random.default_rng(7)
    rho = rng.standard_normal((n,) * 3)
    faces = [rng.standard_normal((n, n)) for _ in range(6)]
    phi, hist, st = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, tol=1e-13, max_cycles=300, scheme="fas")
    f = FPG * rho
    if all(k in (PERIODIC, ZERO_GRADIENT) for k in kinds):
        f = f - f.mean()
    assert st in (oracle.OK, oracle.STALLED)
    assert _rel(phi, ex.dense_solve(f, 1.0 / n, kinds, faces)) < 1e-11


@pytest.mark.parametrize("kinds", [[FIXED] * 6, [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, ZERO_GRADIENT]])
def test_exact_solution_is_a_fixed_point(kinds):
    """With the exact discrete solution as the iterate the restricted defect is zero, so the
    FAS coarse problem (source d + L phibar) is solved by phibar itself and the correction
    vanishes: one FAS iteration leaves the solution unchanged (a sign slip in the coarse
    source, a missing subtraction of phibar or mismatched coarse operators would move it)."""
    n = 8
    rng = np.random.default_rng(3)
    rho = rng.standard_normal((n,) * 3)
    faces = [rng.uniform(-1, 1, (n, n)) for _ in range(6)]
    exact = ex.dense_solve(FPG * rho, 1.0 / n, kinds, faces)
    phi, hist, st = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, mode="mgi", phi0=exact, fixed_cycles=1,
                                 scheme="fas")
    assert np.max(np.abs(phi - exact)) < 1e-12 * np.abs(exact).max()
    assert hist[1] < 1e-12
