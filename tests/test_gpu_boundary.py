"""The rest of the C-ABI boundary on the GPU: the ghost-fill operator against the oracle's fill
(Sec. 2.3.6; faces, edges and corners, every boundary mix), the short solve call against the
full one and the oracle, and the context's HBM budget."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import FIXED, MULTIPOLE, PERIODIC, ZERO_GRADIENT
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


@pytest.fixture(scope="module")
def mg():
    import paper_2302_13903_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("n", [1, 2, 8, 64])
@pytest.mark.parametrize("ks", range(len(KIND_SETS)))
def test_fill_matches_oracle(mg, n, ks):
    """Every one of the (n+2)^3 values, ghosts included, equals the oracle's: active cells and
    face ghosts bitwise (a copy or one 2 b - u on both sides); edge and corner ghosts, which
    compose two or three face rules, to a few ulps (the two sides round the composition in a
    different order)."""
    kinds = KIND_SETS[ks]
    rng = np.random.default_rng(n * 10 + ks)
    u = rng.standard_normal((n,) * 3)
    bext = [rng.standard_normal((n + 2, n + 2)) if kinds[q] == FIXED else None for q in range(6)]
    ref = oracle.fill(u, kinds, bext)
    out = torch.full((n + 2,) * 3, float("nan"), dtype=torch.float64, device="cuda:0")
    mg.mg_op_fill(dev(u), out, kinds, [None if b is None else dev(b) for b in bext])
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert not np.isnan(got).any()
    idx = np.arange(n + 2)
    ghost = ((idx == 0) | (idx == n + 1)).astype(int)
    nghost = ghost[:, None, None] + ghost[None, :, None] + ghost[None, None, :]
    single = nghost <= 1
    assert np.array_equal(got[single], ref[single]), (n, kinds)
    bmax = max([0.0] + [float(np.abs(b).max()) for b in bext if b is not None])
    bound = 8 * np.finfo(float).eps * (np.abs(u).max() + 6 * bmax)
    assert float(np.max(np.abs(got - ref))) <= bound, (n, kinds, np.max(np.abs(got - ref)))


def test_fill_multipole_faces_are_fixed(mg):
    """A MULTIPOLE face of a level description is a FIXED face with the given values."""
    n = 16
    rng = np.random.default_rng(3)
    u = rng.standard_normal((n,) * 3)
    bext = [rng.standard_normal((n + 2, n + 2)) for _ in range(6)]
    out = torch.zeros((n + 2,) * 3, dtype=torch.float64, device="cuda:0")
    as_fixed = torch.zeros_like(out)
    mg.mg_op_fill(dev(u), out, [MULTIPOLE] * 6, [dev(b) for b in bext])
    mg.mg_op_fill(dev(u), as_fixed, [FIXED] * 6, [dev(b) for b in bext])
    torch.cuda.synchronize()
    assert torch.equal(out, as_fixed)
    ref = oracle.fill(u, [FIXED] * 6, bext)
    assert float(np.max(np.abs(out.cpu().numpy() - ref))) <= 8 * np.finfo(float).eps * 7 * np.abs(ref).max()


@pytest.mark.parametrize("kind", ["periodic", "fixed", "zero_gradient", "multipole"])
def test_solve_simple(mg, kind):
    """The short call equals mg_solve with the defaults (bitwise) and the oracle (1e-10)."""
    n = 64
    if kind == "multipole":
        rho, _ = wl.uniform_sphere(n, 4)
    else:
        rho = wl.gaussian_clumps(n, 12, remove_mean=kind == "periodic")
    drho = dev(rho)
    phi = torch.zeros_like(drho)
    hist, st = mg.mg_solve_simple(drho, kind, 1.0 / n, 1e-10, phi)
    full, fh, fst = mg.solve(drho, 1.0 / n, kind, tol=1e-10, lmax=4)
    torch.cuda.synchronize()
    assert st == fst and hist == fh
    assert torch.equal(phi, full)
    ref, rh, rst = oracle.solve(rho, 1.0 / n, kind, fixed_cycles=len(hist) - 1, lmax=4)
    assert rel(phi.cpu().numpy(), ref) < 1e-10
    assert st in (mg.MG_OK, mg.MG_STALLED)


def test_solve_simple_rejects_bad_arguments(mg):
    n = 8
    rho = dev(np.zeros((n,) * 3))
    phi = torch.zeros_like(rho)
    with pytest.raises(mg.MgError, match="INVALID_ARG"):
        mg.mg_solve_simple(rho, 7, 1.0 / n, 1e-10, phi)
    with pytest.raises(mg.MgError, match="INVALID_ARG"):
        mg.mg_solve_simple(rho, "periodic", 1.0 / n, -1.0, phi)


def test_context_budget(mg):
    """A context whose budget is one 64^3 footprint solves 64^3 and refuses 128^3 with
    MG_ERR_OOM (nothing allocated); the refusal leaves the context usable."""
    fp = mg.mg_footprint_bytes(mg.params(64, 1 / 64))
    ctx = mg.Context(0, hbm_budget=fp)
    rho64 = dev(wl.gaussian_clumps(64, 1))
    phi64, h64, st = mg.solve(rho64, 1 / 64, "periodic", ctx=ctx)
    assert st == mg.MG_OK
    rho128 = dev(wl.gaussian_clumps(128, 1))
    with pytest.raises(mg.MgError, match="OOM"):
        mg.solve(rho128, 1 / 128, "periodic", ctx=ctx)
    again, h2, st2 = mg.solve(rho64, 1 / 64, "periodic", ctx=ctx)
    assert st2 == mg.MG_OK and torch.equal(again, phi64) and h2 == h64
    # mixed precision needs more than the FP64 footprint of the same size
    assert mg.mg_footprint_bytes(mg.params(64, 1 / 64, precision="mixed")) > fp
    with pytest.raises(mg.MgError, match="OOM"):
        mg.solve(rho64, 1 / 64, "periodic", precision="mixed", ctx=ctx)
    # unlimited context for comparison
    free, _, _ = mg.solve(rho128, 1 / 128, "periodic", ctx=mg.Context(0))
    assert math.isfinite(float(free.abs().max()))
