"""GPU parity of the Full Approximation Scheme solve (Alg. 3; FMG with FAS, Sec. 2.3.5) with
the oracle's FAS, through mg_solve with scheme = FAS: equal cycle counts, residual histories
elementwise and phi to 1e-10 relative, every boundary kind, FMG and warm starts, both the
per-operator levels and the streaming smoothing passes; and at the benchmark size, FAS against
the correction scheme on the device (equal up to rounding on this linear problem)."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import FIXED, MULTIPOLE, PERIODIC, ZERO_GRADIENT

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KIND_SETS = {
    "periodic": [PERIODIC] * 6,
    "fixed": [FIXED] * 6,
    "zero_gradient": [ZERO_GRADIENT] * 6,
    "mixed": [FIXED, ZERO_GRADIENT, ZERO_GRADIENT, FIXED, PERIODIC, PERIODIC],
    "multipole": [MULTIPOLE] * 6,
}


@pytest.fixture(scope="module")
def mg():
    import paper_2302_13903_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


from parity import rel, rel_l2  # noqa: E402  (relative L2 and element-wise bounds together)


def floor_of(phi, rho, kinds):
    """Round-off floor of the relative residual (12 eps max|phi| / h^2 per defect)."""
    n = phi.shape[0]
    f = 4 * math.pi * rho
    if all(k in (PERIODIC, ZERO_GRADIENT) for k in kinds):
        f = f - f.mean()
    return 12 * np.finfo(float).eps * np.abs(phi).max() * n * n / math.sqrt(np.mean(f * f))


@pytest.mark.parametrize("mode", ["fmg", "mgi"])
@pytest.mark.parametrize("name", list(KIND_SETS))
@pytest.mark.parametrize("n,tuning", [(16, ""), (64, ""), (128, "fusedmin fp64 64\n")])
def test_fas_matches_oracle(mg, n, tuning, name, mode):
    kinds = KIND_SETS[name]
    print(f"fas n={n} {name} {mode} {tuning.strip()}", flush=True)
    rng = np.random.default_rng(n + len(name))
    rho = wl.gaussian_clumps(n, 21, n_clumps=6, remove_mean=False)
    faces = [rng.uniform(-0.5, 0.5, (n, n)) if k == FIXED else None for k in kinds]
    phi0 = rng.uniform(-1, 1, (n, n, n)) if mode == "mgi" else None
    ref, rh, rst = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, mode=mode, phi0=phi0, fixed_cycles=5,
                                scheme="fas")
    ctx = mg.Context(0)
    if tuning:
        ctx.set_tuning(tuning)
    phi = dev(phi0) if phi0 is not None else None
    got, gh, st = mg.solve(dev(rho), 1.0 / n, kinds, fixed_b=[None if b is None else dev(b) for b in faces],
                           fixed_cycles=5, mode=mode, phi=phi, scheme="fas", ctx=ctx)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert st == mg.MG_OK
    assert rel(got, ref) < 1e-10
    fl = floor_of(ref, rho, kinds)
    assert len(gh) == len(rh) == 6
    for a, b in zip(gh, rh):
        assert abs(a - b) <= 1e-6 * b + 10 * fl, (gh, list(rh), fl)


def test_fas_equals_correction_scheme_256(mg):
    """256^3 clumps with fixed faces, FMG + 6 cycles: FAS and the correction scheme on the
    device agree to rounding (the paper's equivalence on linear problems), cycle by cycle."""
    print("fas vs cs 256^3", flush=True)
    n = 256
    rho = dev(wl.gaussian_clumps(n, 9, remove_mean=False))
    faces = [torch.full((n, n), -0.3, dtype=torch.float64, device="cuda:0")] * 6
    a, ha, sa = mg.solve(rho, 1.0 / n, "fixed", fixed_b=faces, fixed_cycles=6)
    b, hb, sb = mg.solve(rho, 1.0 / n, "fixed", fixed_b=faces, fixed_cycles=6, scheme="fas")
    assert len(ha) == len(hb) == 7
    for x, y in zip(ha, hb):
        assert abs(x - y) <= 1e-6 * x + 1e-12
    assert float((a - b).norm() / a.norm()) < 1e-11


def test_fas_bench_size_converges(mg):
    """The bench workload (512^3 periodic clumps, tolerance 1e-10) with FAS: converges in the
    correction scheme's cycle count to the same potential."""
    print("fas 512^3", flush=True)
    n = 512
    rho = dev(wl.gaussian_clumps(n, 2))
    a, ha, sa = mg.solve(rho, 1.0 / n, "periodic", tol=1e-10)
    b, hb, sb = mg.solve(rho, 1.0 / n, "periodic", tol=1e-10, scheme="fas")
    assert sb == mg.MG_OK and hb[-1] <= 1e-10
    assert len(hb) == len(ha)
    assert float((a - b).norm() / a.norm()) < 1e-10


def test_fas_unsupported_forms(mg):
    n = 32
    rho = dev(wl.gaussian_clumps(n, 1))
    with pytest.raises(mg.MgError, match="UNSUPPORTED"):
        mg.solve(rho, 1.0 / n, "periodic", scheme="fas", precision="mixed")
    with pytest.raises(mg.MgError, match="UNSUPPORTED"):
        mg.solve(mg.to_blocks(rho, 8), 1.0 / n, "periodic", scheme="fas", layout="blocks", block_n=8)


@pytest.mark.parametrize("npre,npost", [(1, 1), (1, 2), (3, 2)])
def test_fas_sweep_counts_streamed(mg, npre, npost):
    """Streamed FAS levels with other sweep counts: the head pass takes the first pre-sweep (or
    the only one), the last remaining pre-sweep carries the restriction, or the restriction
    runs on its own; cycle by cycle as the oracle."""
    n = 128
    kinds = [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, ZERO_GRADIENT]
    print(f"fas sweeps {npre},{npost}", flush=True)
    rng = np.random.default_rng(7)
    rho = wl.gaussian_clumps(n, 22, n_clumps=6, remove_mean=False)
    faces = [rng.uniform(-0.5, 0.5, (n, n)) if k == FIXED else None for k in kinds]
    ref, rh, _ = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, fixed_cycles=4, npre=npre, npost=npost,
                              scheme="fas")
    ctx = mg.Context(0)
    ctx.set_tuning("fusedmin fp64 64\n")
    got, gh, st = mg.solve(dev(rho), 1.0 / n, kinds, fixed_b=[None if b is None else dev(b) for b in faces],
                           fixed_cycles=4, npre=npre, npost=npost, scheme="fas", ctx=ctx)
    got = got.cpu().numpy()
    assert st == mg.MG_OK and rel(got, ref) < 1e-10
    fl = floor_of(ref, rho, kinds)
    assert len(gh) == len(rh) == 5
    for a, b in zip(gh, rh):
        assert abs(a - b) <= 1e-6 * b + 10 * fl, (gh, list(rh), fl)


@pytest.mark.parametrize("name", ["periodic", "fixed"])
def test_fas_tolerance_streamed(mg, name):
    """FAS to a tolerance on streamed levels: the head pass of each next cycle measures the
    cycle's result and is discarded when the test stops; cycle count and potential as the
    oracle's."""
    n = 128
    kinds = KIND_SETS[name]
    print(f"fas tol streamed {name}", flush=True)
    rng = np.random.default_rng(31)
    rho = wl.gaussian_clumps(n, 23, n_clumps=6, remove_mean=name == "periodic")
    faces = [rng.uniform(-0.5, 0.5, (n, n)) if k == FIXED else None for k in kinds]
    ref, rh, _ = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, tol=1e-9, scheme="fas")
    ctx = mg.Context(0)
    ctx.set_tuning("fusedmin fp64 64\n")
    got, gh, st = mg.solve(dev(rho), 1.0 / n, kinds, fixed_b=[None if b is None else dev(b) for b in faces],
                           tol=1e-9, scheme="fas", ctx=ctx)
    assert st == mg.MG_OK and len(gh) == len(rh)
    assert rel(got.cpu().numpy(), ref) < 1e-10


@pytest.mark.parametrize("mode", ["fmg", "mgi"])
@pytest.mark.parametrize("n", [16, 64])
@pytest.mark.parametrize("kinds", [[FIXED] * 6, [FIXED, ZERO_GRADIENT, ZERO_GRADIENT, FIXED, PERIODIC, PERIODIC]])
def test_fas_zero_valued_fixed_faces(mg, n, kinds, mode):
    """Fixed faces with zero values: no level's description carries face values, so the levels
    <= 16^3 run the FAS cycle in the LDS tail (its wall form), whose single cell is then solved
    (a fixed face fixes the zero point).  Against the oracle's FAS at equal cycle counts."""
    print(f"fas zero-fixed n={n} kinds={kinds} {mode}", flush=True)
    rng = np.random.default_rng(n + 7)
    rho = wl.gaussian_clumps(n, 23, n_clumps=6, remove_mean=False)
    phi0 = rng.uniform(-1, 1, (n, n, n)) if mode == "mgi" else None
    ref, rh, _ = oracle.solve(rho, 1.0 / n, kinds, mode=mode, phi0=phi0, fixed_cycles=5, scheme="fas")
    phi = dev(phi0) if phi0 is not None else None
    got, gh, st = mg.solve(dev(rho), 1.0 / n, kinds, fixed_cycles=5, mode=mode, phi=phi, scheme="fas")
    torch.cuda.synchronize()
    assert st == mg.MG_OK
    got = got.cpu().numpy()
    assert rel(got, ref) < 1e-10
    fl = floor_of(ref, rho, kinds)
    assert len(gh) == len(rh) == 6
    for a, b in zip(gh, rh):
        assert abs(a - b) <= 1e-6 * b + 10 * fl, (gh, list(rh), fl)
