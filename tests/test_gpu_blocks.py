"""MeshBlock layout (Sec. 3.2) on the GPU: the batched block-structured solve is the uniform
solve of the same density (the block decomposition with ghost exchange before each colour and
the root grid below one cell per block is the same algorithm), so it must match the oracle at
equal cycle counts (FP64: phi to 1e-10 relative, residual histories to the round-off floor),
match the dense GPU path, and give bitwise the same result under every sweep schedule the
autotuner can pick."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import FIXED, MULTIPOLE, PERIODIC, ZERO_GRADIENT

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mg():
    import paper_2302_13903_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


from parity import rel, rel_l2  # noqa: E402  (relative L2 and element-wise bounds together)


def floor_of(phi, rho, gauge_free):
    n = phi.shape[0]
    f = 4 * math.pi * rho
    if gauge_free:
        f = f - f.mean()
    return 12 * np.finfo(float).eps * np.abs(phi).max() * n * n / math.sqrt(np.mean(f * f))


def solve_blocks(mg, rho, kinds, block_n, faces=None, ctx=None, **kw):
    n = rho.shape[0]
    dfaces = None if faces is None else [None if b is None else dev(b) for b in faces]
    rb = mg.to_blocks(dev(rho), block_n)
    phib, hist, st = mg.solve(rb, 1.0 / n, kinds, fixed_b=dfaces, layout="blocks", block_n=block_n, ctx=ctx, **kw)
    torch.cuda.synchronize()
    return mg.from_blocks(phib, n, block_n).cpu().numpy(), np.asarray(hist), st, phib


CASES = [  # (n, block_n, kinds)
    (16, 2, "periodic"),
    (32, 4, [ZERO_GRADIENT] * 6),
    (32, 8, [FIXED] * 6),
    (64, 16, "periodic"),
    (64, 8, [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, ZERO_GRADIENT]),
    (64, 2, [FIXED, ZERO_GRADIENT, ZERO_GRADIENT, FIXED, PERIODIC, PERIODIC]),
    (128, 16, [FIXED] * 6),
]


@pytest.mark.parametrize("n,block_n,kinds", CASES)
def test_blocks_match_oracle(mg, n, block_n, kinds):
    print(f"blocks vs oracle n={n} block_n={block_n} kinds={kinds}", flush=True)
    periodic_all = kinds == "periodic"
    rho = wl.gaussian_clumps(n, 5 + n + block_n, n_clumps=8, remove_mean=periodic_all)
    faces = None
    gauge_free = periodic_all or kinds == [ZERO_GRADIENT] * 6
    if not gauge_free:
        rng = np.random.default_rng(n + block_n)
        faces = [rng.normal(size=(n, n)) * 0.1 for _ in range(6)]
    ref, rh, rst = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, fixed_cycles=5)
    got, gh, st, _ = solve_blocks(mg, rho, kinds, block_n, faces=faces, fixed_cycles=5)
    assert st == mg.MG_OK
    assert rel(got, ref) < 1e-10
    fl = floor_of(ref, rho, gauge_free)
    assert len(gh) == len(rh)
    for a, b in zip(gh, rh):
        assert abs(a - b) <= 1e-6 * b + 10 * fl, (gh, rh)


@pytest.mark.parametrize("kinds", ["periodic", [FIXED] * 6])
def test_blocks_match_dense_gpu(mg, kinds):
    print(f"blocks vs dense kinds={kinds}", flush=True)
    n = 128
    rho = wl.gaussian_clumps(n, 3, remove_mean=kinds == "periodic")
    dense, dh, dst = mg.solve(dev(rho), 1.0 / n, kinds, tol=1e-10)
    got, gh, st, _ = solve_blocks(mg, rho, kinds, 16, tol=1e-10)
    assert st == dst == mg.MG_OK
    assert len(gh) == len(dh)
    d = dense.cpu().numpy()
    assert rel(got, d) < 1e-11
    assert np.allclose(gh, dh, rtol=1e-6, atol=10 * floor_of(d, rho, kinds == "periodic"))


@pytest.mark.parametrize("kinds", ["periodic", [FIXED] * 6])
def test_blocks_mixed_precision(mg, kinds):
    print(f"blocks mixed kinds={kinds}", flush=True)
    n = 64
    rho = wl.gaussian_clumps(n, 8, remove_mean=kinds == "periodic")
    ref, _, _ = oracle.solve(rho, 1.0 / n, kinds, tol=1e-13, max_cycles=40)
    got, gh, st, _ = solve_blocks(mg, rho, kinds, 8, precision="mixed", tol=1e-11, max_cycles=40)
    assert st in (mg.MG_OK, mg.MG_STALLED)
    assert gh[-1] < 1e-10
    assert rel(got, ref) < 1e-10


def test_schedules_are_bitwise_identical(mg):
    """Every schedule (threads, blocks per workgroup, sweeps per launch) gives the same bits."""
    print("block schedules bitwise", flush=True)
    n, block_n = 64, 8
    rho = wl.gaussian_clumps(n, 21, remove_mean=False)
    faces = [np.full((n, n), 0.05)] * 6
    base_ctx = mg.Context(0)
    want, wh, _, wb = solve_blocks(mg, rho, [FIXED] * 6, block_n, faces=faces, ctx=base_ctx, fixed_cycles=3)
    Lb = 3  # 8 blocks per side
    schedules = []
    for S in (1, 2):
        for threads in (256, 1024):
            for G in (1, 4):
                schedules.append((threads, G, S))
    for threads, G, S in schedules:
        ctx = mg.Context(0)
        text = "".join(f"blk fp64 {Lm} {Lb} {threads} {G} {S}\n" for Lm in (1, 2, 3))
        ctx.set_tuning(text)
        _, gh, _, gb = solve_blocks(mg, rho, [FIXED] * 6, block_n, faces=faces, ctx=ctx, fixed_cycles=3)
        assert torch.equal(gb, wb), (threads, G, S)
        assert list(gh) == list(wh)


def test_autotune_runs_and_keeps_results(mg, tmp_path):
    print("autotune", flush=True)
    n, block_n = 64, 16
    ctx = mg.Context(0)
    cache = str(tmp_path / "tune.json")
    text = ctx.autotune(n, block_n, "fp64", reps=2, cache=cache)
    lines = [l.split() for l in text.strip().splitlines()]
    assert {int(l[2]) for l in lines} == {1, 2, 3, 4}
    ctx2 = mg.Context(0)
    assert ctx2.autotune(n, block_n, "fp64", cache=cache) == text   # from the cache
    rho = wl.gaussian_clumps(n, 2)
    a, ah, _, ab = solve_blocks(mg, rho, "periodic", block_n, ctx=ctx, fixed_cycles=3)
    b, bh, _, bb = solve_blocks(mg, rho, "periodic", block_n, fixed_cycles=3)
    assert torch.equal(ab, bb)


def test_bad_schedule_rejected(mg):
    ctx = mg.Context(0)
    with pytest.raises(mg.MgError):
        ctx.set_tuning("blk fp64 4 4 512 4096 1\n")   # far beyond the LDS of a workgroup
    with pytest.raises(mg.MgError):
        ctx.set_tuning("blk fp64 4 4 300 1 1\n")


@pytest.mark.parametrize("n,block_n,tuning", [(32, 8, ""), (64, 16, ""), (128, 16, "fusedmin fp64 64\n")])
def test_blocks_multipole_matches_oracle(mg, n, block_n, tuning):
    """Multipole faces in the MeshBlock layout: the moments are summed over the blocks (cell
    positions from the block coordinates), the rest is the same V-cycle."""
    print(f"blocks multipole n={n} block_n={block_n}", flush=True)
    rho, _ = wl.uniform_sphere(n, 5)
    ref, rh, _ = oracle.solve(rho, 1.0 / n, [MULTIPOLE] * 6, fixed_cycles=5, lmax=4)
    ctx = mg.Context(0)
    if tuning:
        ctx.set_tuning(tuning)
    got, gh, st, _ = solve_blocks(mg, rho, "multipole", block_n, ctx=ctx, fixed_cycles=5, lmax=4)
    assert st == mg.MG_OK
    assert rel(got, ref) < 1e-10
    fl = floor_of(ref, rho, False)
    for a, b in zip(gh, rh):
        assert abs(a - b) <= 1e-6 * b + 10 * fl, (gh, rh)


def test_c4_lognormal_256_blocks_vs_oracle(mg):
    """Configuration 4 at full size: 256^3 = 4096 MeshBlocks of 16^3, lognormal field
    exp(GRF, P ~ k^-4), periodic.  FP64 against the oracle at its own cycle count to 1e-10:
    phi (relative L2 and element-wise) and the residual history cycle by cycle; mixed precision
    against the oracle converged to its round-off floor, to 1e-10; both also against the dense
    GPU solve."""
    print("C4 256^3 blocks", flush=True)
    n = 256
    rho = wl.lognormal_grf(n, 4)
    rho = rho - rho.mean()
    ref, rh, rst = oracle.solve(rho, 1.0 / n, "periodic", tol=1e-10)
    assert rst == oracle.OK
    cycles = len(rh) - 1
    print(f"C4 oracle: {cycles} cycles to {rh[-1]:.2e}", flush=True)
    got, gh, st, _ = solve_blocks(mg, rho, "periodic", 16, tol=1e-10)
    assert st == mg.MG_OK and len(gh) == len(rh), (gh, rh)
    assert rel(got, ref) < 1e-10, rel(got, ref)
    fl = floor_of(ref, rho, True)
    for a, b in zip(gh, rh):
        assert abs(a - b) <= 1e-6 * b + 10 * fl, (gh, rh)
    dense, dh, _ = mg.solve(dev(rho), 1.0 / n, "periodic", tol=1e-10)
    assert rel(got, dense.cpu().numpy()) < 1e-11
    del dense
    conv, ch, _ = oracle.solve(rho, 1.0 / n, "periodic", tol=1e-13, max_cycles=40)
    print(f"C4 oracle converged: {len(ch) - 1} cycles to {ch[-1]:.2e}", flush=True)
    mixed, mh, mst, _ = solve_blocks(mg, rho, "periodic", 16, precision="mixed", tol=1e-11, max_cycles=40)
    assert mst == mg.MG_OK and mh[-1] <= 1e-11, (mst, mh)
    assert len(mh) - 1 <= cycles + 2, (mh, rh)     # FP32 inner cycles contract like FP64 ones
    assert rel(mixed, conv) < 1e-10, rel(mixed, conv)


@pytest.mark.parametrize("n,block_n,kinds", [c for c in CASES if c[0] >= 64])
def test_blocks_streaming_passes_match_oracle(mg, n, block_n, kinds):
    """The streaming z-marching passes run across block boundaries (forced down to 64^3 here;
    they need at least 64 cells per side): the same V-cycles as the oracle."""
    print(f"blocks z-march vs oracle n={n} block_n={block_n} kinds={kinds}", flush=True)
    periodic_all = kinds == "periodic"
    rho = wl.gaussian_clumps(n, 7 + n + block_n, n_clumps=8, remove_mean=periodic_all)
    gauge_free = periodic_all or kinds == [ZERO_GRADIENT] * 6
    faces = None
    if not gauge_free:
        rng = np.random.default_rng(n * block_n)
        faces = [rng.normal(size=(n, n)) * 0.1 for _ in range(6)]
    ref, rh, rst = oracle.solve(rho, 1.0 / n, kinds, fixed_b=faces, fixed_cycles=5)
    ctx = mg.Context(0)
    ctx.set_tuning("fusedmin fp64 64\nblkz fp64 1\n")
    got, gh, st, _ = solve_blocks(mg, rho, kinds, block_n, faces=faces, ctx=ctx, fixed_cycles=5)
    assert st == mg.MG_OK
    assert rel(got, ref) < 1e-10
    fl = floor_of(ref, rho, gauge_free)
    for a, b in zip(gh, rh):
        assert abs(a - b) <= 1e-6 * b + 10 * fl, (gh, rh)


def test_blocks_streaming_mixed(mg):
    n = 128
    rho = wl.gaussian_clumps(n, 17, remove_mean=True)
    ref, _, _ = oracle.solve(rho, 1.0 / n, "periodic", tol=1e-13, max_cycles=40)
    ctx = mg.Context(0)
    ctx.set_tuning("fusedmin fp32 64\nblkz fp32 1\n")
    got, gh, st, _ = solve_blocks(mg, rho, "periodic", 16, ctx=ctx, precision="mixed", tol=1e-11, max_cycles=40)
    assert gh[-1] < 1e-10
    assert rel(got, ref) < 1e-10
