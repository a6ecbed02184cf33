"""Operator parity at the benchmark size (512^3), element by element against the oracle, with
the launch shapes the solver uses there: two sweeps, the down step (two sweeps, restricted
defect, cleared coarse correction) under both defect schedules, and the up step (trilinear
correction entering with the first of two sweeps).  Mixed boundary kinds: periodic in x,
fixed in y, zero-gradient in z."""
import numpy as np
import pytest

import oracle
from oracle import FIXED, PERIODIC, ZERO_GRADIENT

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N = 512
KINDS = [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, ZERO_GRADIENT]
HOM = [PERIODIC, PERIODIC, FIXED, FIXED, ZERO_GRADIENT, ZERO_GRADIENT]
TOL = 1e-13


@pytest.fixture(scope="module")
def mg():
    import paper_2302_13903_amd as m
    return m


@pytest.fixture(scope="module")
def data():
    rng = np.random.default_rng(512)
    u = rng.standard_normal((N,) * 3)
    f = rng.standard_normal((N,) * 3) * N * N
    bext = [rng.standard_normal((N + 2, N + 2)) if KINDS[q] == FIXED else None for q in range(6)]
    return u, f, bext


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def dbext(bext):
    return [None if b is None else dev(b) for b in bext]


def close(a, b, scale):
    return float(np.max(np.abs(a - b))) <= TOL * scale


def test_two_sweeps_512(mg, data):
    print("512^3 two sweeps", flush=True)
    u, f, bext = data
    h = 1.0 / N
    ref = oracle.smooth(oracle.smooth(u, f, h, 1.15, KINDS, bext), f, h, 1.15, KINDS, bext)
    du = dev(u)
    mg.mg_op_smooth(du, dev(f), h, 1.15, 2, KINDS, dbext(bext))
    assert close(host(du), ref, np.abs(ref).max())


@pytest.mark.parametrize("split", [1, 0])
def test_down_512(mg, data, split):
    print(f"512^3 down split={split}", flush=True)
    u, f, bext = data
    h = 1.0 / N
    ref = oracle.smooth(oracle.smooth(u, f, h, 1.15, KINDS, bext), f, h, 1.15, KINDS, bext)
    ref_fc = oracle.restrict(oracle.defect(ref, f, h, KINDS, bext))
    ctx = mg.Context(0)
    ctx.set_tuning(f"pass fp64 9 {split}\n")
    du = dev(u)
    fc = torch.full((N // 2,) * 3, 7.0, dtype=torch.float64, device="cuda:0")
    uc = torch.full((N // 2,) * 3, 7.0, dtype=torch.float64, device="cuda:0")
    mg.mg_op_down(du, dev(f), fc, uc, h, 1.15, 2, KINDS, dbext(bext), ctx=ctx)
    assert close(host(du), ref, np.abs(ref).max())
    assert close(host(fc), ref_fc, np.abs(f).max() + 12 * np.abs(ref).max() / h ** 2)
    assert float(uc.abs().max()) == 0.0


def test_up_512(mg, data):
    print("512^3 up", flush=True)
    u, f, bext = data
    h = 1.0 / N
    rng = np.random.default_rng(9)
    e = rng.standard_normal((N // 2,) * 3)
    ref = oracle.prolong_add(e, u, HOM)
    ref = oracle.smooth(oracle.smooth(ref, f, h, 1.15, KINDS, bext), f, h, 1.15, KINDS, bext)
    du = dev(u)
    mg.mg_op_up(du, dev(f), dev(e), h, 1.15, 2, KINDS, dbext(bext), kinds_coarse=HOM)
    assert close(host(du), ref, np.abs(ref).max())
