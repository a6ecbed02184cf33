"""mg_solve_noalloc (the solve in the library's static device scratch, for callers that cannot
allocate) against mg_solve through the C ABI: the same inputs give the same phi and residual
history, bitwise (the same kernels and reductions in the same order).  Two calls in a row,
the second smaller, so the second runs on scratch the first left behind; a solve beyond the
scratch's limit is refused without writing anything."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mg():
    import paper_2302_13903_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def pair(mg, ctx, n, bc, precision, seed, **kw):
    """Both entry points on one input: returns (phi, hist, status) of each."""
    remove = bc == "periodic"
    rho = dev(wl.gaussian_clumps(n, seed, remove_mean=remove))
    p = mg.params(n, 1.0 / n, precision=precision, tol=1e-10, **kw)
    b = mg.boundary(bc, None, 4)
    phi_a = torch.full_like(rho, 3.0)
    st_a, h_a = mg.mg_solve(ctx, p, b, rho, phi_a)
    phi_b = torch.full_like(rho, -5.0)
    st_b, h_b = mg.mg_solve_noalloc(ctx, p, b, rho, phi_b)
    torch.cuda.synchronize()
    return (phi_a, h_a, st_a), (phi_b, h_b, st_b)


@pytest.mark.parametrize("first,second", [
    ((128, "periodic", "fp64", {}), (64, "fixed", "fp64", {})),
    ((128, "multipole", "mixed", {}), (32, "periodic", "mixed", {})),
    ((128, "periodic", "fp64", dict(layout="blocks", block_n=16)), (64, "zero_gradient", "fp64", dict(scheme="fas"))),
])
def test_noalloc_equals_mg_solve(mg, first, second):
    print(f"noalloc {first} then {second}", flush=True)
    ctx = mg.Context(0)
    for k, (n, bc, prec, kw) in enumerate((first, second)):
        if kw.get("layout") == "blocks":
            # the MeshBlock layout takes rho and phi in Morton block order
            rho_d = wl.gaussian_clumps(n, 40 + k, remove_mean=bc == "periodic")
            rho = mg.to_blocks(dev(rho_d), kw["block_n"])
            p = mg.params(n, 1.0 / n, precision=prec, tol=1e-10, **kw)
            b = mg.boundary(bc, None, 4)
            phi_a, phi_b = torch.zeros_like(rho), torch.full_like(rho, 9.0)
            st_a, h_a = mg.mg_solve(ctx, p, b, rho, phi_a)
            st_b, h_b = mg.mg_solve_noalloc(ctx, p, b, rho, phi_b)
            torch.cuda.synchronize()
            a, b_ = (phi_a, h_a, st_a), (phi_b, h_b, st_b)
        else:
            a, b_ = pair(mg, ctx, n, bc, prec, 40 + k, **kw)
        assert a[2] == b_[2] == mg.MG_OK, (a[2], b_[2])
        assert a[1] == b_[1], (a[1], b_[1])
        assert torch.equal(a[0], b_[0]), float((a[0] - b_[0]).abs().max())


def test_noalloc_refuses_beyond_the_scratch(mg):
    n = 256
    ctx = mg.Context(0)
    rho = dev(np.zeros((n,) * 3))
    phi = torch.full_like(rho, 2.0)
    with pytest.raises(mg.MgError, match="OOM.*static scratch"):
        mg.mg_solve_noalloc(ctx, mg.params(n, 1.0 / n), mg.boundary("periodic"), rho, phi)
    torch.cuda.synchronize()
    assert float(phi.min()) == float(phi.max()) == 2.0     # nothing written
