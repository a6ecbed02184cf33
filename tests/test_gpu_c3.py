"""Configuration 3 at full size: the 512^3 uniform sphere (radius 0.25, centre offset by a
seeded |delta| <= 0.05, sub-cell volume fractions on cut cells; Sec. 4.2) with fixed faces
(the analytic potential at the face centres) and with multipole faces (l <= 4, App. A), in
FP64 and mixed precision, solved to a relative residual of 1e-10.

Checks: phi against the exact discrete solution of the same boundary values (the oracle's
spectral solve; for multipole faces with the face values the oracle's own expansion gives),
against the analytic potential (discretisation error only), and mixed against FP64."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import FIXED, MULTIPOLE
from oracle import exact as ex

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N = 512
R = 0.25


@pytest.fixture(scope="module")
def mg():
    import paper_2302_13903_amd as m
    return m


@pytest.fixture(scope="module")
def sphere():
    print("C3: building the 512^3 sphere", flush=True)
    rho, centre = wl.uniform_sphere(N, 3, radius=R)
    return rho, centre


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


from parity import rel, rel_l2  # noqa: E402  (relative L2 and element-wise bounds together)


def analytic(centre):
    x = wl.cell_centres(N)
    return wl.sphere_potential(x[None, None, :], x[None, :, None], x[:, None, None], centre, R,
                               4.0 / 3.0 * math.pi * R ** 3)


@pytest.mark.parametrize("kind", ["fixed", "multipole"])
def test_c3_sphere_512(mg, sphere, kind):
    rho, centre = sphere
    h = 1.0 / N
    mass = 4.0 / 3.0 * math.pi * R ** 3
    if kind == "fixed":
        faces = wl.sphere_face_values(N, centre, R, mass)
    else:
        # the oracle's own expansion about the centre of mass, evaluated at the face centres
        st = oracle.State(rho, h, [MULTIPOLE] * 6, lmax=4)
        faces = [st.face(st.levels(), f)[1:-1, 1:-1].copy() for f in range(6)]
        del st
    print(f"C3 {kind}: exact discrete solution", flush=True)
    exact = ex.spectral_solve(4.0 * math.pi * rho, h, [FIXED] * 6, faces)
    phi_a = analytic(centre)
    dfaces = [dev(b) for b in faces] if kind == "fixed" else None
    out, ncyc = {}, {}
    for prec in ("fp64", "mixed"):
        print(f"C3 {kind} {prec}: GPU solve", flush=True)
        phi, hist, status = mg.solve(dev(rho), h, kind, fixed_b=dfaces, lmax=4, tol=1e-10, precision=prec)
        torch.cuda.synchronize()
        assert status == mg.MG_OK, (prec, hist)
        assert hist[-1] <= 1e-10
        out[prec] = phi.cpu().numpy()
        ncyc[prec] = len(hist) - 1
        e_exact = rel(out[prec], exact)
        e_analytic = rel_l2(out[prec], phi_a)
        print(f"C3 {kind} {prec}: cycles {len(hist) - 1}, vs exact {e_exact:.2e}, vs analytic {e_analytic:.2e}",
              flush=True)
        assert e_exact < 1e-10, (prec, e_exact)
        # second-order discretisation error of the sphere at h = 1/512 (and, for multipole
        # faces, the truncation of the expansion, which vanishes outside a sphere)
        assert e_analytic < 3e-6, (prec, e_analytic)
    assert rel(out["mixed"], out["fp64"]) < 1e-10
    # the mixed form's outer steps (1..3 FP32 V-cycles each) contract at least like FP64
    # V-cycles (no stall, at most one step more)
    assert ncyc["mixed"] <= ncyc["fp64"] + 1, ncyc
