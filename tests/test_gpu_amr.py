"""GPU parity of the refined-mesh solver (Sec. 3.3: FAS V-cycles over MeshBlock, Octet and root
levels with the conservative and normal level boundaries) with the oracle: residual histories
cycle by cycle and the potential on every patch to 1e-10 relative, for one and two levels of
refinement, off-centre and non-cubic boxes, periodic, zero-gradient, fixed and multipole faces,
zero and random initial guesses and the full-multigrid start; plus the rejected forms."""
import math

import numpy as np
import pytest

from oracle import amr

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mg():
    import paper_2302_13903_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


MESHES = {
    "one level": (4, 4, [((1, 1, 1), (3, 3, 3))]),
    "two levels": (4, 4, [((1, 1, 1), (3, 3, 3)), ((3, 3, 3), (5, 5, 5))]),
    "off-centre, non-cubic": (4, 2, [((1, 2, 1), (3, 3, 2))]),
    "larger": (8, 8, [((2, 3, 3), (6, 5, 5))]),
}
KINDS = {"periodic": [amr.PERIODIC] * 6, "fixed": [amr.FIXED] * 6, "zero_gradient": [amr.ZERO_GRADIENT] * 6,
         "mixed": [amr.PERIODIC, amr.PERIODIC, amr.FIXED, amr.FIXED, amr.ZERO_GRADIENT, amr.ZERO_GRADIENT]}


def case(NB, nb, boxes, kinds, seed):
    m = amr.AmrMesh(NB, nb, boxes)
    rho = []
    for l in range(m.Lam + 1):
        x, y, z = m.centres(l)
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        r2 = (X - 0.55) ** 2 + (Y - 0.45) ** 2 + (Z - 0.5) ** 2
        rho.append(np.exp(-r2 / (2 * 0.08 ** 2)) + 0.3 * np.sin(2 * math.pi * X))
    N = NB * nb
    rng = np.random.default_rng(seed)
    faces = [rng.uniform(-0.5, 0.5, (N, N)) if k == amr.FIXED else None for k in kinds]
    return m, rho, faces


from parity import rel, rel_l2  # noqa: E402  (relative L2 and element-wise bounds together)


@pytest.mark.parametrize("kname", list(KINDS))
@pytest.mark.parametrize("mname", list(MESHES))
def test_amr_matches_oracle(mg, mname, kname):
    NB, nb, boxes = MESHES[mname]
    kinds = KINDS[kname]
    print(f"amr {mname} {kname}", flush=True)
    m, rho, faces = case(NB, nb, boxes, kinds, 5)
    bf = amr.FaceArrays([f if f is not None else np.zeros((NB * nb,) * 2) for f in faces]) \
        if any(f is not None for f in faces) else None
    ref, rh = amr.solve(m, rho, kinds, bf, cycles=5)
    mesh = mg.amr_mesh(NB, nb, boxes)
    for l in range(m.Lam + 1):
        assert mg.amr_patch_dims(mesh, l) == m.patches[l][m.K].n
    phi, hist, st = mg.amr_solve(mesh, [dev(r) for r in rho], kinds,
                                 fixed_b=[None if f is None else dev(f) for f in faces], fixed_cycles=5)
    torch.cuda.synchronize()
    got = [p.cpu().numpy() for p in phi]
    assert st == mg.MG_OK and len(hist) == len(rh) == 6
    for a, b in zip(hist, rh):
        assert abs(a - b) <= 1e-6 * b + 1e-12, (hist, rh)
    assert rel(got, ref) < 1e-10
    # covered cells are zero on output
    for l in range(m.Lam):
        (x0, y0, z0), (x1, y1, z1) = m.patches[l][m.K].hole
        assert float(np.abs(got[l][z0:z1, y0:y1, x0:x1]).max()) == 0.0


@pytest.mark.parametrize("kname", ["periodic", "fixed", "mixed"])
@pytest.mark.parametrize("mname", list(MESHES))
def test_amr_fmg_matches_oracle(mg, mname, kname):
    """Full multigrid on the refined hierarchy (sources on every level, root, Octet and
    MeshBlock stages each from the tricubic prolongation below) and 3 V-cycles: the residual
    after FMG and after each cycle, and the potential, as the oracle's."""
    NB, nb, boxes = MESHES[mname]
    kinds = KINDS[kname]
    print(f"amr fmg {mname} {kname}", flush=True)
    m, rho, faces = case(NB, nb, boxes, kinds, 6)
    bf = amr.FaceArrays([f if f is not None else np.zeros((NB * nb,) * 2) for f in faces]) \
        if any(f is not None for f in faces) else None
    ref, rh = amr.solve(m, rho, kinds, bf, cycles=3, mode="fmg")
    phi, hist, st = mg.amr_solve(mg.amr_mesh(NB, nb, boxes), [dev(r) for r in rho], kinds,
                                 fixed_b=[None if f is None else dev(f) for f in faces], fixed_cycles=3, mode="fmg")
    torch.cuda.synchronize()
    assert st == mg.MG_OK and len(hist) == len(rh) == 4
    if kname == "periodic":
        # (the fixed cases carry random face values that no coarse level can represent, so
        # their FMG start stays near 1, on both sides)
        assert hist[0] < 0.1
    for a, b in zip(hist, rh):
        assert abs(a - b) <= 1e-6 * b + 1e-12, (hist, rh)
    assert rel([p.cpu().numpy() for p in phi], ref) < 1e-10


def test_amr_warm_start_and_tolerance(mg):
    """From a random initial guess, to tolerance: same cycle count and potential as the oracle."""
    NB, nb, boxes = MESHES["two levels"]
    kinds = KINDS["fixed"]
    m, rho, faces = case(NB, nb, boxes, kinds, 9)
    rng = np.random.default_rng(3)
    phi0 = [rng.uniform(-1, 1, m.patches[l][m.K].n[::-1]) for l in range(m.Lam + 1)]
    bf = amr.FaceArrays(faces)
    ref, rh = amr.solve(m, rho, kinds, bf, phi0=phi0, tol=1e-10)
    mesh = mg.amr_mesh(NB, nb, boxes)
    phi, hist, st = mg.amr_solve(mesh, [dev(r) for r in rho], kinds, fixed_b=[dev(f) for f in faces],
                                 phi=[dev(p) for p in phi0], tol=1e-10)
    assert st == mg.MG_OK and len(hist) == len(rh)
    assert rel([p.cpu().numpy() for p in phi], ref) < 1e-10


def test_amr_rejected_forms(mg):
    NB, nb, boxes = MESHES["one level"]
    m, rho, _ = case(NB, nb, boxes, KINDS["periodic"], 1)
    r = [dev(x) for x in rho]
    mesh = mg.amr_mesh(NB, nb, boxes)
    ctx = mg.Context(0)
    p = mg.params(NB * nb, 1.0 / (NB * nb), mode="mgi", precision="mixed")
    with pytest.raises(mg.MgError, match="UNSUPPORTED"):
        mg.mg_amr_solve(ctx, p, mesh, mg.boundary("periodic"), r, [torch.zeros_like(x) for x in r])
    with pytest.raises(mg.MgError, match="INVALID_ARG"):
        mg.amr_solve(mesh, r, "multipole", lmax=5)
    with pytest.raises(mg.MgError, match="INVALID_ARG"):
        mg.amr_patch_dims(mg.amr_mesh(4, 4, [((0, 1, 1), (3, 3, 3))]), 1)    # touches the domain face
    with pytest.raises(mg.MgError, match="INVALID_ARG"):
        mg.amr_patch_dims(mg.amr_mesh(4, 4, [((1, 1, 1), (3, 3, 3)), ((2, 3, 3), (5, 5, 5))]), 2)  # no margin


def test_binary_potential(mg):
    """The paper's refined-mesh test (Sec. 4.3) at root resolution 1/64 with four nested levels
    (1/1024 at the stars): FMG and 3 V-cycles as the oracle's, then to 1e-10 with the
    normalised error against the analytic potential below 1e-3."""
    import workloads as wl
    print("amr binary", flush=True)
    NB, nb = 4, 16
    boxes = wl.binary_mesh_boxes(NB)
    m = amr.AmrMesh(NB, nb, boxes)
    rho = [wl.binary_density_on_axes(*m.centres(l), m.patches[l][m.K].h) for l in range(m.Lam + 1)]
    N = NB * nb
    x = (np.arange(N) + 0.5) / N
    faces = []
    for face in range(6):
        axis, side = face // 2, face % 2
        t = [q for q in range(3) if q != axis]
        co = [None, None, None]
        co[axis] = np.array(0.0 if side == 0 else 1.0)
        co[t[0]] = x[None, :]
        co[t[1]] = x[:, None]
        faces.append(np.array(np.broadcast_to(wl.binary_potential(*co), (N, N))))
    ref, rh = amr.solve(m, rho, [amr.FIXED] * 6, amr.FaceArrays(faces), cycles=3, mode="fmg")
    mesh = mg.amr_mesh(NB, nb, boxes)
    drho = [dev(r) for r in rho]
    dfaces = [dev(f) for f in faces]
    phi, hist, st = mg.amr_solve(mesh, drho, "fixed", fixed_b=dfaces, fixed_cycles=3, mode="fmg")
    assert len(hist) == len(rh) == 4
    for a, b in zip(hist, rh):
        assert abs(a - b) <= 1e-6 * b + 1e-12, (hist, rh)
    assert rel([p.cpu().numpy() for p in phi], ref) < 1e-10
    phi, hist, st = mg.amr_solve(mesh, drho, "fixed", fixed_b=dfaces, tol=1e-10, mode="fmg")
    assert st == mg.MG_OK
    err = []
    for l in range(m.Lam + 1):
        xs, ys, zs = m.centres(l)
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        ex = wl.binary_potential(X, Y, Z)
        err.append(((phi[l].cpu().numpy() - ex) / ex)[m.patches[l][m.K].active()])
    e = np.concatenate(err)
    assert math.sqrt(np.mean(e * e)) < 1e-3


@pytest.mark.parametrize("mode", ["mgi", "fmg"])
@pytest.mark.parametrize("kname", ["periodic", "fixed"])
def test_amr_large_root_grid(mg, kname, mode):
    """A 32^3 root grid: its upper levels run one launch per operator, the levels from 16^3
    down in one workgroup; both as the oracle, cycle by cycle."""
    NB, nb, boxes = 32, 2, [((12, 13, 12), (20, 19, 21))]
    kinds = KINDS[kname]
    print(f"amr root 32^3 {kname} {mode}", flush=True)
    m, rho, faces = case(NB, nb, boxes, kinds, 8)
    bf = amr.FaceArrays(faces) if kname == "fixed" else None
    ref, rh = amr.solve(m, rho, kinds, bf, cycles=3, mode=mode)
    phi, hist, st = mg.amr_solve(mg.amr_mesh(NB, nb, boxes), [dev(r) for r in rho], kinds,
                                 fixed_b=[None if f is None else dev(f) for f in faces], fixed_cycles=3, mode=mode)
    torch.cuda.synchronize()
    assert st == mg.MG_OK and len(hist) == len(rh) == 4
    for a, b in zip(hist, rh):
        assert abs(a - b) <= 1e-6 * b + 1e-12, (hist, rh)
    assert rel([p.cpu().numpy() for p in phi], ref) < 1e-10


@pytest.mark.parametrize("mode", ["mgi", "fmg"])
def test_amr_six_levels(mg, mode):
    """Six nested refinement levels (seven patches per MeshBlock level in one batched launch,
    seven Octet levels in the single-workgroup middle of the cycle): as the oracle."""
    boxes, lo = [], 1
    for _ in range(6):
        boxes.append(((lo, lo, lo), (lo + 2, lo + 2, lo + 2)))
        lo = 2 * lo + 1
    NB, nb = 4, 4
    kinds = KINDS["mixed"]
    print(f"amr six levels {mode}", flush=True)
    m, rho, faces = case(NB, nb, boxes, kinds, 12)
    bf = amr.FaceArrays([f if f is not None else np.zeros((NB * nb,) * 2) for f in faces])
    ref, rh = amr.solve(m, rho, kinds, bf, cycles=3, mode=mode)
    phi, hist, st = mg.amr_solve(mg.amr_mesh(NB, nb, boxes), [dev(r) for r in rho], kinds,
                                 fixed_b=[None if f is None else dev(f) for f in faces], fixed_cycles=3, mode=mode)
    torch.cuda.synchronize()
    assert st == mg.MG_OK and len(hist) == len(rh) == 4
    for a, b in zip(hist, rh):
        assert abs(a - b) <= 1e-6 * b + 1e-12, (hist, rh)
    assert rel([p.cpu().numpy() for p in phi], ref) < 1e-10


MP_KINDS = {"multipole": ["multipole"] * 6,
            "mixed": ["multipole", "multipole", "periodic", "periodic", "multipole", "zero_gradient"]}


@pytest.mark.parametrize("origin", [None, (0.52, 0.47, 0.5)])
@pytest.mark.parametrize("kname", list(MP_KINDS))
@pytest.mark.parametrize("mname", list(MESHES))
def test_amr_multipole_matches_oracle(mg, mname, kname, origin):
    """Multipole faces (Appendix A) on the refined mesh: moments over the composite grid's
    active cells, faces at every root level's face centres; V-cycles and FMG as the oracle's."""
    NB, nb, boxes = MESHES[mname]
    names = MP_KINDS[kname]
    kinds = [amr.FIXED if k == "multipole" else amr.PERIODIC if k == "periodic" else amr.ZERO_GRADIENT
             for k in names]
    print(f"amr multipole {mname} {kname} {origin}", flush=True)
    m, rho, _ = case(NB, nb, boxes, kinds, 5)
    bf = amr.multipole_faces(m, rho, 4, None if origin is None else np.array(origin))
    mesh = mg.amr_mesh(NB, nb, boxes)
    drho = [dev(r) for r in rho]
    for mode, cyc in (("mgi", 5), ("fmg", 3)):
        ref, rh = amr.solve(m, rho, kinds, bf, cycles=cyc, mode=mode)
        phi, hist, st = mg.amr_solve(mesh, drho, names, fixed_cycles=cyc, mode=mode, origin=origin)
        torch.cuda.synchronize()
        assert st == mg.MG_OK and len(hist) == len(rh) == cyc + 1
        for a, b in zip(hist, rh):
            assert abs(a - b) <= 1e-6 * b + 1e-12, (mode, hist, rh)
        assert rel([p.cpu().numpy() for p in phi], ref) < 1e-10, mode


@pytest.mark.parametrize("lmax", [0, 2])
def test_amr_multipole_lower_orders(mg, lmax):
    """Multipole faces truncated below the hexadecapole on the refined mesh."""
    NB, nb, boxes = MESHES["two levels"]
    kinds = [amr.FIXED] * 6
    print(f"amr multipole lmax {lmax}", flush=True)
    m, rho, _ = case(NB, nb, boxes, kinds, 3)
    ref, rh = amr.solve(m, rho, kinds, amr.multipole_faces(m, rho, lmax), cycles=4)
    mesh = mg.amr_mesh(NB, nb, boxes)
    phi, hist, st = mg.amr_solve(mesh, [dev(r) for r in rho], "multipole", lmax=lmax, fixed_cycles=4)
    torch.cuda.synchronize()
    assert st == mg.MG_OK and len(hist) == len(rh) == 5
    for a, b in zip(hist, rh):
        assert abs(a - b) <= 1e-6 * b + 1e-12, (hist, rh)
    assert rel([p.cpu().numpy() for p in phi], ref) < 1e-10


def test_binary_potential_multipole(mg):
    """The paper's refined-mesh test with its own boundaries (Sec. 4.3: open faces from the
    hexadecapole expansion): FMG and 3 V-cycles as the oracle's, then to 1e-10 with the
    normalised error against the analytic potential below 1e-3."""
    import workloads as wl
    print("amr binary multipole", flush=True)
    NB, nb = 4, 16
    boxes = wl.binary_mesh_boxes(NB)
    m = amr.AmrMesh(NB, nb, boxes)
    rho = [wl.binary_density_on_axes(*m.centres(l), m.patches[l][m.K].h) for l in range(m.Lam + 1)]
    ref, rh = amr.solve(m, rho, [amr.FIXED] * 6, amr.multipole_faces(m, rho, 4), cycles=3, mode="fmg")
    mesh = mg.amr_mesh(NB, nb, boxes)
    drho = [dev(r) for r in rho]
    phi, hist, st = mg.amr_solve(mesh, drho, "multipole", fixed_cycles=3, mode="fmg")
    assert len(hist) == len(rh) == 4
    for a, b in zip(hist, rh):
        assert abs(a - b) <= 1e-6 * b + 1e-12, (hist, rh)
    assert rel([p.cpu().numpy() for p in phi], ref) < 1e-10
    phi, hist, st = mg.amr_solve(mesh, drho, "multipole", tol=1e-10, mode="fmg")
    assert st == mg.MG_OK
    err = []
    for l in range(m.Lam + 1):
        xs, ys, zs = m.centres(l)
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        ex = wl.binary_potential(X, Y, Z)
        err.append(((phi[l].cpu().numpy() - ex) / ex)[m.patches[l][m.K].active()])
    e = np.concatenate(err)
    assert math.sqrt(np.mean(e * e)) < 1e-3


def test_amr_workspace_kept_across_calls(mg):
    """The refined-mesh workspace belongs to the context: a small mesh, a larger one (the
    workspace grows) and the small one again on one context give bitwise the results of fresh
    contexts; a budget below the workspace's size is refused with MG_ERR_OOM."""
    def run(ctx, name):
        NB, nb, boxes = MESHES[name]
        m, rho, faces = case(NB, nb, boxes, KINDS["fixed"], 5)
        mesh = mg.amr_mesh(NB, nb, boxes)
        phi, hist, st = mg.amr_solve(mesh, [dev(r) for r in rho], KINDS["fixed"],
                                     fixed_b=[None if f is None else dev(f) for f in faces], fixed_cycles=3, ctx=ctx)
        torch.cuda.synchronize()
        assert st == mg.MG_OK
        return [p.cpu().numpy() for p in phi], hist

    shared = mg.Context(0)
    for name in ("one level", "larger", "one level"):
        print(f"amr workspace: {name}", flush=True)
        got, h = run(shared, name)
        ref, hr = run(mg.Context(0), name)
        assert h == hr
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
    small = mg.Context(0, hbm_budget=1 << 20)
    with pytest.raises(mg.MgError, match="OOM"):
        run(small, "larger")
