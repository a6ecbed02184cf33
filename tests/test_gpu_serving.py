"""Serving runtime on the GPU: a request's result does not depend on what runs beside it
(alone == in-mix, bitwise: every kernel and reduction is deterministic), the server's solve is
the plain mg_solve, and resident hierarchies are reused across requests."""
import numpy as np
import pytest

import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2302_13903_amd as mg  # noqa: E402
from paper_2302_13903_amd import serving  # noqa: E402
from paper_2302_13903_amd._abi import MG_ERR_INVALID_ARG  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def clumps(n, seed, remove_mean):
    return dev(wl.gaussian_clumps(n, seed, remove_mean=remove_mean))


CASES = [  # (n, bc, precision)
    (64, "periodic", "fp64"),
    (128, "fixed", "fp64"),
    (64, "multipole", "mixed"),
    (128, "periodic", "mixed"),
    (64, "zero_gradient", "fp64"),
]


def make_requests(rhos, phis):
    return [serving.Request(rho=rhos[i], bc=bc, precision=prec, phi=phis[i], want_hist=True, tol=1e-10)
            for i, (n, bc, prec) in enumerate(CASES)]


def test_alone_equals_in_mix_bitwise():
    print("serving alone vs mix", flush=True)
    rhos = [clumps(n, 100 + i, bc == "periodic") for i, (n, bc, _) in enumerate(CASES)]
    alone_phi = [torch.zeros_like(r) for r in rhos]
    srv1 = serving.Server(workers=1)
    alone = []
    for i in range(len(CASES)):
        rq = make_requests(rhos, alone_phi)[i]
        srv1.run([rq])
        assert rq.status >= 0, (CASES[i], rq.status)
        alone.append(rq)
    torch.cuda.synchronize()
    mix_phi = [torch.full_like(r, 7.0) for r in rhos]
    mix = make_requests(rhos, mix_phi)
    fill = [serving.Request(rho=clumps(256, 7, True), bc="periodic"),
            serving.Request(rho=clumps(128, 8, False), bc="multipole", precision="mixed"),
            serving.Request(rho=clumps(256, 9, True), bc="periodic", precision="mixed")]
    for k, r in enumerate(fill):
        r.arrival_ms = 0.0
    for k, r in enumerate(mix):
        r.arrival_ms = 1.0 * k
    srv4 = serving.Server(workers=4)
    out = srv4.run(fill + mix)
    assert all(r.status == 0 for r in out), [r.status for r in out]
    assert srv4.stats()["max_concurrent"] >= 2
    for i, (a, b) in enumerate(zip(alone, mix)):
        assert a.hist == b.hist, CASES[i]
        assert torch.equal(alone_phi[i], mix_phi[i]), CASES[i]


def test_server_matches_direct_solve():
    """A served solve equals a direct solve on a context with the server's settings (its
    contexts run every pass as one launch: "split fp64 0"), bitwise, history included."""
    print("serving vs direct", flush=True)
    rho = clumps(128, 3, False)
    ctx = mg.Context(0)
    ctx.set_tuning("split fp64 0\n")
    phi_d, hist_d, st_d = mg.solve(rho, 1.0 / 128, "multipole", tol=1e-10, ctx=ctx)
    phi_s = torch.zeros_like(rho)
    srv = serving.Server(workers=2)
    (r,) = srv.run([serving.Request(rho=rho, bc="multipole", phi=phi_s, want_hist=True)])
    assert r.status == st_d
    assert r.hist == hist_d
    assert torch.equal(phi_s, phi_d)


def test_reuse_and_repeat_are_identical():
    print("serving reuse", flush=True)
    rho = clumps(64, 4, True)
    srv = serving.Server(workers=2)
    phis = [torch.zeros_like(rho) for _ in range(4)]
    # a 128^3 request between dirties nothing it shares: hierarchies are per (n, precision)
    rs = [serving.Request(rho=rho, phi=phis[0]), serving.Request(rho=clumps(128, 5, True), arrival_ms=0.0),
          serving.Request(rho=rho, phi=phis[1], arrival_ms=5.0)]
    srv.run(rs)
    srv.run([serving.Request(rho=rho, phi=phis[2]), serving.Request(rho=rho, phi=phis[3])])
    assert all(r.status == 0 for r in rs)
    for p in phis[1:]:
        assert torch.equal(p, phis[0])
    st = srv.stats()
    assert st["reused"] >= 2 and st["created"] <= 4


def test_mgi_without_phi_is_an_error():
    rho = clumps(32, 6, True)
    srv = serving.Server(workers=1)
    (r,) = srv.run([serving.Request(rho=rho, mode="mgi")])
    assert r.status == MG_ERR_INVALID_ARG


def test_admission_under_a_small_budget():
    """A budget of about two 128^3 hierarchies: 256^3 requests are rejected, 64^3 and 128^3
    ones are served with hierarchies created, reused and evicted on the device while other
    workers solve; every served result equals the direct solve."""
    print("serving small budget", flush=True)
    fp128 = mg.mg_footprint_bytes(mg.params(128, 1 / 128)) + 128 ** 3 * 8 + 256
    srv = serving.Server(workers=3, hbm_budget=int(2.5 * fp128))
    rhos = {64: clumps(64, 31, True), 128: clumps(128, 32, True), 256: clumps(256, 33, True)}
    want = {n: mg.solve(rhos[n], 1.0 / n, "periodic")[0] for n in (64, 128)}
    sizes = [128, 64, 256, 128, 64, 128, 64, 128]
    phis = [torch.zeros_like(rhos[n]) for n in sizes]
    reqs = [serving.Request(rho=rhos[n], phi=phis[i], arrival_ms=0.5 * i) for i, n in enumerate(sizes)]
    srv.run(reqs)
    st = srv.stats()
    assert reqs[2].status == mg._abi.MG_ERR_OOM
    for i, r in enumerate(reqs):
        if sizes[i] == 256:
            continue
        assert r.status == 0, (i, r.status)
        assert torch.equal(phis[i], want[sizes[i]]), i
    assert st["rejected"] == 1 and st["peak_bytes"] <= int(2.5 * fp128)
    assert st["created"] >= 2


def test_served_results_match_the_oracle():
    """Per-request oracle check of a served mix: every boundary kind of the request stream
    (periodic, fixed b = 0, multipole l <= 4) at 64^3 and 128^3 in both precisions, served
    together by four workers.  FP64 requests equal the oracle at their own cycle count (phi to
    1e-10, relative L2 and element-wise; histories cycle by cycle); mixed-precision requests
    equal the oracle converged to its round-off floor (phi to 1e-10)."""
    import math

    import oracle
    from parity import rel
    print("serving vs oracle", flush=True)
    cases = [(n, bc, prec) for n in (64, 128) for bc in ("periodic", "fixed", "multipole")
             for prec in ("fp64", "mixed")]
    rhos_h = [wl.gaussian_clumps(n, 300 + i, remove_mean=bc == "periodic") for i, (n, bc, _) in enumerate(cases)]
    rhos = [dev(r) for r in rhos_h]
    phis = [torch.zeros_like(r) for r in rhos]
    reqs = [serving.Request(rho=rhos[i], bc=bc, precision=prec, phi=phis[i], want_hist=True,
                            tol=1e-10 if prec == "fp64" else 1e-11, arrival_ms=0.5 * i)
            for i, (n, bc, prec) in enumerate(cases)]
    srv = serving.Server(workers=4)
    srv.run(reqs)
    torch.cuda.synchronize()
    assert srv.stats()["max_concurrent"] >= 2
    for i, (n, bc, prec) in enumerate(cases):
        r = reqs[i]
        assert r.status == 0, (cases[i], r.status, r.hist)
        got = phis[i].cpu().numpy()
        if prec == "fp64":
            ref, rh, _ = oracle.solve(rhos_h[i], 1.0 / n, bc, fixed_cycles=len(r.hist) - 1)
            f = 4 * math.pi * rhos_h[i]
            if bc == "periodic":
                f = f - f.mean()
            floor = 12 * np.finfo(float).eps * np.abs(ref).max() * n * n / math.sqrt(np.mean(f * f))
            for a, b in zip(r.hist, rh):
                assert abs(a - b) <= 1e-6 * b + 10 * floor, (cases[i], r.hist, rh)
        else:
            ref, rh, _ = oracle.solve(rhos_h[i], 1.0 / n, bc, tol=1e-13, max_cycles=40)
        err = rel(got, ref)
        print(f"served {cases[i]}: cycles {len(r.hist) - 1}, vs oracle {err:.2e}", flush=True)
        assert err < 1e-10, (cases[i], err)
