"""Scheduler of the serving runtime, run in simulate mode (no device work): admission by HBM
footprint, FIFO and skip-ahead policies, resident-hierarchy reuse and eviction, rejection,
open-loop arrivals.  The native scheduler is the same code that drives the GPU solves."""
import pytest

import paper_2302_13903_amd as mg
from paper_2302_13903_amd import serving
from paper_2302_13903_amd._abi import MG_ERR_OOM


def fp(n, precision="fp64"):
    """Bytes the server accounts per hierarchy: the solver footprint plus the result slot."""
    return mg.mg_footprint_bytes(mg.params(n, 1.0 / n, precision=precision)) + n ** 3 * 8 + 256


def req(n, sim_ms, arrival_ms=0.0, precision="fp64"):
    return serving.Request(n=n, sim_ms=sim_ms, arrival_ms=arrival_ms, precision=precision)


def overlaps(a, b):
    return a.start_ms < b.end_ms and b.start_ms < a.end_ms


def test_single_worker_is_fifo():
    srv = serving.Server(workers=1, hbm_budget=1 << 40, simulate=True)
    rs = srv.run([req(64, 5.0, arrival_ms=0.5 * i) for i in range(6)])
    assert all(r.status == 0 for r in rs)
    for a, b in zip(rs, rs[1:]):
        assert b.start_ms >= a.end_ms - 1e-6
    for r in rs:
        assert r.end_ms - r.start_ms >= 5.0 - 0.5
        assert r.start_ms >= r.arrival_ms - 1e-6


def test_workers_overlap_when_memory_allows():
    srv = serving.Server(workers=4, hbm_budget=1 << 40, simulate=True)
    rs = srv.run([req(128, 40.0) for _ in range(4)])
    assert srv.stats()["max_concurrent"] == 4
    assert sum(overlaps(rs[0], r) for r in rs[1:]) == 3


def test_admission_bounds_resident_bytes():
    # room for exactly two 256^3 hierarchies: at most two run at once with four workers
    budget = 2 * fp(256) + fp(256) // 2
    srv = serving.Server(workers=4, hbm_budget=budget, simulate=True)
    rs = srv.run([req(256, 20.0) for _ in range(6)])
    st = srv.stats()
    assert all(r.status == 0 for r in rs)
    assert st["max_concurrent"] == 2
    assert st["peak_bytes"] <= budget
    assert st["created"] == 2 and st["reused"] == 4
    # at every start instant at most two solves hold memory
    for r in rs:
        assert sum(o.start_ms <= r.start_ms < o.end_ms for o in rs) <= 2


def test_too_large_request_is_rejected_not_blocking():
    srv = serving.Server(workers=2, hbm_budget=fp(128) + 1024, simulate=True)
    rs = srv.run([req(512, 1.0), req(128, 2.0), req(128, 2.0)])
    assert rs[0].status == MG_ERR_OOM and rs[0].worker == -1
    assert rs[1].status == 0 and rs[2].status == 0
    assert srv.stats()["rejected"] == 1


def test_eviction_makes_room_for_another_size():
    budget = fp(256) + fp(64) // 2
    srv = serving.Server(workers=1, hbm_budget=budget, simulate=True)
    srv.run([req(256, 1.0), req(128, 1.0), req(256, 1.0)])
    st = srv.stats()
    # 256 resident -> evicted for 128 -> 128 evicted for 256 again
    assert st["created"] == 3 and st["evicted"] == 2
    assert st["peak_bytes"] <= budget


def test_resident_hierarchies_persist_across_runs():
    srv = serving.Server(workers=2, hbm_budget=1 << 40, simulate=True)
    srv.reserve(128, count=2)
    rs = srv.run([req(128, 1.0), req(128, 1.0)])
    assert all(r.reused for r in rs)
    rs = srv.run([req(128, 1.0)])
    assert rs[0].reused
    assert srv.stats()["created"] == 2


def test_precisions_are_separate_hierarchies():
    srv = serving.Server(workers=1, hbm_budget=1 << 40, simulate=True)
    srv.run([req(64, 1.0, precision="fp64"), req(64, 1.0, precision="mixed"), req(64, 1.0, precision="fp64")])
    st = srv.stats()
    assert st["created"] == 2 and st["reused"] == 1


def test_fifo_blocks_behind_head_skip_does_not():
    budget = fp(256) + fp(128) + 1024
    reqs = lambda: [req(256, 60.0), req(256, 5.0, arrival_ms=1.0), req(128, 5.0, arrival_ms=2.0)]
    fifo = serving.Server(workers=3, hbm_budget=budget, policy="fifo", simulate=True).run(reqs())
    # FIFO: the 128^3 request waits behind the second 256^3, which waits for the first
    assert fifo[2].start_ms >= fifo[1].start_ms - 1e-6
    assert fifo[2].start_ms >= 50.0
    skip = serving.Server(workers=3, hbm_budget=budget, policy="skip", simulate=True).run(reqs())
    assert skip[2].start_ms < 30.0
    assert skip[1].start_ms >= skip[0].end_ms - 1e-6


def test_open_loop_arrivals_and_summary():
    tr = [req(64, 1.0, arrival_ms=3.0 * i) for i in range(10)]
    srv = serving.Server(workers=2, hbm_budget=1 << 40, simulate=True)
    rs = srv.run(tr)
    for r in rs:
        assert r.start_ms >= r.arrival_ms - 1e-6
        assert 1.0 - 0.5 <= r.latency_ms < 50.0
    s = serving.summary(rs)
    assert s["completed"] == 10 and s["errors"] == 0
    assert s["latency_ms"]["p50"] <= s["latency_ms"]["p99"]
    assert s["makespan_ms"] >= 27.0


@pytest.mark.parametrize("bad", [dict(workers=0), dict(workers=65), dict(policy="lifo")])
def test_invalid_config(bad):
    kw = dict(workers=2, hbm_budget=1 << 30, simulate=True)
    kw.update(bad)
    with pytest.raises((mg.MgError, KeyError)):
        serving.Server(**kw)


def test_hierarchies_are_keyed_by_workspace_class():
    """Requests of one size but another layout or scheme need another workspace: each gets a
    hierarchy of its own class, accounted with its own footprint, and reuses only its class."""
    kinds = [dict(), dict(layout="blocks", block_n=16), dict(layout="blocks", block_n=8), dict(scheme="fas")]
    srv = serving.Server(workers=1, hbm_budget=1 << 40, simulate=True)
    rs = []
    for rep in range(2):
        for kw in kinds:
            rs.append(serving.Request(n=128, sim_ms=1.0, **kw))
    srv.run(rs)
    st = srv.stats()
    assert all(r.status == 0 for r in rs)
    assert st["created"] == len(kinds) and st["reused"] == len(kinds)
    want = sum(mg.mg_footprint_bytes(mg.params(128, 1 / 128, **kw)) + 128 ** 3 * 8 + 256 for kw in kinds)
    assert st["resident_bytes"] == want
    # the FAS class holds the restricted potentials: a larger footprint than the plain one
    assert mg.mg_footprint_bytes(mg.params(128, 1 / 128, scheme="fas")) > mg.mg_footprint_bytes(mg.params(128, 1 / 128))
