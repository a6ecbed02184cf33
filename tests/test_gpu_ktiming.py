"""Per-kernel timing of the finest-level passes (mg_set_kernel_timing / mg_kernel_timing), the
records that the benchmark's roofline figures come from.  A pass that is one kernel is timed by
the start and end timestamps of its own dispatch; a split pass (interior and wall tiles on two
streams) by events around both launches.  Every record must count one launch per V-cycle of
the last solve, and the timed passes must fit inside the cycles' own times."""
import statistics

import pytest
import torch

import paper_2302_13903_amd as mg
import workloads as wl

pytestmark = pytest.mark.gpu

N = 256


def _rho(remove_mean):
    return torch.from_numpy(wl.gaussian_clumps(N, 3, remove_mean=remove_mean)).to("cuda:0")


@pytest.mark.parametrize("bc,layout,scheme", [
    ("periodic", "dense", "cs"),      # one kernel per pass: dispatch timestamps
    ("fixed", "dense", "cs"),         # split passes on two streams: events around both
    ("periodic", "blocks", "cs"),     # MeshBlock layout
    ("periodic", "dense", "fas"),     # FAS down pass
])
def test_kernel_timing_records(bc, layout, scheme):
    rho = _rho(remove_mean=bc == "periodic")
    x = mg.to_blocks(rho, 16) if layout == "blocks" else rho
    ctx = mg.Context(0)
    ctx.set_kernel_timing(True)
    for _ in range(2):                    # the second solve's records are read
        phi, hist, st = mg.solve(x, 1.0 / N, bc, tol=1e-10, layout=layout, block_n=16, scheme=scheme, ctx=ctx)
    torch.cuda.synchronize()
    assert st == 0, (st, hist)
    cycles = len(hist) - 1
    cyc = ctx.last_timing()[2]
    recs = ctx.kernel_timing()
    print(bc, layout, scheme, cycles, [(r["name"], r["launches"], round(r["total_ms"], 4)) for r in recs],
          flush=True)
    assert len(recs) >= 2
    assert len(cyc) == cycles
    per_cycle = 0.0
    for r in recs:
        assert r["launches"] == cycles, r
        avg = r["total_ms"] / r["launches"]
        assert 0.005 < avg < max(cyc), r
        assert r["bytes_per_launch"] > 0
        per_cycle += avg
    # the finest level's down and up passes are part of every cycle
    assert per_cycle < 1.02 * statistics.median(cyc), (per_cycle, cyc)
    ctx.set_kernel_timing(False)
    phi2, hist2, st2 = mg.solve(x, 1.0 / N, bc, tol=1e-10, layout=layout, block_n=16, scheme=scheme, ctx=ctx)
    torch.cuda.synchronize()
    # timing changes nothing in the result
    assert st2 == 0 and len(hist2) == len(hist)
    assert torch.equal(phi2, phi)
