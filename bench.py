#!/usr/bin/env python3
"""Benchmark of the multigrid hot path on one MI355X.

Workload (default): the 512^3 periodic Gaussian-clump problem (64 clumps, widths 0.01-0.05,
lognormal amplitudes, mean removed), FMG + V(2,2) cycles to a relative residual of 1e-10,
FP64 and FP32/FP64 mixed precision.  One step = one whole solve with rho already resident
in HBM.  The JSON line reports:

  value         GDoF/s per V-cycle (FP64) = n^3 / median V-cycle time, V-cycles timed with
                HIP events inside the library during the timed steps;
  ms_per_step   wall time of one FP64 solve (set-up + FMG + cycles to tolerance);
  roofline      the dominant kernel (the finest-level pass with the largest summed time):
                algorithmic bytes per launch / its mean launch time (HIP events on the solve
                stream) against 8 TB/s; beside it, the V-cycle's algorithmic efficiency (the
                57 bytes per DoF a fully fused V(2,2) cycle must move, over the V-cycle time)
                and its counted bytes (profiler FETCH + WRITE of the finest-level passes x 8/7,
                over the V-cycle time);
  cpu_baseline  the CPU oracle timed on a bounded sample of the same workload;
  mixed         the same numbers for the mixed-precision solve; p50/p99 solve latency.
  fas           the same solve with Full Approximation Scheme iterations (Alg. 3): per-cycle
                rate, its finest-level passes and the roofline of the dominant one;
  amr           the paper's refined-mesh test (binary potential, 128^3 root grid, four nested
                levels, multipole faces): FMG and FAS V-cycles to 1e-10, composite cells per
                second per cycle,
                the numpy oracle beside it;
  gravity       g = -grad phi and rho g of the solved potential (Sec. 2.4): mean launch time
                and its HBM roofline (64 algorithmic bytes per cell), CPU oracle beside it;
  batched       the 256^3 lognormal field as 4096 MeshBlocks of 16^3 (autotuned), FP64 and
                mixed, beside the dense FP64 solve of the same field;
  serving       a mixed-size request stream through the serving runtime: saturated
                throughput and p50/p99 latency at 0.5 and 0.9 of it, FP64 and mixed.

python bench.py [--steps K] [--warmup W] [--n N] [--no-cpu-baseline] [--no-mixed]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2302_13903_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h", ".inl")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(kernel: str) -> str:
    """Kernel name as the profile summaries key it: no return type, namespaces or arguments."""
    k = kernel.replace("(anonymous namespace)::", "").replace("mg::", "").replace("void ", "")
    return k.split("(")[0]


def measured_traffic(kernel: str, n: int):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None
    when there is none or the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    entry = t.get("kernels", {}).get(f"{short_name(kernel)}@{n}")
    return None if entry is None else entry.get("bytes_per_launch")


def run_solves(mg, ctx, rho, n, precision, steps, warmup, tol, scheme="cs", bc="periodic", fixed_b=None,
               label="C2"):
    """`warmup` + `steps` solves; returns latencies, the V-cycle times of the timed solves (HIP
    events in the library; mixed precision: the outer steps), their histories, kernel timings,
    the last phi and the FP32 V-cycles of each timed solve (mixed precision)."""
    import torch
    phi = torch.zeros_like(rho)
    lat, cyc, hists, kt, inner = [], [], [], [], []
    for it in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi, hist, st = mg.solve(rho, 1.0 / n, bc, fixed_b=fixed_b, lmax=4, tol=tol, precision=precision, phi=phi,
                                 ctx=ctx, scheme=scheme)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if st < 0 or hist[-1] > tol:
            raise RuntimeError(f"solve did not converge: status {st}, hist {hist}")
        if it >= warmup:
            lat.append((t1 - t0) * 1e3)
            setup_ms, fmg_ms, cms = ctx.last_timing()
            cyc.extend(cms)
            hists.append(hist)
            kt.append(ctx.kernel_timing())
            inner.append(ctx.last_inner())
        print(f"# {label} {bc} {precision} {scheme} step {it - warmup:+d}: {1e3 * (t1 - t0):.2f} ms, "
              f"cycles {len(hist) - 1}, r = {hist[-1]:.2e}", file=sys.stderr, flush=True)
    return lat, cyc, hists, kt, phi, inner


def mixed_rate(n, cyc, inner):
    """GDoF/s per V-cycle of mixed-precision solves: n^3 times the FP32 V-cycles they ran, over
    the time of their outer steps (each outer step: its FP32 V-cycles and the FP64 update and
    defect)."""
    return n ** 3 * sum(inner) / (sum(cyc) * 1e-3) / 1e9


def phi_error(phi, ref):
    """Relative L2 and max-norm difference of two device fields."""
    import torch
    d = phi - ref
    return {"rel_l2": float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(ref)),
            "rel_max": float(d.abs().max() / ref.abs().max())}


FUSED_BYTES_PER_DOF = 57.0   # fully fused V(2,2) cycle, FP64: 50 B per finest cell x 8/7 for all levels


def v_cycle_efficiency(n: int, t_v_ms: float):
    """The V-cycle against the traffic a fully fused V(2,2) cycle needs (read phi, f and write
    phi and the coarse source going down; read the coarse correction, phi, f and write phi going
    up: 50 B per finest cell, 57 B per DoF over all levels), at 8 TB/s."""
    achieved = FUSED_BYTES_PER_DOF * n ** 3 / (t_v_ms * 1e-3) / 1e9
    return {"bytes_per_dof": FUSED_BYTES_PER_DOF, "v_cycle_ms": t_v_ms, "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS}


def v_cycle_counted(n: int, t_v_ms: float):
    """The V-cycle against the HBM bytes the profiler counted for whole V-cycles: FETCH + WRITE
    summed over every kernel dispatched from one finest-level down pass to the next (all levels,
    the tail and the norm reduction), averaged over the cycles of the profiled FP64 solves (the
    committed counter summary); None when it is missing or the kernel sources changed."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    vc = t.get("v_cycle", {}).get(str(n))
    if t.get("source_hash") != kernel_source_hash() or vc is None:
        return None
    per_cycle = vc["bytes_per_cycle"]
    achieved = per_cycle / (t_v_ms * 1e-3) / 1e9
    return {"bytes_per_cycle": per_cycle, "cycles_counted": vc["cycles"], "v_cycle_ms": t_v_ms, "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "over_algorithmic": per_cycle / (FUSED_BYTES_PER_DOF * n ** 3)}


def pass_table(kt):
    """Per kernel (finest-level passes), summed over the timed steps."""
    agg = {}
    for recs in kt:
        for r in recs:
            a = agg.setdefault(r["name"], {"launches": 0, "total_ms": 0.0, "bytes_per_launch": r["bytes_per_launch"]})
            a["launches"] += r["launches"]
            a["total_ms"] += r["total_ms"]
    passes = []
    for name, a in agg.items():
        avg = a["total_ms"] / max(a["launches"], 1)
        passes.append({"kernel": name, "launches": a["launches"], "avg_launch_ms": avg,
                       "algorithmic_bytes_per_launch": a["bytes_per_launch"],
                       "achieved_GBs": a["bytes_per_launch"] / (avg * 1e-3) / 1e9 if avg > 0 else None})
    return passes


def cpu_baseline(n: int, cycles: int = 3, c3=None):
    """The CPU oracle on bounded samples, V(2,2) cycles from zero after its set-up (FMG not
    timed); GDoF/s per V-cycle = n^3 / mean cycle time.  The headline figure is configuration 2
    (the same n^3 clump density as the GPU leg) on all the host threads the oracle's OpenMP
    runtime gets; `rows` adds that configuration on one thread and configurations 1, 3
    (`c3` = (rho, faces) of the sphere leg, fixed faces) and 4 (the 256^3 lognormal field as one
    dense grid: the MeshBlock form is the same algorithm) on all threads."""
    import numpy as np

    import oracle
    import workloads as wl
    nproc = oracle.num_threads()

    def rate(rho, kinds, faces, k, threads):
        oracle.set_threads(threads)
        m = rho.shape[0]
        st = oracle.State(rho, 1.0 / m, kinds, fixed_b=faces)
        st.set_phi(np.zeros_like(rho))
        t0 = time.perf_counter()
        for _ in range(k):
            st.vcycle()
        dt = (time.perf_counter() - t0) / k
        del st
        return m ** 3 / dt / 1e9, dt

    rows = []

    def row(config, rho, kinds, faces, k, threads, what):
        v, dt = rate(rho, kinds, faces, k, threads)
        rows.append({"config": config, "threads": threads, "value": v, "unit": "GDoF/s per V-cycle",
                     "sample": f"{what}, {k} V(2,2) cycles from zero, {dt * 1e3:.0f} ms per cycle"})
        print(f"# cpu oracle {config} on {threads} threads: {v:.4f} GDoF/s per V-cycle", file=sys.stderr,
              flush=True)
        return v, dt

    rho = wl.gaussian_clumps(n, 2)
    v, dt = row("C2", rho, "periodic", None, cycles, nproc, f"{n}^3 clump density")
    out = {"value": v, "unit": "GDoF/s per V-cycle", "cores": nproc, "kind": "oracle",
           "sample": f"{n}^3 clump density (the GPU leg's), {cycles} V(2,2) cycles from zero (FMG not timed), "
                     f"{dt * 1e3:.0f} ms per cycle, oracle built -O3 -march=x86-64-v3 without contraction"}
    row("C2", rho, "periodic", None, 1, 1, f"{n}^3 clump density")
    del rho
    row("C1", wl.sine_modes(32, 1)[0], "periodic", None, 20, nproc, "32^3 sine modes")
    if c3 is not None:
        row("C3", c3[0], "fixed", c3[1], 1, nproc, f"{c3[0].shape[0]}^3 uniform sphere, fixed faces")
    r4 = wl.lognormal_grf(256, 2)
    r4 -= r4.mean()
    row("C4", r4, "periodic", None, 2, nproc, "256^3 lognormal field as one dense grid")
    oracle.set_threads(nproc)
    out["rows"] = rows
    out["c5"] = "a request stream, not a solve: its CPU cost per solve follows from the C2 and C3 rows"
    return out


def gravity_leg(mg, ctx, rho, n: int, reps: int, with_cpu: bool):
    """g = -grad phi and rho g of the solved potential (the step after the solve): one launch
    of the streaming gravity kernel per call, reps calls bracketed by HIP events on the stream
    they run on.  Algorithmic bytes per cell: phi and rho read, g and rho g written = 64."""
    import torch
    phi, _, _ = mg.solve(rho, 1.0 / n, "periodic", tol=1e-10, ctx=ctx)
    p = mg.params(n, 1.0 / n)
    b = mg.boundary("periodic")
    g = torch.empty((3, n, n, n), dtype=torch.float64, device=rho.device)
    rg = torch.empty_like(g)
    s = torch.cuda.current_stream()
    for _ in range(3):
        mg.mg_gravity(ctx, p, b, phi, rho, g, rg, None, s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        mg.mg_gravity(ctx, p, b, phi, rho, g, rg, None, s)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    kernel = mg.mg_gravity_kernel_name(p, True, True, False)
    by = 64 * n ** 3
    achieved = by / (ms * 1e-3) / 1e9
    out = {"kernel": kernel, "outputs": "g, rho g", "launches": reps, "avg_launch_ms": ms,
           "algorithmic_bytes_per_launch": by, "Gcells_per_s": n ** 3 / (ms * 1e-3) / 1e9,
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kernel, n)}}
    del g, rg
    if with_cpu:
        import numpy as np

        import oracle
        m = 256
        rng = np.random.default_rng(0)
        ph, rh = rng.uniform(-1, 1, (m, m, m)), rng.uniform(0, 2, (m, m, m))
        t0 = time.perf_counter()
        oracle.gravity(ph, 1.0 / m, "periodic", rho=rh)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": m ** 3 / dt / 1e9, "unit": "Gcells/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"{m}^3 random potential and density, g and rho g, "
                                                           f"{dt * 1e3:.0f} ms"}
    return out


def c3_leg(mg, ctx, steps: int, seed: int = 3, n: int = 512):
    """Configuration 3: the n^3 uniform sphere (radius 0.25, seeded centre offset, sub-cell
    volume fractions on cut cells) with fixed faces (the analytic potential at the face centres)
    and with multipole faces (l <= 4), FP64 and mixed precision to 1e-10.  Per face kind: the
    V-cycle rate of each precision, phi against the analytic potential (the discretisation
    error at this h) and the mixed phi against the FP64 phi of the same problem."""
    import numpy as np
    import torch

    import workloads as wl
    R = 0.25
    t0 = time.perf_counter()
    rho_h, centre = wl.uniform_sphere(n, seed, radius=R)
    mass = 4.0 / 3.0 * math.pi * R ** 3
    faces_h = wl.sphere_face_values(n, centre, R, mass)
    x = wl.cell_centres(n)
    phi_a = torch.from_numpy(wl.sphere_potential(x[None, None, :], x[None, :, None], x[:, None, None], centre, R,
                                                 mass)).to("cuda:0")
    rho = torch.from_numpy(rho_h).to("cuda:0")
    faces = [torch.from_numpy(np.ascontiguousarray(b)).to("cuda:0") for b in faces_h]
    print(f"# C3 input {n}^3 generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    out = {"workload": f"C3 uniform sphere {n}^3 (R = {R}, centre {[round(float(c), 4) for c in centre]}), "
                       f"FMG + V(2,2) to relative residual 1e-10", "tol": 1e-10}
    for kind in ("fixed", "multipole"):
        res, phis = {}, {}
        for prec in ("fp64", "mixed"):
            lat, cyc, hists, _, phi, inner = run_solves(mg, ctx, rho, n, prec, steps, 1, 1e-10, bc=kind,
                                                        fixed_b=faces if kind == "fixed" else None, label="C3")
            t_v = statistics.median(cyc)
            phis[prec] = phi.clone()
            res[prec] = {"value": n ** 3 / (t_v * 1e-3) / 1e9 if prec == "fp64" else mixed_rate(n, cyc, inner),
                         "unit": "GDoF/s per V-cycle",
                         "cycle_ms_median": t_v, "cycles_per_solve": len(hists[-1]) - 1,
                         "solve_latency_ms": {"p50": pct(lat, 0.5), "p99": pct(lat, 0.99)},
                         "error_vs_analytic": phi_error(phi, phi_a)}
            if prec == "mixed":
                res[prec]["inner_cycles_per_solve"] = inner[-1]
        res["mixed"]["error_vs_fp64"] = phi_error(phis["mixed"], phis["fp64"])
        out[kind] = res
        del phis
    return out, (rho_h, faces_h)


AMR_NB, AMR_NB_CELLS = 8, 16   # binary test: 128^3 root grid (8^3 blocks of 16^3), four nested levels


def binary_case(NB, nb):
    """The paper's refined-mesh test (Sec. 4.3): the unequal-mass binary on four nested levels
    of refinement, per-patch densities (sub-cell averaged) and the analytic potential on the
    domain faces (in place of the multipole faces, which the refined path does not take)."""
    import numpy as np

    import workloads as wl
    boxes = wl.binary_mesh_boxes(NB)
    rho = []
    for lam in range(len(boxes) + 1):
        h = 1.0 / (NB * nb * (1 << lam))
        if lam == 0:
            lo, n = (0, 0, 0), (NB * nb,) * 3
        else:
            blo, bhi = boxes[lam - 1]
            lo = tuple(2 * blo[a] * nb for a in range(3))
            n = tuple(2 * (bhi[a] - blo[a]) * nb for a in range(3))
        ax = [(lo[a] + np.arange(n[a]) + 0.5) * h for a in range(3)]
        rho.append(wl.binary_density_on_axes(ax[0], ax[1], ax[2], h))
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
    return boxes, rho, faces


def amr_leg(mg, steps: int, with_cpu: bool):
    """Refined mesh (the paper's Sec. 3.3, its binary test of Sec. 4.3): 128^3 root grid of
    16^3-cell MeshBlocks with four nested refined levels (the finest at 1/2048 around the
    stars), FMG then FAS V-cycles to 1e-10.  The rate counts the composite (active) cells per
    V-cycle (solve time over cycles, FMG included)."""
    import numpy as np
    import torch
    NB, nb = AMR_NB, AMR_NB_CELLS
    boxes, rho_h, _ = binary_case(NB, nb)
    rho = [torch.from_numpy(r).to("cuda:0") for r in rho_h]
    mesh = mg.amr_mesh(NB, nb, boxes)
    covered = sum(int(np.prod([(b[1][a] - b[0][a]) * nb for a in range(3)])) for b in boxes)
    dof = sum(r.size for r in rho_h) - covered
    ctx = mg.Context(0)
    lat, cyc = [], []
    for it in range(1 + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi, hist, st = mg.amr_solve(mesh, rho, "multipole", lmax=4, tol=1e-10, mode="fmg", ctx=ctx)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) * 1e3
        if st < 0 or hist[-1] > 1e-10:
            raise RuntimeError(f"refined-mesh solve did not converge: {st}, {hist}")
        if it > 0:
            lat.append(dt)
            cyc.append(len(hist) - 1)
        print(f"# amr step {it - 1:+d}: {dt:.1f} ms, cycles {len(hist) - 1}, r = {hist[-1]:.2e}", file=sys.stderr,
              flush=True)
    ms_cycle = statistics.median(lat) / statistics.median(cyc)
    out = {"workload": "binary potential (Sec. 4.3): 128^3 root grid (8^3 blocks of 16^3), four nested levels "
                       "refined 2:1 around the stars, open faces from the hexadecapole expansion (Appendix A) of the "
                       "composite density, FMG + FAS V(2,2) to 1e-10",
           "composite_cells": dof, "cycles_per_solve": cyc[-1], "solve_ms": statistics.median(lat),
           "ms_per_cycle_incl_fmg": ms_cycle, "value": dof / (ms_cycle * 1e-3) / 1e9,
           "unit": "GDoF/s per V-cycle (composite cells)"}
    if with_cpu:
        import oracle.amr as oamr
        NBs, nbs = 4, 8
        bxs, rho_s, _ = binary_case(NBs, nbs)
        m = oamr.AmrMesh(NBs, nbs, bxs)
        st_o = oamr.AmrState(m, rho_s, [oamr.FIXED] * 6, oamr.multipole_faces(m, rho_s, 4))
        t0 = time.perf_counter()
        st_o.vcycle()
        dt = time.perf_counter() - t0
        cells_o = sum(int(np.prod(m.patches[l][m.K].n)) for l in range(m.Lam + 1)) - \
            sum(int(np.prod([(b[1][a] - b[0][a]) * nbs for a in range(3)])) for b in bxs)
        out["cpu_baseline"] = {"value": cells_o / dt / 1e9, "unit": "GDoF/s per V-cycle (composite cells)",
                               "cores": 1, "kind": "oracle",
                               "sample": f"one V-cycle of the numpy oracle on the binary mesh at root resolution "
                                         f"1/32 ({cells_o} cells), {dt * 1e3:.0f} ms"}
    return out


def batched_leg(steps: int, seed: int, n: int = 256, block_n: int = 16):
    """Configuration 4: the 256^3 lognormal field (exp of a Gaussian random field with
    P(k) ~ k^-4, mean removed, periodic) as 4096 MeshBlocks of 16^3 with autotuned block
    sweeps, FP64 and mixed precision, beside the dense FP64 solve of the same field."""
    import torch

    import paper_2302_13903_amd as mg
    import workloads as wl
    rho_h = wl.lognormal_grf(n, seed)
    rho_h -= rho_h.mean()
    rho = torch.from_numpy(rho_h).to("cuda:0")
    rho_b = mg.to_blocks(rho, block_n)
    ctx = mg.Context(0)
    out = {"workload": f"C4 lognormal GRF {n}^3 periodic as {(n // block_n) ** 3} blocks of {block_n}^3",
           "tol": 1e-10}
    tune = {}
    for prec in ("fp64", "mixed"):
        tune[prec] = ctx.autotune(n, block_n, prec, reps=5)
    out["schedules"] = tune
    phi_dense = None
    for name, x, layout, prec in (("dense_fp64", rho, "dense", "fp64"), ("blocks_fp64", rho_b, "blocks", "fp64"),
                                  ("blocks_mixed", rho_b, "blocks", "mixed")):
        lat, cyc, inner = [], [], []
        for it in range(steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            phi, hist, st = mg.solve(x, 1.0 / n, "periodic", tol=1e-10, precision=prec, layout=layout,
                                     block_n=block_n, ctx=ctx)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if st != 0:
                raise RuntimeError(f"{name}: status {st}, hist {hist}")
            if it > 0:
                lat.append((t1 - t0) * 1e3)
                cyc.extend(ctx.last_timing()[2])
                inner.append(ctx.last_inner())
        rate = n ** 3 / (statistics.median(cyc) * 1e-3) / 1e9 if prec == "fp64" else mixed_rate(n, cyc, inner)
        rec = {"value": rate, "unit": "GDoF/s per V-cycle",
               "cycle_ms_median": statistics.median(cyc), "cycles": len(hist) - 1,
               "solve_ms": {"p50": pct(lat, 0.5), "p99": pct(lat, 0.99)}}
        if prec == "mixed":
            rec["inner_cycles"] = inner[-1]
        if name == "dense_fp64":
            phi_dense = phi
        else:
            phi_d = mg.from_blocks(phi, n, block_n)
            rec["rel_diff_vs_dense"] = float(torch.linalg.norm(phi_d - phi_dense) / torch.linalg.norm(phi_dense))
        if name == "blocks_fp64":
            # per-kernel times from one more solve with kernel timing on (the timed solves above
            # run without it, as the dense one does: timing adds a few microseconds per pass)
            ctx.set_kernel_timing(True)
            mg.solve(x, 1.0 / n, "periodic", tol=1e-10, precision=prec, layout=layout, block_n=block_n, ctx=ctx)
            torch.cuda.synchronize()
            ctx.set_kernel_timing(False)
            rec["kernels"] = [{"kernel": k["name"], "launches": k["launches"],
                               "avg_launch_ms": k["total_ms"] / max(k["launches"], 1),
                               "achieved_GBs": k["bytes_per_launch"] * k["launches"] / (k["total_ms"] * 1e-3) / 1e9}
                              for k in ctx.kernel_timing()]
        out[name] = rec
        print(f"# batched {name}: {rec['value']:.2f} GDoF/s per V-cycle, {rec['cycles']} cycles",
              file=sys.stderr, flush=True)
    ctx.set_kernel_timing(False)
    return out


SERVE_POOL = {64: 64, 128: 32, 256: 16, 512: 8}   # distinct densities per size


def serving_leg(n_requests: int, workers: int, seed: int):
    """Configuration 5: a Poisson-arrival stream of mixed-size requests (sizes 64-512 and
    periodic / fixed / multipole faces, uniform) through the native serving runtime: first all
    requests at once (saturated throughput mu), then open-loop at 0.9 mu (and 0.5 mu in FP64);
    FP64 and mixed precision.  Each request's density is picked by its own seed from a pool of
    distinct clump densities per size (two generated fields per size, each periodically shifted
    by seeded offsets: the clump centres stay uniform), resident in HBM before the runs."""
    import numpy as np
    import torch

    import workloads as wl
    from paper_2302_13903_amd import serving
    sizes = (64, 128, 256, 512)
    rng = np.random.default_rng(seed)
    pool = {}
    for n in sizes:
        base = [torch.from_numpy(wl.gaussian_clumps(n, seed + 17 * k + n, remove_mean=False)).to("cuda:0")
                for k in range(2)]
        pool[n] = [torch.roll(base[k % 2], tuple(int(v) for v in rng.integers(0, n, 3)), dims=(0, 1, 2)).contiguous()
                   for k in range(SERVE_POOL[n])]
        del base
    srv = serving.Server(workers=workers)
    out = {"workers": workers, "requests": n_requests, "sizes": list(sizes),
           "bcs": ["periodic", "fixed", "multipole"], "tol": 1e-10,
           "densities_per_size": {str(k): v for k, v in SERVE_POOL.items()}}
    for prec in ("fp64", "mixed"):
        def reqs(rate):
            tr = wl.serving_trace(n_requests, seed, rate if rate else 1.0, sizes=sizes)
            return [serving.Request(rho=pool[t["n"]][t["seed"] % SERVE_POOL[t["n"]]], bc=t["bc"], precision=prec,
                                    arrival_ms=t["t"] if rate else 0.0) for t in tr]
        srv.run([serving.Request(rho=pool[n][k], bc="multipole", precision=prec)
                 for n in sizes for k in range(workers)])  # warm-up: resident hierarchies
        res = {}
        sat = serving.summary(srv.run(reqs(None)))
        res["saturated"] = sat
        mu = sat["solves_per_s"] / 1e3  # requests per ms
        for frac in ((0.5, 0.9) if prec == "fp64" else (0.9,)):
            r = srv.run(reqs(frac * mu))
            bad = [q.status for q in r if q.status != 0]
            if bad:
                raise RuntimeError(f"serving: {len(bad)} requests failed: {bad[:5]}")
            res[f"rate_{frac}"] = serving.summary(r)
        out[prec] = res
        print(f"# serving {prec}: saturated {sat['solves_per_s']:.1f} solves/s, "
              f"p99 at 0.9 mu {res['rate_0.9']['latency_ms']['p99']:.1f} ms", file=sys.stderr, flush=True)
    out["hierarchies"] = srv.stats()
    return out


# ---------------------------------------------------------------- profile summaries (no GPU)

PROFILE_ARGS = "--steps 2 --warmup 1 --no-cpu-baseline --no-batched --serve-requests 0 --no-c3 --calibrate-copy"
PROFILE_RUNS = {
    "kernel_stats_c2_512.md": (
        "Kernel time, C2 Gaussian clumps 512^3 periodic: FP64, FAS and mixed solves to 1e-10, gravity, refined mesh",
        "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/p_trace -o run -- python3 bench.py "
        + PROFILE_ARGS),
    "kernel_stats_c4_blocks_256.md": (
        "Kernel time, C4 lognormal 256^3 as 4096 MeshBlocks of 16^3 (autotune, dense FP64, blocks FP64 and mixed)",
        "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/p_trace_c4 -o run -- python3 bench.py "
        "--only batched --steps 2"),
}
COUNTER_CMDS = [f"rocprofv3 --pmc {c} --output-format csv -d gpurun_out/p_{c.split('_')[0].lower()} -o run -- "
                f"python3 bench.py {PROFILE_ARGS}" for c in ("FETCH_SIZE", "WRITE_SIZE")]
# kernels that run once per solve (set-up, FMG, gauge fix) or belong to another scheme: a span
# between two finest-level down passes that holds one of them is not a plain V-cycle
NOT_IN_CYCLE = ("k_source", "k_shift", "k_restrict<", "k_prolong<double, 1>", "k_fas", "k_mix", "k_copy_convert",
                "k_grav")


def _read_csv(path):
    import csv
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def summarize_trace(trace_dir: str, out_name: str):
    """profiles/<out_name>: per kernel and per (kernel, grid) call counts and mean durations from a
    rocprofv3 kernel trace of this script."""
    title, cmd = PROFILE_RUNS[out_name]
    rows = _read_csv(os.path.join(trace_dir, "run_kernel_trace.csv"))
    per, per_grid = {}, {}
    for r in rows:
        k = short_name(r["Kernel_Name"])
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
        g = int(r.get("Grid_Size") or r.get("Grid_Size_X"))
        for key, tab in ((k, per), ((k, g), per_grid)):
            a = tab.setdefault(key, [0, 0.0])
            a[0] += 1
            a[1] += d
    tot = sum(v[1] for v in per.values())
    lines = [f"# {title} (rocprofv3 --kernel-trace --stats)", "",
             "Command (from the repository root, after `cd /tmp && export TMPDIR=/tmp` and back):", "", "```", cmd,
             "```", "", "Per kernel (all levels):", "", "| kernel | calls | avg us | total ms | % |",
             "|---|---:|---:|---:|---:|"]
    for k, (c, t) in sorted(per.items(), key=lambda x: -x[1][1])[:30]:
        lines.append(f"| `{k}` | {c} | {t / c:.1f} | {t * 1e-3:.2f} | {100 * t / tot:.1f} |")
    lines += ["", f"Total kernel time {tot * 1e-3:.1f} ms.", "",
              "Per kernel and grid size (grid = threads launched; a kernel's largest grid is its finest level):", "",
              "| kernel | grid | calls | avg us |", "|---|---:|---:|---:|"]
    for (k, g), (c, t) in sorted(per_grid.items(), key=lambda x: -x[1][1])[:40]:
        lines.append(f"| `{k}` | {g} | {c} | {t / c:.1f} |")
    with open(os.path.join(ROOT, "profiles", out_name), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize_counters(fetch_dir: str, write_dir: str, n: int, out_dir: str = ""):
    """profiles/traffic.json and profiles/hbm_traffic_c2_<n>.md from the FETCH_SIZE and WRITE_SIZE
    runs: bytes per launch of each kernel at its largest grid (its finest level), scaled by what
    the counters read for the 1 GiB calibration copy, and the bytes of whole FP64 V-cycles (every
    dispatch from one finest-level down pass to the next)."""
    runs = {}
    for ctr, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _read_csv(os.path.join(d, "run_counter_collection.csv")) if r["Counter_Name"] == ctr]
        disp = {}
        for r in rows:
            key = int(r["Dispatch_Id"])
            e = disp.setdefault(key, {"name": short_name(r["Kernel_Name"]), "grid": int(r["Grid_Size"]), "v": 0.0})
            e["v"] += float(r["Counter_Value"])
        runs[ctr] = [disp[k] for k in sorted(disp)]
    gib = float(1 << 30)
    scale = {}
    for ctr in runs:
        cal = max((e["v"] for e in runs[ctr] if e["name"].startswith("__amd_rocclr_copyBuffer")), default=None)
        if not cal:
            raise SystemExit(f"{ctr}: no calibration copy in the counter run (use --calibrate-copy)")
        scale[ctr] = gib / (cal * 1024.0)
    kernels = {}
    for ctr, key in (("FETCH_SIZE", "read_bytes"), ("WRITE_SIZE", "write_bytes")):
        top = {}
        for e in runs[ctr]:
            if e["name"].startswith("__amd"):
                continue
            t = top.get(e["name"])
            if t is None or e["grid"] > t[0]:
                top[e["name"]] = [e["grid"], [e["v"]]]
            elif e["grid"] == t[0]:
                t[1].append(e["v"])
        for name, (g, vs) in top.items():
            rec = kernels.setdefault(f"{name}@{n}", {"grid": g, "dispatches": len(vs)})
            rec[key] = statistics.mean(vs) * 1024.0 * scale[ctr]
    for rec in kernels.values():
        rec["bytes_per_launch"] = rec.get("read_bytes", 0.0) + rec.get("write_bytes", 0.0)
    # whole V-cycles: spans between consecutive dispatches of the FP64 finest-level down pass
    cyc = {}
    for ctr in runs:
        ev = runs[ctr]
        downs = [e for e in ev if e["name"].startswith("k_march<double") and ", false, false," in e["name"]
                 and not e["name"].endswith("true>")]
        if not downs:
            raise SystemExit("no FP64 two-sweep down pass in the counter run")
        gmax = max(e["grid"] for e in downs)
        marks = [i for i, e in enumerate(ev) if e in downs and e["grid"] == gmax]
        spans = []
        for a, b in zip(marks, marks[1:]):
            seg = ev[a:b]
            if any(x in e["name"] for e in seg for x in NOT_IN_CYCLE):
                continue
            spans.append(sum(e["v"] for e in seg) * 1024.0 * scale[ctr])
        cyc[ctr] = spans
    nc = min(len(cyc["FETCH_SIZE"]), len(cyc["WRITE_SIZE"]))
    if nc == 0:
        raise SystemExit("no complete V-cycle in the counter runs")
    rd, wr = statistics.mean(cyc["FETCH_SIZE"]), statistics.mean(cyc["WRITE_SIZE"])
    out = {"source_hash": kernel_source_hash(), "fetch_scale": scale["FETCH_SIZE"], "write_scale": scale["WRITE_SIZE"],
           "command": COUNTER_CMDS, "kernels": dict(sorted(kernels.items(), key=lambda x: -x[1]["bytes_per_launch"])),
           "v_cycle": {str(n): {"bytes_per_cycle": rd + wr, "read_bytes": rd, "write_bytes": wr, "cycles": nc,
                                "algorithmic_bytes": FUSED_BYTES_PER_DOF * n ** 3}}}
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    with open(os.path.join(out_dir, os.path.basename(TRAFFIC_FILE)), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    lines = [f"# HBM traffic, C2 {n}^3 FP64 and mixed solves, FAS, gravity (rocprofv3 --pmc)", "",
             "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two separate runs of the same script:", "", "```"]
    lines += COUNTER_CMDS + ["```", "",
                             f"Calibration: the 1 GiB device-to-device copy that `--calibrate-copy` runs first "
                             f"(`__amd_rocclr_copyBuffer`) gives bytes = FETCH_SIZE x 1024 x {scale['FETCH_SIZE']:.3f} "
                             f"and WRITE_SIZE x 1024 x {scale['WRITE_SIZE']:.3f}.", "",
                             f"Whole FP64 V-cycles ({nc} counted; every dispatch from one {n}^3 down pass to the "
                             f"next: all levels, the tail, the norm reduction): read {rd / 1e9:.3f} GB + write "
                             f"{wr / 1e9:.3f} GB = {(rd + wr) / 1e9:.3f} GB per cycle, "
                             f"{(rd + wr) / (FUSED_BYTES_PER_DOF * n ** 3):.2f}x the {FUSED_BYTES_PER_DOF:.0f} B/DoF "
                             f"a fully fused V(2,2) cycle moves ({FUSED_BYTES_PER_DOF * n ** 3 / 1e9:.2f} GB).", "",
                             "Per kernel at its largest grid (its finest level):", "",
                             "| kernel | grid | dispatches | read GB | write GB |", "|---|---:|---:|---:|---:|"]
    for k, rec in list(out["kernels"].items())[:30]:
        lines.append(f"| `{k.rsplit('@', 1)[0]}` | {rec['grid']} | {rec['dispatches']} | "
                     f"{rec.get('read_bytes', 0.0) / 1e9:.3f} | {rec.get('write_bytes', 0.0) / 1e9:.3f} |")
    with open(os.path.join(out_dir, f"hbm_traffic_c2_{n}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize_profiles(trace_dir: str, fetch_dir: str, write_dir: str, n: int):
    summarize_trace(trace_dir, "kernel_stats_c2_512.md")
    summarize_counters(fetch_dir, write_dir, n)
    c4 = os.path.join(os.path.dirname(os.path.abspath(trace_dir)), "p_trace_c4")
    if os.path.isdir(c4):
        summarize_trace(c4, "kernel_stats_c4_blocks_256.md")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests per serving run (0: skip the serving leg)")
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--no-batched", action="store_true", help="skip the MeshBlock (4096 x 16^3) leg")
    ap.add_argument("--no-gravity", action="store_true", help="skip the g = -grad phi leg")
    ap.add_argument("--no-fas", action="store_true", help="skip the Full Approximation Scheme leg")
    ap.add_argument("--no-amr", action="store_true", help="skip the refined-mesh leg")
    ap.add_argument("--no-c3", action="store_true", help="skip the 512^3 sphere (fixed and multipole faces) leg")
    ap.add_argument("--only", choices=("batched",),
                    help="run only that leg and print its record (for profiling it alone)")
    ap.add_argument("--summarize-profiles", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="write the profiles/ summaries from rocprofv3 output of this script (no GPU work)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device to device (reference for profiler byte counters)")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(*args.summarize_profiles, n=args.n)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        return 2

    import torch

    import paper_2302_13903_amd as mg
    import workloads as wl

    if args.only == "batched":
        print(json.dumps({"batched": batched_leg(args.steps, args.seed)}), flush=True)
        return 0
    n = args.n
    t0 = time.perf_counter()
    rho_h = wl.gaussian_clumps(n, args.seed)
    rho = torch.from_numpy(rho_h).to("cuda:0")
    del rho_h
    print(f"# input {n}^3 generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("# calibration copy: 1073741824 bytes read, 1073741824 bytes written", file=sys.stderr, flush=True)
        del src, dst

    ctx = mg.Context(0)
    ctx.set_kernel_timing(True)
    lat, cyc, hists, kt, phi64, _ = run_solves(mg, ctx, rho, n, "fp64", args.steps, args.warmup, args.tol)
    phi64 = phi64.clone()
    t_v = statistics.median(cyc)
    value = n ** 3 / (t_v * 1e-3) / 1e9
    passes = pass_table(kt)
    dom = max(passes, key=lambda q: q["avg_launch_ms"] * q["launches"])
    achieved = dom["achieved_GBs"]
    traffic = measured_traffic(dom["kernel"], n)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": None if achieved is None else achieved / HBM_PEAK_GBS, "traffic": traffic,
                "scope": "the dominant kernel (finest-level pass with the largest summed time); the whole V-cycle "
                         "is in v_cycle_algorithmic and v_cycle_counted",
                "kernel": dom["kernel"], "algorithmic_bytes_per_launch": dom["algorithmic_bytes_per_launch"],
                "avg_launch_ms": dom["avg_launch_ms"], "launches": dom["launches"], "passes": passes,
                "v_cycle_algorithmic": v_cycle_efficiency(n, t_v),
                "v_cycle_counted": v_cycle_counted(n, t_v)}

    out = {
        "metric": "GDoF/s per V-cycle + % HBM roofline at 512^3; p50/p99 solve latency, mixed vs FP64",
        "value": value,
        "unit": "GDoF/s per V-cycle",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": statistics.mean(lat),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"C2 Gaussian clumps {n}^3 periodic, FMG + V(2,2) to relative residual "
                               f"{args.tol:g}", "n": n, "tol": args.tol, "cycles_per_solve": len(hists[-1]) - 1},
        "roofline": roofline,
        "v_cycle_ms_median": t_v,
        "solve_latency_ms": {"p50": pct(lat, 0.5), "p99": pct(lat, 0.99)},
    }
    ctx.set_kernel_timing(False)
    if not args.no_gravity:
        out["gravity"] = gravity_leg(mg, ctx, rho, n, 20, not args.no_cpu_baseline)
    if not args.no_fas:
        ctx.set_kernel_timing(True)
        lat_f, cyc_f, hists_f, kt_f, _, _ = run_solves(mg, ctx, rho, n, "fp64", max(2, args.steps // 2), 1, args.tol,
                                                    scheme="fas")
        ctx.set_kernel_timing(False)
        tvf = statistics.median(cyc_f)
        pf = pass_table(kt_f)
        domf = max(pf, key=lambda q: q["avg_launch_ms"] * q["launches"])
        out["fas"] = {"value": n ** 3 / (tvf * 1e-3) / 1e9, "unit": "GDoF/s per FAS cycle",
                      "ms_per_step": statistics.mean(lat_f), "cycles_per_solve": len(hists_f[-1]) - 1,
                      "cycle_ms_median": tvf,
                      "roofline": {"bound": "hbm", "achieved": domf["achieved_GBs"], "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": domf["achieved_GBs"] / HBM_PEAK_GBS,
                                   "traffic": measured_traffic(domf["kernel"], n), "kernel": domf["kernel"],
                                   "passes": pf}}
    if not args.no_amr:
        out["amr"] = amr_leg(mg, 2, not args.no_cpu_baseline)
    if not args.no_mixed:
        lat_m, cyc_m, hists_m, _, phim, inner_m = run_solves(mg, ctx, rho, n, "mixed", args.steps, args.warmup,
                                                             args.tol)
        tvm = statistics.median(cyc_m)
        out["mixed"] = {"value": mixed_rate(n, cyc_m, inner_m),
                        "unit": "GDoF/s per V-cycle (an outer step of k FP32 V-cycles counts as k)",
                        "ms_per_step": statistics.mean(lat_m), "cycles_per_solve": len(hists_m[-1]) - 1,
                        "inner_cycles_per_solve": inner_m[-1], "cycle_ms_median": tvm,
                        "solve_latency_ms": {"p50": pct(lat_m, 0.5), "p99": pct(lat_m, 0.99)},
                        "error_vs_fp64": phi_error(phim, phi64)}
        del phim
    del phi64
    c3_inputs = None
    if not args.no_c3:
        out["c3"], c3_inputs = c3_leg(mg, ctx, max(2, args.steps // 2))
    if not args.no_batched:
        out["batched"] = batched_leg(args.steps, args.seed)
    if args.serve_requests > 0:
        out["serving"] = serving_leg(args.serve_requests, args.serve_workers, args.seed)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, c3=c3_inputs)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
