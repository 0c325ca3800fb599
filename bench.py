#!/usr/bin/env python3
"""Benchmark of the lattice Boltzmann hot path on one MI355X.

Workload (one "step" = one fused stream-collide pass over the lattice):
lid-driven cavity 512^3, D3Q19 TRT (magic 1/4), tau 0.6, lid velocity 0.1
along y, walls on all faces; FP32 arithmetic with FP16S storage for `value`,
and the same run with FP32, FP16C, FP16, P16 and FP64 storage reported next
to it.  Inputs are synthetic (the cavity starts at rest) and resident in HBM
before timing.

Prints one JSON line: MLUPs/s (10^6 cell updates per second, all cells of the
box), the HBM roofline of the dominant kernel (algorithmic bytes per launch /
measured launch time vs 8 TB/s, and the HBM traffic from the committed
rocprofv3 counter summary when it was taken on the current kernel sources),
the L2 velocity error of each FP32 storage format against the FP64 GPU path
on a 64^3 cavity after 1000 steps, the FP64 CPU reference timed on the host
cores on a bounded sample, and, unless switched off, the 256-lattice
ensemble, the full-size Karman channel (1024x256x64, D3Q27) and the periodic
256^3 boxes of the paper's performance table.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X datasheet HBM3E bandwidth
HEADLINE = "fp16s"
OTHERS = ["fp32", "fp16c", "fp16", "p16_0s", "p16_1s", "p16_2c", "fp64"]
BYTES = {"fp64": 8, "fp32": 4}


def ddf_bytes(storage: str) -> int:
    return BYTES.get(storage, 2)


def code_only(text: str) -> str:
    """C++ source without its comments and blank lines, string and character
    literals kept as they are (a comment-only edit leaves the code the
    same)."""
    out, i, n = [], 0, len(text)
    while i < n:
        ch = text[i]
        if ch in "\"'":
            j = i + 1
            while j < n and text[j] != ch:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            i = text.find("\n", i)
            i = n if i < 0 else i
        elif text.startswith("/*", i):
            i = text.find("*/", i + 2)
            i = n if i < 0 else i + 2
        else:
            out.append(ch)
            i += 1
    return "\n".join(line.rstrip() for line in "".join(out).splitlines() if line.strip())


def kernel_source_hash() -> str:
    """Hash of the code (comments left out) the step kernels and their
    launchers are built from (every file of csrc/ but the host runtime), so
    that stored counter readings are used only for the kernel they were
    taken on."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2112_08926_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name == "lbm_runtime.hip":
            continue
        with open(os.path.join(csrc, name), encoding="utf-8") as fh:
            h.update(name.encode())
            h.update(code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def cavity(n, storage, tau=0.6, lid=0.1, q=19, collision="trt"):
    import paper_2112_08926_amd as lbm
    import lbm_workloads as wl
    arith = "fp64" if storage == "fp64" else "fp32"
    p = lbm.make_params(n, n, n, q=q, collision=collision, storage=storage, arith=arith, tau=tau,
                        wall_u=(0.0, lid, 0.0))
    g = lbm.Lattices(p)
    flags = wl.cavity_flags(n, n, n)
    g.set_boundaries(0, flags)
    return g, flags


def time_steps(g, steps, warmup, chunks=None):
    """Average time of one step (= one stream-collide launch) over `steps`
    launches, measured with events on the stream the kernels run on.  With a
    list `chunks`, the timed steps are also split into 5 equal runs (when
    `steps` is a multiple of 5) whose ms per step are appended to it, events
    only, so the total is timed exactly as without."""
    import torch
    stream = g.stream
    g.step(warmup)
    torch.cuda.synchronize()
    parts = 5 if (chunks is not None and steps % 5 == 0) else 1
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(parts + 1)]
    ev[0].record(stream)
    for k in range(parts):
        g.step(steps // parts)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    if parts > 1:
        chunks.extend(ev[k].elapsed_time(ev[k + 1]) / (steps // parts) for k in range(parts))
    return ev[0].elapsed_time(ev[parts]) / steps


def diag_cost(g, flags, q, storage, every, steps):
    """Cost of the FP64 diagnostics.  The separate pass (lbm_diagnostics:
    first pass, both reduction passes and the copy of the results to the
    host, which synchronises): the time of one call measured with events on
    the handle's stream and its algorithmic bytes (Q b + 1 per fluid cell,
    the flag byte per other cell) per second.  The fused step
    (lbm_step_diagnostics: a step that also reduces the state it reads): its
    time against a plain step.  And the wall-clock overhead per step of
    taking the diagnostics every `every` steps with the fused step, over
    `steps` steps, against the same steps without them."""
    import torch
    stream = g.stream

    def timed(fn, reps=5):
        torch.cuda.synchronize()
        out, times = None, []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            out = fn()
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        return float(np.median(times)), out

    ms, d = timed(lambda: g.diagnostics(0))
    fused_ms, _ = timed(lambda: g.step_diagnostics())
    step_ms, _ = timed(lambda: g.step(1))
    N = flags.size
    n_fluid = int(np.count_nonzero(flags == 0))
    alg = n_fluid * (q * ddf_bytes(storage) + 1) + (N - n_fluid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    g.synchronize()
    plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(steps // every):
        g.step(every - 1)
        d = g.step_diagnostics()
    g.synchronize()
    with_diag = time.perf_counter() - t0
    return {"every": every, "diag_ms": round(ms, 4), "diag_alg_bytes": alg,
            "diag_GBps": round(alg / (ms * 1e-3) / 1e9, 1),
            "diag_frac_of_8TBps": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "fused_step_ms": round(fused_ms, 4), "plain_step_ms": round(step_ms, 4),
            "fused_extra_ms": round(fused_ms - step_ms, 4),
            "overhead_ms_per_step": round((with_diag - plain) / steps * 1e3, 4),
            "plain_ms_per_step": round(plain / steps * 1e3, 4),
            "last": {"kinetic_energy": d["kinetic_energy"], "mass": d["mass"],
                     "force_on_solid": [float(v) for v in d["force_on_solid"]],
                     "nonfinite_updates": d["nonfinite_updates"]}}


LAUNCH_KINDS = {0: "row tiles", 1: "batched row tiles", 2: "cell-contiguous tiles"}


def launch_desc(cfg):
    """The autotuned launch: its kind (include/lbm.h lbm_launch_mode),
    workgroup size and cells per lane."""
    return {"kind": LAUNCH_KINDS.get(cfg["mode"], str(cfg["mode"])), "block": cfg["block"],
            "cells_per_lane": cfg["cells_per_lane"]}


def measure_format(storage, n, steps, warmup, diag_every=0):
    g, flags = cavity(n, storage)
    try:
        g.step(2)
        cfg = g.autotune(5)                      # leaves the state unchanged
        chunks = []
        ms = time_steps(g, steps, warmup, chunks)
        d = g.diagnostics(0)
        diag = diag_cost(g, flags, 19, storage, diag_every, 5 * diag_every) if diag_every else None
    finally:
        g.close()
    N = n ** 3
    n_fluid = int(np.count_nonzero(flags == 0))
    b = ddf_bytes(storage)
    alg_bytes = n_fluid * (2 * 19 * b + 1) + (N - n_fluid) * 1
    gbs = alg_bytes / (ms * 1e-3) / 1e9
    return {"storage": storage, "ms_per_step": ms, "mlups": N / (ms * 1e-3) / 1e6,
            "mlups_fluid": n_fluid / (ms * 1e-3) / 1e6, "alg_bytes_per_launch": alg_bytes,
            "achieved_GBps": gbs, "frac_of_8TBps": gbs / HBM_PEAK_GBS,
            "kinetic_energy": d["kinetic_energy"], "nonfinite": d["nonfinite_cells"],
            "nonfinite_updates": d["nonfinite_updates"],
            "launch": launch_desc(cfg), "diagnostics": diag,
            "runs_ms_per_step": [round(c, 4) for c in chunks],
            "runs_median_ms": round(float(np.median(chunks)), 4) if chunks else None,
            "runs_spread": round((max(chunks) - min(chunks)) / float(np.median(chunks)), 4) if chunks else None}


def periodic_box(steps=50, warmup=5):
    """The paper's performance workload (its Table 5): D3Q19 SRT on a periodic
    256^3 box without boundaries, in the five arithmetic/storage columns the
    paper reports (FP64/FP64, FP64/FP32, FP32/FP32, FP32/FP16S, FP32/FP16C);
    the SRT/TRT/MRT triplet of its roofline (Sec. 5); and the other velocity
    sets with FP32 and FP16S storage (D2Q9 on a 4096^2 box, D3Q15 and D3Q27
    on 256^3).  Each configuration is autotuned first.  Bytes per cell are
    the algorithmic 2 Q b + 1."""
    import paper_2112_08926_amd as lbm
    import lbm_workloads as wl
    rows = []
    cols = [(19, "srt", "fp64", "fp64"), (19, "srt", "fp64", "fp32"), (19, "srt", "fp32", "fp32"),
            (19, "srt", "fp32", "fp16s"), (19, "srt", "fp32", "fp16c"),
            (19, "trt", "fp32", "fp32"), (19, "trt", "fp32", "fp16s"), (19, "trt", "fp32", "fp16c"),
            (19, "mrt", "fp32", "fp32"), (19, "mrt", "fp32", "fp16s"), (19, "mrt", "fp32", "fp16c"),
            (9, "srt", "fp32", "fp32"), (9, "srt", "fp32", "fp16s"), (15, "srt", "fp32", "fp32"),
            (15, "srt", "fp32", "fp16s"), (27, "srt", "fp32", "fp32"), (27, "srt", "fp32", "fp16s")]
    for q, coll, arith, storage in cols:
        nx, ny, nz = (4096, 4096, 1) if q == 9 else (256, 256, 256)
        p = lbm.make_params(nx, ny, nz, q=q, collision=coll, storage=storage, arith=arith, tau=0.6)
        g = lbm.Lattices(p)
        try:
            rho, u = wl.taylor_green_fields(nx, ny, nz, 0.05)
            g.set_rho_u(0, rho, u)
            cfg = g.autotune(2)
            ms = time_steps(g, steps, warmup)
        finally:
            g.close()
        N = nx * ny * nz
        gbs = N * (2 * q * ddf_bytes(storage) + 1) / (ms * 1e-3) / 1e9
        rows.append({"velset": f"D{2 if q == 9 else 3}Q{q}", "collision": coll, "arith": arith, "storage": storage,
                     "cells": N, "ms_per_step": round(ms, 4), "mlups": round(N / (ms * 1e-3) / 1e6, 1),
                     "achieved_GBps": round(gbs, 1), "frac_of_8TBps": round(gbs / HBM_PEAK_GBS, 4),
                     "launch": {k: cfg[k] for k in ("mode", "block", "cells_per_lane")}})
        print(f"[bench] periodic {rows[-1]['velset']} {coll} {arith}/{storage}: {rows[-1]['mlups']:.0f} MLUPs/s, "
              f"{gbs:.0f} GB/s", file=sys.stderr, flush=True)
    return rows


def ensemble(storage="fp16s", count=256, steps=50, warmup=10):
    """The batched workload: `count` independent D3Q19 BGK lattices with sizes
    uniform in 32..96 per axis and tau uniform in [0.55, 1.0] (splitmix64,
    seed 2112), half Taylor-Green, half Poiseuille.  MLUPs/s of one launch
    per lattice per step, one batched launch per step over row tiles and over
    cell-contiguous tiles, the persistent batched launch (8 workgroups of 256
    per CU: full occupancy), the same replayed as a HIP graph of 100 steps,
    and the autotuned configuration."""
    import paper_2112_08926_amd as lbm
    import lbm_workloads as wl
    specs = wl.ensemble_specs(count=count, seed=2112, lo=32, hi=96)
    params = [lbm.make_params(sp["nx"], sp["ny"], sp["nz"], q=19, collision="srt", storage=storage,
                              tau=sp["tau"], force=sp["force"]) for sp in specs]
    cells = sum(sp["nx"] * sp["ny"] * sp["nz"] for sp in specs)
    g = lbm.Lattices(params)
    fluid = 0
    try:
        for k, sp in enumerate(specs):
            flags, rho, u = wl.ensemble_member_inputs(sp)
            fluid += int(np.count_nonzero(flags == 0))
            g.set_boundaries(k, flags)
            g.set_rho_u(k, rho, u)
        out = {"lattices": count, "cells": cells, "storage": storage}
        for name, cfg in [("per_lattice", dict(mode=0, block=128, cells_per_lane=1, persistent=0,
                                                 graph_steps=0)),
                          ("batched_rows", dict(mode=1, block=128, cells_per_lane=1, persistent=0,
                                                graph_steps=0)),
                          ("batched", dict(mode=2, block=256, cells_per_lane=1, persistent=0,
                                           graph_steps=0)),
                          ("persistent", dict(mode=2, block=256, cells_per_lane=1, persistent=8,
                                              graph_steps=0)),
                          ("persistent_graph100", dict(mode=2, block=256, cells_per_lane=1,
                                                       persistent=8, graph_steps=100))]:
            g.set_launch(**cfg)
            n = 100 if cfg["graph_steps"] else steps
            ms = time_steps(g, n, warmup if not cfg["graph_steps"] else 100)
            out[name + "_mlups"] = round(cells / (ms * 1e-3) / 1e6, 1)
            print(f"[bench] ensemble {storage} {name}: {out[name + '_mlups']:.0f} MLUPs/s", file=sys.stderr,
                  flush=True)
        g.set_launch(graph_steps=0)
        best = g.autotune(3)
        g.set_launch(graph_steps=100)
        ms = time_steps(g, 100, 100)
        out["autotuned"] = {k: best[k] for k in ("mode", "block", "cells_per_lane", "persistent")}
        out["autotuned_graph100_mlups"] = round(cells / (ms * 1e-3) / 1e6, 1)
        print(f"[bench] ensemble {storage} autotuned {out['autotuned']}: {out['autotuned_graph100_mlups']:.0f} "
              "MLUPs/s", file=sys.stderr, flush=True)
        # algorithmic bytes: 2 Q b + 1 per fluid cell, the flag byte per wall cell
        alg = fluid * (2 * 19 * ddf_bytes(storage) + 1) + (cells - fluid)
        out["fluid_cells"] = fluid
        out["autotuned_alg_bytes_per_step"] = alg
        out["autotuned_GBps"] = round(alg / (ms * 1e-3) / 1e9, 1)
        out["autotuned_frac_of_8TBps"] = round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        return out
    finally:
        g.close()


def karman(storages=("fp16s", "fp16c", "fp32"), steps=50, warmup=10):
    """The Karman channel at full size: 1024 x 256 x 64, D3Q27 TRT (magic
    1/4), cylinder of radius 16 along z at (256, 128), equilibrium inflow and
    outflow cells with u = 0.05 on the x and y faces, tau 0.532 (Re = 150 on
    the diameter), FP32 arithmetic.  Per storage: MLUPs/s of the autotuned
    step from the asymmetric start, and the FP64 momentum-exchange force on
    the cylinder after the timed steps."""
    import paper_2112_08926_amd as lbm
    import lbm_workloads as wl
    nx, ny, nz, R, u0, tau = 1024, 256, 64, 16.0, 0.05, 0.532
    flags = wl.karman_flags(nx, ny, nz, R, nx / 4, ny / 2)
    rho, u = wl.karman_fields(nx, ny, nz, u0)
    N = nx * ny * nz
    n_fluid = int(np.count_nonzero(flags == 0))
    rows = []
    for storage in storages:
        p = lbm.make_params(nx, ny, nz, q=27, collision="trt", storage=storage, tau=tau,
                            eq_rho=1.0, eq_u=(u0, 0.0, 0.0))
        g = lbm.Lattices(p)
        try:
            g.set_boundaries(0, flags)
            g.set_rho_u(0, rho, u)
            g.step(2)
            cfg = g.autotune(5)
            ms = time_steps(g, steps, warmup)
            d = g.diagnostics(0)
            diag = diag_cost(g, flags, 27, storage, 10, 200)
        finally:
            g.close()
        alg = n_fluid * (2 * 27 * ddf_bytes(storage) + 1) + (N - n_fluid)
        gbs = alg / (ms * 1e-3) / 1e9
        rows.append({"storage": storage, "cells": N, "ms_per_step": round(ms, 4),
                     "mlups": round(N / (ms * 1e-3) / 1e6, 1), "achieved_GBps": round(gbs, 1),
                     "frac_of_8TBps": round(gbs / HBM_PEAK_GBS, 4),
                     "force_on_cylinder": [float(v) for v in d["force_on_solid"]],
                     "nonfinite": d["nonfinite_cells"], "drag_every_10": diag,
                     "launch": launch_desc(cfg)})
        print(f"[bench] karman D3Q27 {storage}: {rows[-1]['mlups']:.0f} MLUPs/s, {gbs:.0f} GB/s",
              file=sys.stderr, flush=True)
    return {"workload": "Karman channel 1024x256x64, D3Q27 TRT, cylinder R 16, EQ inflow/outflow u 0.05, "
                        "tau 0.532 (Re 150)", "steps_from_start": steps + warmup + 2, "rows": rows}


def placement(n=512, handles=5, steps=50, warmup=10):
    """The headline step (512 threads, one cell per lane) on fresh handles
    whose buffers land in different places: before handle k the allocator's
    cache is emptied and a spacer of k (64 MiB + 4 KiB) is taken and held, so
    every handle's DDF buffers start at a different address and on different
    physical pages.  ms per step of each (events, as the headline)."""
    import torch
    times, spacers = [], []
    for k in range(handles):
        torch.cuda.empty_cache()
        spacers.append(torch.empty(k * ((64 << 20) + 4096) + 4096, dtype=torch.uint8, device="cuda"))
        g, _ = cavity(n, HEADLINE)
        try:
            g.set_launch(mode=0, block=512, cells_per_lane=1)
            times.append(time_steps(g, steps, warmup))
        finally:
            g.close()
    del spacers
    torch.cuda.empty_cache()
    med = float(np.median(times))
    return {"handles": handles, "steps": steps, "ms_per_step": [round(t, 4) for t in times],
            "spread": round((max(times) - min(times)) / med, 4)}


def memory_bandwidths(nbytes=4 << 30, reps=10):
    """Achievable HBM bandwidth of the library's memory microbenchmarks (the
    paper's appendix memory benchmarks): a plain copy (bytes read + bytes
    written) and coalesced / misaligned 4-byte reads and writes, each timed
    over `reps` launches on 4 GiB buffers, in GB/s."""
    import torch
    import paper_2112_08926_amd as lbm
    a = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")   # zero source: the read sink is never written
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    out = {}
    for kind in ("copy", "read", "read_misaligned", "write", "write_misaligned"):
        lbm.lbm_memory_probe(kind, a.data_ptr(), b.data_ptr(), nbytes, stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            lbm.lbm_memory_probe(kind, a.data_ptr(), b.data_ptr(), nbytes, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        moved = 2 * nbytes if kind == "copy" else nbytes - (4 if kind.endswith("misaligned") else 0)
        out[kind] = round(moved / (ms * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def accuracy_vs_fp64(formats, n=64, steps=1000):
    """Relative L2 of u of each storage format against the FP64 GPU path on the
    same cavity (the FP64 path matches the CPU reference to 1e-12)."""
    ref_g, _ = cavity(n, "fp64")
    ref_g.step(steps)
    _, u_ref = ref_g.get_rho_u(0)
    ref_g.close()
    out = {}
    for s in formats:
        g, _ = cavity(n, s)
        g.step(steps)
        _, u = g.get_rho_u(0)
        g.close()
        out[s] = float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref))
    return out


def traffic_from_profile(storage):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel code, comments aside (else None)."""
    path = os.path.join(ROOT, "profiles", f"ldc512_{storage}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(budget_s=12.0):
    """The FP64 CPU reference timed on the host cores: the same cavity at a
    reduced 128^3, D3Q19 TRT, FP64 arithmetic with FP16S storage emulation,
    as many steps as fit the time budget (at least 2) with all the threads
    OpenMP is given, then the same on one thread."""
    import oracle
    import lbm_workloads as wl
    n = 128
    flags = wl.cavity_flags(n, n, n)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))

    def rate(nthreads, budget):
        lat = oracle.Lattice(n, n, n, q=19, tau=0.6, collision="trt", storage=HEADLINE,
                             wall_u=(0.0, 0.1, 0.0), flags=flags, nthreads=nthreads).init()
        t0 = time.perf_counter()
        lat.step(1)
        one = time.perf_counter() - t0
        steps = max(2, int(budget / max(one, 1e-3)))
        t0 = time.perf_counter()
        lat.step(steps)
        dt = time.perf_counter() - t0
        return n ** 3 * steps / dt / 1e6, steps, dt

    v, steps, dt = rate(threads, budget_s)
    v1, steps1, dt1 = rate(1, budget_s / 2)
    return {"value": v, "unit": "MLUPs/s", "cores": threads, "kind": "oracle",
            "sample": f"cavity {n}^3 D3Q19 TRT FP64 arithmetic, FP16S storage emulated, {steps} steps, "
                      f"{dt:.1f} s on {threads} threads; {steps1} steps, {dt1:.1f} s on 1 thread",
            "one_core_value": v1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=512, help="cavity edge length")
    ap.add_argument("--formats", default="all", help="'all', 'headline' or a comma list")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU reference timing")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 256-lattice ensembles")
    ap.add_argument("--no-karman", action="store_true", help="skip the full-size Karman channel (D3Q27)")
    ap.add_argument("--placement", type=int, default=0,
                    help="also time the headline step on this many fresh handles placed apart")
    ap.add_argument("--no-periodic", action="store_true",
                    help="skip the periodic-box runs (the paper's performance workload, other velocity sets)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the step runs on one GPU; --gpus {args.gpus} is not supported (splitting the "
              "lattice into z slabs with a halo exchange per step is not implemented)", file=sys.stderr)
        return 2
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    import paper_2112_08926_amd  # noqa: F401  (fails loudly without liblbm.so)

    formats = [HEADLINE] + (OTHERS if args.formats == "all" else
                            ([] if args.formats == "headline" else
                             [f for f in args.formats.split(",") if f != HEADLINE]))
    results = {}
    for s in formats:
        print(f"[bench] {s} {args.n}^3 ...", file=sys.stderr, flush=True)
        results[s] = measure_format(s, args.n, args.steps, args.warmup, diag_every=100 if s == HEADLINE else 0)
        print(f"[bench] {s}: {results[s]['mlups']:.0f} MLUPs/s, "
              f"{results[s]['achieved_GBps']:.0f} GB/s, launch {results[s]['launch']}",
              file=sys.stderr, flush=True)
    head = results[HEADLINE]
    print("[bench] memory probes", file=sys.stderr, flush=True)
    probes = memory_bandwidths()
    copy_gbs = probes["copy"]
    acc = None
    if not args.no_accuracy:
        print("[bench] accuracy vs FP64 (64^3, 1000 steps)", file=sys.stderr, flush=True)
        acc = accuracy_vs_fp64([s for s in formats if s != "fp64"])
    ens = None
    if not args.no_ensemble:
        print("[bench] ensemble of 256 lattices", file=sys.stderr, flush=True)
        ens = {s: ensemble(s) for s in ("fp16s", "fp16c")}
    kar = None
    if not args.no_karman:
        print("[bench] Karman channel 1024x256x64", file=sys.stderr, flush=True)
        kar = karman()
    per = None
    if not args.no_periodic:
        print("[bench] periodic boxes", file=sys.stderr, flush=True)
        per = periodic_box()
    place = None
    if args.placement > 0:
        print(f"[bench] placement: {args.placement} fresh handles", file=sys.stderr, flush=True)
        place = placement(args.n, args.placement)
    cpu = None
    if not args.no_cpu:
        print("[bench] CPU reference timing", file=sys.stderr, flush=True)
        cpu = cpu_baseline()
    traffic = traffic_from_profile(HEADLINE)
    line = {
        "metric": "MLUPs/s and % of HBM roofline, D3Q19 FP32/16-bit vs FP32/FP32, L2 err vs FP64",
        "value": round(head["mlups"], 1),
        "unit": "MLUPs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"lid-driven cavity {args.n}^3, D3Q19 TRT (Lambda 1/4), tau 0.6, lid 0.1, "
                               f"FP32 arithmetic / FP16S storage",
                   "cells": args.n ** 3, "storage": HEADLINE, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(head["achieved_GBps"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(head["frac_of_8TBps"], 4),
                     "traffic": traffic, "copy_probe_GBps": round(copy_gbs, 1),
                     "frac_of_copy": round(head["achieved_GBps"] / copy_gbs, 4)},
        "cpu_baseline": cpu,
        "formats": {s: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
                    for s, r in results.items()},
        "fp16s_vs_fp32_speedup": (round(head["mlups"] / results["fp32"]["mlups"], 3)
                                  if "fp32" in results else None),
        "memory_probes_GBps": probes,
        "l2_vs_fp64": acc,
        "ensemble": ens,
        "karman": kar,
        "periodic_box": per,
        "placement": place,
        "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
