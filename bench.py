"""Benchmark of the MAP block update on one MI355X.

Workload (default): the 3-D Harris current sheet, base 128^3, 4 levels
(22016 blocks of 16^3 cells, 19328 leaves = 79.2 M leaf cells), FP32 state
with FP64 pressure recovery / CFL, LF + minmod, FASTSPEED GLM, eta = 1e-3,
one batched persistent launch per stage, the step cycle captured in a HIP
graph.  A step = cfl_dt + step + reflux + restriction + ghost fill over all
leaves.  value = leaf cell-updates per second (inputs resident in HBM).

Also reported on the same workload and initial data:
  * whole WENO + TVD Runge-Kutta 2 cycles (Sec. 3.3), with the Rusanov and
    with the HLLC face flux, their rates and the time of one two-stage
    update;
  * whole LF cycles with the thermal-conduction subcycle (Sec. 3.4) along the
    field, their rate and the time per sub-step;
  * the FP64 path launched once per block ("plain") and its rate;
  * roofline of the dominant kernel (the step kernel), timed with HIP events
    on the stream it is launched on;
  * the FP64 CPU oracle on a bounded sample, the reduced Harris sheet (base
    32^3, 4 levels), on all host cores and on one (cpu_baseline), and the
    relative L1 distance of the FP32 batched path from the oracle after the
    same cycles of that sample (l1_fp32_vs_oracle).

    python bench.py [--gpus 1] [--steps 50] [--warmup 3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "cell-updates/s at fixed L1 err, FP32 batched vs FP64 plain; % HBM peak"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_workload(name, precision):
    from paper_1204_5849_amd import workloads as W
    if name == "harris3d":
        return W.harris3d(nbase=8, levels=4, precision=precision)
    if name == "blast3d":
        return W.blast3d(nbase=8, levels=2, precision=precision)
    if name == "kh_ensemble":
        return W.kh_ensemble(nsims=64, precision=precision)
    if name == "orszag_tang":
        return W.orszag_tang(8, precision=precision)
    if name == "ot_amr":
        keys = np.loadtxt(os.path.join(ROOT, "tests", "golden", "ot_amr_grid.txt"), dtype=np.int32,
                          comments="#")
        return W.ot_amr(keys, precision=precision)
    raise SystemExit(f"unknown workload {name}")


def step_bytes_per_launch(wl, nleaves, word):
    """Algorithmic HBM bytes of one step launch: every leaf reads its padded
    tile (20^d cells x 9 variables) and writes its interior (16^d x 9)."""
    P = 20 ** wl.ndim
    I = 16 ** wl.ndim
    return nleaves * 9 * (P + I) * word


# FP operations of the LF block update per leaf cell-update (add, sub, mul,
# div, sqrt: 1; fused multiply-add: 2), counted from the scheme as the step
# kernel evaluates it, including the ring of cells one outside the interior
# that a per-block update must predict (5632 cells per 4096 in 3-D, 320 per
# 256 in 2-D).  Per predicted cell (3-D): slopes 81, six half-step states
# 6 x (18 state + 28 primitives + 28 flux) = 444, flux differences 81,
# u~ 9, six face states 6 x (18 + 28) = 276 -> 891 x 1.375 = 1225.  Per face:
# primitives 18, two fluxes 56, two fast speeds 28, Rusanov combination 45,
# max 1 -> 148, three faces per cell -> 444.  Update 81, EGLM sources 33,
# resistivity 75, psi damping 1.  2-D: (54 + 296 + 54 + 9 + 184) x 1.25 =
# 746, two faces 296, update 54, sources 26, damping 1.
FLOPS_PER_CELL = {(3, True): 1860, (3, False): 1785, (2, True): 1123 + 60, (2, False): 1123}

# FP operations of one WENO stage per leaf cell-update, counted the same way
# (Sec. 3.3): per cell, dimension and variable the two WENO face states cost
# 30 (differences 2, smoothness 4, squares 2, each state 11 with one
# division), primitives of the six face states 168 -> 978 in 3-D; the ring
# of cells outside the interior needs one face state each (30 x 9 + 28 =
# 298 for 1536 ring cells per 4096); faces 444, update 81, EGLM sources 33,
# resistivity 75; stage 2 adds the Runge-Kutta average (18) and the psi
# damping (1).  2-D: 540 + 112 = 652, ring 64 x 298 / 256, faces 296,
# update 54, sources 26, resistivity 60.
WENO_FLOPS_PER_CELL = {(3, True): (1723, 1742), (3, False): (1648, 1667),
                       (2, True): (1163, 1182), (2, False): (1103, 1122)}

# The HLLC face flux in place of the Rusanov one, counted the same way for a
# face inside the fan: the GLM pair 12, per side the state with B_d = B_m
# (primitives 9, pressure 6, flux 28, total pressure 2, fast speed 15,
# v.B 5) 65, outer speeds 5, HLL mean and contact speed 66, star state 25,
# flux 24, psi flux 1 -> 263 against 148 for Rusanov: 115 more per face.
HLLC_EXTRA_PER_FACE = 115

# MI355X vector peak for FP32 (non-packed) and FP64: 256 CUs x 4 SIMDs x
# 16 lanes x 2 (FMA) x 2.4 GHz = 78.6 TFLOP/s
ALU_PEAK_TFLOPS = 78.6


def step_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("k_step2.hip", "k_step3.hpp", "k_step3_ilp.hip", "k_step3.hip", "step_common.hpp",
              "tile.hpp", "physics.hpp", "kernels.hpp", "map_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1204_5849_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# library sources whose code the 3-D LF cycle does not run (regrid, the
# conduction subcycle, MMC and the 2-D update): a change to them leaves the
# cycle's counters valid
NOT_IN_3D_LF_CYCLE = ("k_regrid.hip", "regrid.cpp", "k_cond.hip", "k_step_mmc.hip",
                      "k_step_mmc3.hip", "k_step2.hip")


def cycle_sources_hash():
    """Hash of the library sources the 3-D LF cycle runs (every source but
    those above)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1204_5849_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".cpp", ".h")) and f not in NOT_IN_3D_LF_CYCLE:
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_cycle_bytes(workload_name):
    """HBM bytes of one whole cycle (all its dispatches) from the committed
    counter summary, if it was taken on the current sources of the cycle."""
    path = os.path.join(ROOT, "profiles", f"{workload_name}_fp32_hbm_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("cycle_traffic:"):
            for kv in line.split()[1:]:
                k, v = kv.split("=")
                vals[k] = v
    if vals.get("sources") != cycle_sources_hash() or "bytes" not in vals:
        return None
    return int(vals["bytes"])


def measured_valu_busy(workload_name):
    """VALU busy fraction of the step kernel from the committed SQ-counter
    summary, if it was taken on the current step-kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"{workload_name}_fp32_step_sq_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("step_valu:"):
            for kv in line.split()[1:]:
                k, v = kv.split("=")
                vals[k] = v
    if vals.get("sources") != step_sources_hash() or "busy" not in vals:
        return None
    return float(vals["busy"])


def measured_traffic(workload_name):
    """HBM bytes per step launch from the committed counter summary, if it was
    taken on the current step-kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"{workload_name}_fp32_hbm_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("step_traffic:"):
            for kv in line.split()[1:]:
                k, v = kv.split("=")
                vals[k] = v
    if vals.get("sources") != step_sources_hash() or "bytes" not in vals:
        return None
    return int(vals["bytes"])


def time_step_kernel(sim, reps):
    """Average duration of the step kernel alone (HIP events on its stream)."""
    import torch
    from paper_1204_5849_amd import native as N
    s = sim.stream
    sim.cfl()
    out = torch.empty_like(sim.U)  # the update must not write its input
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    N.map_step(sim.ctx, sim.U, out, sim.dt, sim.sp)  # warm
    e0.record(s)
    for _ in range(reps):
        N.map_step(sim.ctx, sim.U, out, sim.dt, sim.sp)
    e1.record(s)
    e1.synchronize()
    del out
    return e0.elapsed_time(e1) / reps * 1e-3


def _reduced_harris(precision):
    """The Harris sheet at base 32^3 with 4 levels (1352 blocks, 4.85 M leaf
    cells): the headline problem at a size the oracle finishes in seconds."""
    from paper_1204_5849_amd import workloads as W
    return W.harris3d(nbase=2, levels=4, precision=precision)


def host_threads():
    """Host cores this process may use, at most 16 (one GPU's share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline_and_l1(cycles=10, one_core_cycles=3):
    """The FP64 oracle on the reduced Harris sheet: `cycles` whole cycles on
    all host cores (OpenMP over blocks) and `one_core_cycles` on one core,
    each timed around its cycle loop; then the FP32 batched GPU path
    (autotuned, graph-captured) runs the same cycles on the same blocks and
    data, and its volume-weighted relative L1 distance from the oracle's
    state is reported per variable."""
    import torch
    import oracle as orc
    from paper_1204_5849_amd.sim import Simulation
    orc.build(force=False)
    w = _reduced_harris("fp64")
    cells = w.n_leaf_cells()
    threads = host_threads()
    orc.set_threads(threads)
    A = orc.load_workload(w)
    t0 = time.perf_counter()
    A.run(cycles)
    tN = time.perf_counter() - t0
    orc.set_threads(1)
    A1 = orc.load_workload(w)
    t0 = time.perf_counter()
    A1.run(one_core_cycles)
    t1 = time.perf_counter() - t0
    del A1
    sample = (f"FP64 oracle, {{n}} whole cycle(s) of the Harris sheet at base 32^3 with 4 levels "
              f"({len(w.keys)} blocks, {cells} leaf cells)")
    base = {"value": cells * cycles / tN, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle", "sample": sample.format(n=cycles) + f", {threads} threads",
            "seconds": round(tN, 2),
            "one_core": {"value": cells * one_core_cycles / t1, "cores": 1,
                         "sample": sample.format(n=one_core_cycles) + ", 1 thread",
                         "seconds": round(t1, 2)}}
    w32 = _reduced_harris("fp32")
    sim = Simulation(w32, precision="fp32")
    sim.load_initial()
    sim.autotune()
    sim.graph_run(cycles)
    sim.sync()
    leaves = np.nonzero(w32.leaf_mask())[0]
    g = sim.state_by_key(leaves)[:, :, 2:-2, 2:-2, 2:-2]
    o = A.state[leaves][:, :, 2:-2, 2:-2, 2:-2]
    vol = np.array([np.prod(w.dx(int(k[0]), int(k[1]))) for k in w.keys[leaves]])
    vol = vol[:, None, None, None]

    def rl1(a, b):
        return float((np.abs(a - b) * vol).sum() / max((np.abs(b) * vol).sum(), 1e-300))

    bg = np.sqrt((g[:, 4:7] ** 2).sum(axis=1))
    bo = np.sqrt((o[:, 4:7] ** 2).sum(axis=1))
    names = ["rho", "mx", "my", "mz", "Bx", "By", "Bz", "e", "psi"]
    l1 = {n: rl1(g[:, k], o[:, k]) for k, n in enumerate(names)}
    l1["absB"] = rl1(bg, bo)
    del sim
    torch.cuda.empty_cache()
    orc.set_threads(1)
    l1_out = {"workload": "harris3d_32_L4", "cycles": cycles, "rel_l1": l1,
              "tolerance": 1e-6,
              "within_tolerance": all(l1[k] <= 1e-6 for k in ("rho", "e", "absB")),
              "note": "FP32 batched path (graph, autotuned) against the FP64 oracle after the "
                      "same whole cycles from the same initial data; volume-weighted relative "
                      "L1 over leaf interiors (each path forms its own dt)"}
    return base, l1_out


def leaf_rel_l1(w, sim, A):
    """Volume-weighted relative L1 of the GPU state (sim) against the oracle's
    (A) over leaf interiors, per variable and for |B|."""
    leaves = np.nonzero(w.leaf_mask())[0]
    num, den = np.zeros(10), np.zeros(10)
    ng = 2
    for s0 in range(0, len(leaves), 2048):
        idx = leaves[s0:s0 + 2048]
        g, o = sim.state_by_key(idx), A.state[idx]
        if w.ndim == 3:
            g, o = g[:, :, ng:-ng, ng:-ng, ng:-ng], o[:, :, ng:-ng, ng:-ng, ng:-ng]
        else:
            g, o = g[:, :, :, ng:-ng, ng:-ng], o[:, :, :, ng:-ng, ng:-ng]
        vol = np.array([np.prod(w.dx(int(k[0]), int(k[1]))[:w.ndim]) for k in w.keys[idx]])
        vol = vol[:, None, None, None]
        for k in range(9):
            num[k] += float((np.abs(g[:, k] - o[:, k]) * vol).sum())
            den[k] += float((np.abs(o[:, k]) * vol).sum())
        bg, bo = np.sqrt((g[:, 4:7] ** 2).sum(axis=1)), np.sqrt((o[:, 4:7] ** 2).sum(axis=1))
        num[9] += float((np.abs(bg - bo) * vol).sum())
        den[9] += float((np.abs(bo) * vol).sum())
    names = ["rho", "mx", "my", "mz", "Bx", "By", "Bz", "e", "psi", "absB"]
    return {n: num[i] / max(den[i], 1e-300) for i, n in enumerate(names)}


def time_cycles(sim, steps, graph=True):
    """Wall time per cycle of `steps` cycles (after two warm-up cycles)."""
    import torch
    run = sim.graph_run if graph else sim.advance
    run(2)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def plain_sim(wl, precision):
    """The per-block ("plain") path: one launch per block and stage.  In 2-D
    it takes the 7-block, two-wave workgroup shape: a launch holds one block,
    and that shape runs it with fewer idle waves and no spilled registers
    (1.32 s against 1.79 s per cycle of the KH ensemble in FP32)."""
    from paper_1204_5849_amd.sim import Simulation
    p = Simulation(wl, precision=precision, launch="per_block")
    if wl.ndim == 2 and wl.scheme != "mmc":
        p.set_launch_config(step_shape=1)
    return p


def measure_config(key, precision_b, precision_p, steps_b, steps_p, l1_cycles=0,
                   plain_graph=False, batched_only=False):
    """One configuration besides the headline: its batched path (autotuned,
    graph-captured) in precision_b, its per-block ("plain") path in
    precision_p (one launch per block and stage), and, if l1_cycles, the
    batched path's relative L1 against the FP64 oracle after that many whole
    cycles from the same initial data."""
    import torch
    import oracle as orc
    from paper_1204_5849_amd.sim import Simulation
    wb = build_workload(key, precision_b)
    cells = wb.n_leaf_cells()
    out = {"workload": wb.name, "blocks": int(len(wb.keys)), "leaves": int(wb.leaf_mask().sum()),
           "leaf_cells": int(cells), "simulations": len(wb.sims), "scheme": wb.scheme,
           "limiter": wb.limiter}
    sim = Simulation(wb, precision=precision_b)
    sim.load_initial()
    cfg = sim.autotune()
    tb = time_cycles(sim, steps_b)
    st, cnt = sim.flags()
    out["batched"] = {"precision": precision_b, "value": cells / tb, "ms_per_step": tb * 1e3,
                      "steps": steps_b, "launch": launch_label(cfg, False),
                      "launch_config": cfg, "flags": [int(c) for c in cnt]}
    out["roofline"] = config_roofline(wb, sim, precision_b)
    del sim
    torch.cuda.empty_cache()
    if batched_only:
        return out
    wp = build_workload(key, precision_p)
    p = plain_sim(wp, precision_p)
    p.load_initial()
    tp = time_cycles(p, steps_p, graph=plain_graph)
    out["plain"] = {"precision": precision_p, "value": cells / tp, "ms_per_step": tp * 1e3,
                    "steps": steps_p, "launch": "one launch per block and stage",
                    "launch_config": p.launch_config()}
    out["speedup_batched_vs_plain"] = tp / tb
    del p
    torch.cuda.empty_cache()
    if l1_cycles:
        w64 = build_workload(key, "fp64")
        orc.build(force=False)
        orc.set_threads(host_threads())
        A = orc.load_workload(w64)
        t0 = time.perf_counter()
        A.run(l1_cycles)
        tN = time.perf_counter() - t0
        n1 = max(1, min(l1_cycles, int(2e6 // max(cells, 1)) + 1))
        orc.set_threads(1)
        A1 = orc.load_workload(w64)
        t0 = time.perf_counter()
        A1.run(n1)
        t1 = time.perf_counter() - t0
        del A1
        out["oracle"] = {"kind": "oracle", "unit": "cell-updates/s",
                         "value": cells * l1_cycles / tN, "cores": host_threads(),
                         "sample": f"FP64 oracle, {l1_cycles} whole cycles of this configuration",
                         "one_core": {"value": cells * n1 / t1, "cores": 1,
                                      "sample": f"FP64 oracle, {n1} whole cycle(s), 1 thread"}}
        q = Simulation(wb, precision=precision_b)
        q.load_initial()
        q.set_launch_config(**cfg)
        q.graph_run(l1_cycles)
        q.sync()
        out["rel_l1_vs_oracle"] = {"cycles": l1_cycles, "precision": precision_b,
                                   **leaf_rel_l1(w64, q, A)}
        del q, A
        torch.cuda.empty_cache()
    return out


def config_roofline(wl, sim, precision):
    """The step kernel of a configuration's batched path alone (HIP events on
    its stream): duration, algorithmic HBM rate and fraction of 8 TB/s, and for
    LF the algorithmic FLOP rate and fraction of the vector peak (the FLOP
    count of MMC is not tabulated); `bound` names the roof with the larger
    fraction."""
    nleaves = int(wl.leaf_mask().sum())
    cells = wl.n_leaf_cells()
    ms = time_step_kernel(sim, 10) * 1e3
    word = 8 if precision == "fp64" else 4
    nbytes = step_bytes_per_launch(wl, nleaves, word)
    gbs = nbytes / ms * 1e-6
    r = {"kernel_ms": ms, "algorithmic_bytes_per_launch": nbytes, "hbm_achieved_GBs": gbs,
         "hbm_peak_GBs": HBM_PEAK_GBS, "hbm_frac": gbs / HBM_PEAK_GBS}
    fpc = FLOPS_PER_CELL.get((wl.ndim, wl.eta > 0)) if wl.scheme == "lf" else None
    if fpc is not None:
        tflops = fpc * cells / ms * 1e-9
        r.update({"flops_per_cell_update": fpc, "alu_achieved_TFLOPs": tflops,
                  "alu_peak_TFLOPs": ALU_PEAK_TFLOPS, "alu_frac": tflops / ALU_PEAK_TFLOPS})
    r["bound"] = "alu" if fpc is not None and r["alu_frac"] > r["hbm_frac"] else "hbm"
    return r


# the configurations measured besides the headline: key -> (batched precision,
# plain precision, batched cycles, plain cycles, oracle L1 cycles)
CONFIGS = {
    "orszag_tang": ("fp64", "fp64", 100, 20, 100),
    "ot_amr": ("fp64", "fp64", 100, 5, 20),
    "blast3d": ("fp32", "fp64", 20, 2, 10),
    "kh_ensemble": ("fp32", "fp32", 50, 3, 10),
}


def cycle_bytes_per_cell(wl, word):
    """Algorithmic bytes of one whole cycle per leaf cell, counted for a
    padded-ghost per-block method (the fill reads and writes the ghost frame,
    the step reads the padded tile and writes the interior): 9 w (3P - I) / I."""
    P, I = 20 ** wl.ndim, 16 ** wl.ndim
    return 9 * word * (3 * P - I) / I


def gather_bytes_per_cell(wl, word):
    """The same for an update that reads its ghost cells from the neighbours'
    interiors in place (as here): 9 w (P + I) / I."""
    P, I = 20 ** wl.ndim, 16 ** wl.ndim
    return 9 * word * (P + I) / I


def time_regrid(sim, wl):
    """One regrid of the current state (Sec. 4.5): the estimator kernel (rho
    and |B| criteria, HIP events on the launch stream), the host tree edit,
    and the remap of the state onto the new tree on device.  Thresholds:
    refine the 2 % roughest leaves below the finest level, coarsen the
    quarter smoothest blocks whose children are all leaves."""
    import torch
    from paper_1204_5849_amd import native as N
    from paper_1204_5849_amd.sim import Simulation
    est = N.make_estimator([("var", 0, 1e-12), ("bmag", 0, 0.1)])
    err = torch.zeros(sim.nslots, dtype=torch.float64, device=sim.device)
    torch.cuda.synchronize()
    N.map_estimate(sim.ctx, sim.U, est, err, sim.sp)  # warm
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    for _ in range(3):
        N.map_estimate(sim.ctx, sim.U, est, err, sim.sp)
    e1.record(sim.stream)
    e1.synchronize()
    t_est = e0.elapsed_time(e1) / 3 * 1e-3
    err_slot = err.cpu().numpy()
    keys = wl.keys
    slot = sim.slot_of_key
    leaf = wl.leaf_mask()
    lmax = int(keys[:, 1].max())
    e_key = err_slot[slot]
    cand_r = e_key[leaf & (keys[:, 1] < lmax)]
    tr = float(np.quantile(cand_r, 0.98)) if len(cand_r) else float("inf")
    tc = float(np.quantile(e_key[~leaf], 0.25)) if (~leaf).any() else -1.0
    t0 = time.perf_counter()
    new_keys = N.map_regrid(sim.ctx, err_slot, tr, tc, lmax)
    t_tree = time.perf_counter() - t0
    import dataclasses
    new = Simulation(dataclasses.replace(wl, keys=new_keys), device=sim.device, stream=sim.stream,
                     precision=sim.precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    N.map_remap(new.ctx, new.U, sim.ctx, sim.U, sim.sp)  # synchronises the stream
    t_remap = time.perf_counter() - t0
    old = {tuple(int(v) for v in k) for k in keys}
    nk = {tuple(int(v) for v in k) for k in new_keys}
    word = 4 if sim.precision == "fp32" else 8
    # the estimator reads rho and B (4 variables) of each padded tile
    est_bytes = sim.nslots * 4 * (20 ** wl.ndim) * word
    out = {"blocks_before": len(keys), "blocks_after": len(new_keys),
           "created": len(nk - old), "destroyed": len(old - nk),
           "tau_refine": tr, "tau_coarsen": tc,
           "estimate_ms": t_est * 1e3, "estimate_algorithmic_GBs": est_bytes / t_est / 1e9,
           "tree_edit_ms": t_tree * 1e3, "remap_ms": t_remap * 1e3,
           "note": "estimator kernel timed with HIP events; tree edit on the host; remap "
                   "(copy, fill, prolongation, restriction, fill) wall time incl. one sync"}
    del new
    torch.cuda.empty_cache()
    return out


def launch_label(cfg, eager):
    """How the cycle is launched: graph or eager, batched over all blocks,
    persistent only when the autotuner chose a persistent update grid."""
    how = "eager" if eager else "hipGraph"
    if cfg is None or cfg.get("mode", 0) != 0:
        return f"{how}, one launch per block"
    kind = "persistent" if cfg.get("grid_step", 0) > 0 else "one workgroup per work item"
    return f"{how}, batched ({kind})"


def time_fp64_batched(name, steps, autotune=True):
    """The LF cycle with an FP64 state on the same workload: batched
    persistent launches captured in a HIP graph, as the FP32 headline run."""
    import torch
    from paper_1204_5849_amd.sim import Simulation
    wl64 = build_workload(name, "fp64")
    sim = Simulation(wl64, precision="fp64")
    sim.load_initial()
    chosen = sim.autotune() if autotune else sim.launch_config()
    sim.graph_run(2)
    sim.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.graph_run(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    st, cnt = sim.flags()
    t_step = time_step_kernel(sim, 5)
    out = {"ms_per_step": el / steps * 1e3, "value": wl64.n_leaf_cells() * steps / el,
           "unit": "cell-updates/s", "steps": steps, "step_kernel_ms": t_step * 1e3,
           "launch": launch_label(chosen, False), "launch_config": chosen,
           "flags": [int(c) for c in cnt], "note": "FP64 state and arithmetic"}
    del sim
    torch.cuda.empty_cache()
    return out


def time_weno(wl, precision, steps, autotune=True, riemann="rusanov"):
    """Whole WENO cycles (two stages, the boundary procedure on the stage,
    reflux, restriction, fill) on the same blocks and initial data, captured
    in a HIP graph, and map_step alone (both stages with the stage's
    restriction and fill) timed with HIP events on its stream."""
    import dataclasses
    import torch
    from paper_1204_5849_amd import native as N
    from paper_1204_5849_amd.sim import Simulation
    ww = dataclasses.replace(wl, scheme="weno", riemann=riemann)
    sim = Simulation(ww, precision=precision)
    sim.load_initial()
    if autotune:
        sim.autotune()
    sim.graph_run(2)
    sim.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.graph_run(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    st, cnt = sim.flags()
    sim.cfl()
    out = torch.empty_like(sim.U)
    torch.cuda.synchronize()
    N.map_step(sim.ctx, sim.U, out, sim.dt, sim.sp)  # warm
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    for _ in range(5):
        N.map_step(sim.ctx, sim.U, out, sim.dt, sim.sp)
    e1.record(sim.stream)
    e1.synchronize()
    t_step = e0.elapsed_time(e1) / 5 * 1e-3
    cells = ww.n_leaf_cells()
    f1, f2 = WENO_FLOPS_PER_CELL[(ww.ndim, ww.eta > 0)]
    if riemann == "hllc":
        f1, f2 = f1 + ww.ndim * HLLC_EXTRA_PER_FACE, f2 + ww.ndim * HLLC_EXTRA_PER_FACE
    out_d = {"riemann": riemann, "ms_per_step": el / steps * 1e3, "value": cells * steps / el, "unit": "cell-updates/s",
             "steps": steps, "step_ms": t_step * 1e3, "flags": [int(c) for c in cnt],
             "flops_per_cell_update_stages": [f1, f2],
             "note": "stage kernels k_step3/k_step2 <..., 1|2, 0, flux>, flux 0 Rusanov, 1 HLLC; per-stage durations in the "
                     "kernel-trace summary"}
    del out, sim
    torch.cuda.empty_cache()
    return out_d


def time_conduction(wl, precision, steps, plain_ms, autotune=True):
    """Whole LF cycles with the conduction subcycle along the field (Sec. 3.4;
    Spitzer kappa = kappa0 T^(5/2), kappa0 = 0.4, at most 8 sub-steps) on the
    same blocks and data, captured in a HIP graph; the subcycle's share is the
    cycle time above the plain cycle's, per sub-step."""
    import dataclasses
    import torch
    from paper_1204_5849_amd import native as N
    from paper_1204_5849_amd.sim import Simulation
    ww = dataclasses.replace(wl, cond="field", kappa0=0.4, kappa_exp=2.5, cond_max_sub=8)
    sim = Simulation(ww, precision=precision)
    sim.load_initial()
    if autotune:
        sim.autotune()
    sim.graph_run(2)
    sim.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.graph_run(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    nsub = int(sim.dt[0].cpu().view(torch.int32)[10])
    st, cnt = sim.flags()
    ms = el / steps * 1e3
    out = {"ms_per_step": ms, "value": ww.n_leaf_cells() * steps / el, "unit": "cell-updates/s",
           "steps": steps, "nsub_last_step": nsub, "max_sub": ww.cond_max_sub,
           "kappa0": ww.kappa0, "kappa_exp": ww.kappa_exp, "mode": "field",
           "subcycle_ms_per_substep": (ms - plain_ms) / max(nsub, 1),
           "flags": [int(c) for c in cnt],
           "note": "LF + minmod + Rusanov with the conduction subcycle after every step; "
                   "inactive sub-steps (index >= nsub) exit at once"}
    del sim
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="harris3d")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-regrid", action="store_true")
    ap.add_argument("--no-weno", action="store_true")
    ap.add_argument("--no-cond", action="store_true")
    ap.add_argument("--weno-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--eager", action="store_true", help="eager launches instead of the graph")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other configurations")
    ap.add_argument("--configs-only", default=None, metavar="KEYS",
                    help="only measure these configurations (comma-separated keys of CONFIGS)")
    ap.add_argument("--batched-only", action="store_true",
                    help="with --configs-only: time the batched path alone (for kernel traces)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = args.copy_probe * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": n * 4, "launches": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library holds every "
              "block on one device, and sharding the block list over GPUs is not implemented",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1204_5849_amd.sim import Simulation

    if args.configs_only:
        res = {}
        for key in args.configs_only.split(","):
            log(f"configuration {key}")
            r = measure_config(key, *CONFIGS[key], batched_only=args.batched_only)
            res[r["workload"]] = r
        print(json.dumps({"configs": res}), flush=True)
        return

    wl = build_workload(args.workload, args.precision)
    nleaf_cells = wl.n_leaf_cells()
    log(f"workload {wl.name}: {len(wl.keys)} blocks, {int(wl.leaf_mask().sum())} leaves, "
        f"{nleaf_cells} leaf cells, {args.precision}")
    t0 = time.time()
    sim = Simulation(wl, precision=args.precision)
    sim.load_initial()
    log(f"initial data on device in {time.time() - t0:.1f}s")
    chosen = sim.launch_config()
    if not args.no_autotune:
        chosen = sim.autotune()  # trial steps write the shadow state, not U
        log(f"autotuned launch shapes: {chosen}")
        sim.sync()
    run = sim.advance if args.eager else sim.graph_run
    run(args.warmup)
    sim.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    elapsed = t2 - t1
    ms = elapsed / args.steps * 1e3
    value = nleaf_cells * args.steps / elapsed
    st, cnt = sim.flags()
    log(f"timed {args.steps} steps: {ms:.3f} ms/step, {value / 1e9:.3f} G cell-updates/s, "
        f"flags {st} {cnt}")

    word = 8 if args.precision == "fp64" else 4
    t_step = time_step_kernel(sim, 10)
    bytes_step = step_bytes_per_launch(wl, sim.sizes.nleaves, word)
    achieved = bytes_step / t_step / 1e9
    fpc = FLOPS_PER_CELL[(wl.ndim, wl.eta > 0)]
    tflops = nleaf_cells * fpc / t_step / 1e12
    traffic = measured_traffic(wl.name) if args.precision == "fp32" else None
    valu_busy = measured_valu_busy(wl.name) if args.precision == "fp32" else None
    log(f"step kernel {t_step * 1e3:.3f} ms/launch, {achieved:.1f} GB/s algorithmic, "
        f"{tflops:.2f} TFLOP/s")

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "blocks": int(len(wl.keys)),
                   "leaves": int(sim.sizes.nleaves), "leaf_cells": int(nleaf_cells),
                   "block": "16^%d + 2 ghosts" % wl.ndim, "scheme": wl.scheme,
                   "limiter": wl.limiter, "glm": wl.glm_mode, "eta": wl.eta,
                   "state": args.precision, "launch": launch_label(chosen, args.eager),
                   "launch_config": chosen},
        "roofline": {"bound": "alu", "achieved": tflops, "peak": ALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / ALU_PEAK_TFLOPS, "traffic": traffic,
                     "valu_busy": valu_busy,
                     "kernel": "k_step3 (LF)" if wl.ndim == 3 else "k_step2 (LF)",
                     "kernel_ms": t_step * 1e3,
                     "flops_per_cell_update": fpc, "algorithmic_bytes_per_launch": bytes_step,
                     "hbm_achieved_GBs": achieved, "hbm_peak_GBs": HBM_PEAK_GBS,
                     "hbm_frac": achieved / HBM_PEAK_GBS, "step_share_of_cycle": t_step * 1e3 / ms},
        "hbm_frac_cycle": nleaf_cells * cycle_bytes_per_cell(wl, word) / (ms * 1e-3) / 1e9
        / HBM_PEAK_GBS,
        "hbm_frac_cycle_gather": nleaf_cells * gather_bytes_per_cell(wl, word) / (ms * 1e-3)
        / 1e9 / HBM_PEAK_GBS,
    }
    cb = measured_cycle_bytes(wl.name) if args.precision == "fp32" else None
    result["hbm_frac_cycle_measured"] = (cb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS) if cb else None

    if not args.no_regrid:
        log("one regrid of the timed state (estimate, tree edit, remap)")
        result["regrid"] = time_regrid(sim, wl)
        r = result["regrid"]
        log(f"regrid: {r['blocks_before']} -> {r['blocks_after']} blocks "
            f"(+{r['created']} -{r['destroyed']}); estimate {r['estimate_ms']:.3f} ms, "
            f"tree edit {r['tree_edit_ms']:.1f} ms, remap {r['remap_ms']:.1f} ms")

    del sim
    torch.cuda.empty_cache()
    if not args.no_weno:
        log("WENO + TVD Runge-Kutta 2 on the same workload")
        result["weno"] = time_weno(wl, args.precision, args.weno_steps, not args.no_autotune)
        r = result["weno"]
        log(f"weno: {r['ms_per_step']:.3f} ms/step, {r['value'] / 1e9:.3f} G cell-updates/s, "
            f"map_step {r['step_ms']:.3f} ms")
        log("WENO + TVD Runge-Kutta 2 with the HLLC flux on the same workload")
        result["weno_hllc"] = time_weno(wl, args.precision, args.weno_steps, not args.no_autotune,
                                        riemann="hllc")
        r = result["weno_hllc"]
        log(f"weno+hllc: {r['ms_per_step']:.3f} ms/step, {r['value'] / 1e9:.3f} G cell-updates/s, "
            f"map_step {r['step_ms']:.3f} ms")

    if not args.no_cond:
        log("LF cycles with the conduction subcycle on the same workload")
        result["conduction"] = time_conduction(wl, args.precision, args.weno_steps, ms,
                                               not args.no_autotune)
        r = result["conduction"]
        log(f"conduction: {r['ms_per_step']:.3f} ms/step with {r['nsub_last_step']} sub-steps, "
            f"{r['subcycle_ms_per_substep']:.3f} ms per sub-step")

    if not args.no_plain and args.precision == "fp32":
        log("FP64 batched path on the same workload")
        result["fp64_batched"] = time_fp64_batched(args.workload, args.weno_steps,
                                                   not args.no_autotune)
        r = result["fp64_batched"]
        log(f"fp64 batched: {r['ms_per_step']:.3f} ms/step, {r['value'] / 1e9:.3f} G "
            f"cell-updates/s, step kernel {r['step_kernel_ms']:.3f} ms")

    if not args.no_plain:
        log("FP64 plain per-block path on the same workload")
        from paper_1204_5849_amd import workloads as W  # noqa: F401
        wl64 = build_workload(args.workload, "fp64")
        p = plain_sim(wl64, "fp64")
        p.load_initial()
        p.advance(1)
        p.sync()
        ta = time.perf_counter()
        p.advance(args.plain_steps)
        p.sync()
        tb = time.perf_counter()
        plain_rate = nleaf_cells * args.plain_steps / (tb - ta)
        del p
        torch.cuda.empty_cache()
        result["fp64_plain"] = {"value": plain_rate, "unit": "cell-updates/s",
                                "steps": args.plain_steps, "launch": "one launch per block",
                                "speedup_of_value": value / plain_rate}
        log(f"fp64 plain {plain_rate / 1e9:.3f} G cell-updates/s")

    if not args.no_configs:
        result["configs"] = {}
        for key, spec in CONFIGS.items():
            log(f"configuration {key}: batched {spec[0]} vs plain {spec[1]}")
            r = measure_config(key, *spec)
            result["configs"][r["workload"]] = r
            l1 = r.get("rel_l1_vs_oracle", {})
            log(f"  {r['batched']['value'] / 1e9:.3f} G vs {r['plain']['value'] / 1e9:.4f} G "
                f"cell-updates/s (x{r['speedup_batched_vs_plain']:.0f}); L1 rho "
                f"{l1.get('rho', float('nan')):.2e}")
            rf, oc = r["roofline"], r.get("oracle")
            log(f"  step kernel {rf['kernel_ms']:.3f} ms: HBM {rf['hbm_frac']:.3f}"
                + (f", ALU {rf['alu_frac']:.3f}" if "alu_frac" in rf else "")
                + (f"; oracle {oc['value'] / 1e6:.2f} M/s on {oc['cores']} cores, "
                   f"{oc['one_core']['value'] / 1e6:.2f} M/s on one" if oc else ""))

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) and the FP32 path's L1 against it")
        result["cpu_baseline"], result["l1_fp32_vs_oracle"] = cpu_baseline_and_l1()
        r = result["l1_fp32_vs_oracle"]["rel_l1"]
        log(f"oracle {result['cpu_baseline']['value'] / 1e6:.2f} M cell-updates/s on "
            f"{result['cpu_baseline']['cores']} cores; FP32 rel L1 rho {r['rho']:.2e} "
            f"e {r['e']:.2e} |B| {r['absB']:.2e}")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
