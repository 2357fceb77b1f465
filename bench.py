"""Throughput of the linked-cell rigid-molecule force path on one MI355X.

One "step" is one md_step: leapfrog kick/drift (+ rotation), linked-cell rebuild (wrap, bin,
stable counting sort, sorted gather) and the full force/torque/energy/virial evaluation with its
deterministic reductions -- every stage of the hot path, on one batch of synthetic input already
resident in HBM.

Default workload: homogeneous LJ liquid, N = 1,048,576 (FCC 64^3 start with 0.05 sigma jitter),
rho = 0.75, T = 0.9, r_c = 2.5 (truncated-shifted), cubic periodic box; FP32 pair arithmetic
(FP64 COM test, accumulation and reductions) timed, FP64 path timed beside it.

Prints ONE JSON line.  Extra fields: steps/s, forces-only interactions/s, FP64-path numbers,
FP32 errors against the FP64 path (full system) and against the CPU oracle (sampled rows),
roofline of the pair kernel (timed with HIP events on its launch stream), and the CPU oracle's
rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12  # MI355X FP32 vector, published (packed-FP32 figure)
PEAK_FP64 = 78.6e12   # MI355X FP64 vector, published
PEAK_HBM = 8.0e12
METRIC = "molecule-pair interactions/s + steps/s, FP32 vs FP64 path at stated force error"


def distance_tests(counts3d):
    """Half-stencil distance-test count D = sum_i n_d(i) - N/2 with
    n_d(i) = N_i/2 (N_i + sum over the 26 neighbour cells N_j) (load-cost equation, Sec. 4.2)."""
    c = counts3d.astype(np.float64)
    nb = np.zeros_like(c)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx or dy or dz:
                    nb += np.roll(c, (dz, dy, dx), axis=(0, 1, 2))
    nd = 0.5 * c * (c + nb)
    return float(nd.sum() - 0.5 * c.sum())


def walk_tests(view):
    """Distance tests of the single-site cutoff walk per evaluation, counted from the cell
    occupancy: every molecule against every molecule of its 27 cells (itself included), and with
    half-edge cells (sub_start present) against the five z half-layers around its own z-half in
    each of its nine cell columns (Sec. 3, cells of edge r_c/2)."""
    nx, ny, nz = view["nc"]
    cells = np.diff(view["cell_start"].cpu().numpy().astype(np.int64)).reshape(nz, ny, nx)
    nb = np.zeros_like(cells)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                nb += np.roll(cells, (dz, dy, dx), axis=(0, 1, 2))
    out = {"full_27_cells": float((cells * nb).sum())}
    if view.get("sub_start") is not None:
        octs = np.diff(view["sub_start"].cpu().numpy().astype(np.int64)).reshape(nz, ny, nx, 8)
        half = np.stack([octs[..., 0:4].sum(-1), octs[..., 4:8].sum(-1)], axis=1).reshape(2 * nz, ny, nx)
        col = np.zeros_like(half)
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                col += np.roll(half, (dy, dx), axis=(1, 2))
        win = sum(np.roll(col, -k, axis=0) for k in range(-2, 3))
        out["half_edge_z_culled"] = float((half * win).sum())
        out["ratio"] = out["half_edge_z_culled"] / out["full_27_cells"]
    return out


# Algorithmic FLOP per unordered molecule pair inside the cutoff, counted from the interaction
# formulas as written (Sec. 2 models; FMA = 2, reciprocal / reciprocal square root = 1,
# compare = 0; each pair once).  Site pair terms include the site separation (6), r^2 (5), the
# energy, the force vector on both molecules and the lever-arm torques on both (24); multipole
# pairs add r-hat, the direction cosines, the energy's derivatives and the axis torques.
LJ_ATOM_FLOP = 24          # single-site LJ pair: rcp, s^6, s^12, u, force scalar and vector, F_i F_j, U, W
LJ_SITE_FLOP = 57
ELEC_SITE_FLOP = {("C", "C"): 52, ("C", "D"): 88, ("C", "Q"): 94, ("D", "D"): 149, ("D", "Q"): 160,
                  ("Q", "Q"): 175}
VIRIAL_FLOP = 6            # r_ij . F_ij per molecule pair
DIST_TEST_FLOP = 8         # 3 sub + 1 mul + 2 fma per half-shell distance test


def pair_flops(model):
    """Algorithmic FLOP per interacting molecule pair of a one-component model."""
    sites = model["components"][0]["sites"]
    if len(model["components"]) == 1 and len(sites) == 1 and sites[0]["kind"] == "lj":
        return LJ_ATOM_FLOP
    code = {"charge": "C", "dipole": "D", "quadrupole": "Q"}
    nlj = sum(1 for x in sites if x["kind"] == "lj")
    el = [code[x["kind"]] for x in sites if x["kind"] != "lj"]
    f = nlj * nlj * LJ_SITE_FLOP + VIRIAL_FLOP
    for a in el:
        for b in el:
            f += ELEC_SITE_FLOP[tuple(sorted((a, b)))]
    return f


def pair_counters(kernel_sources, name="k_pair_lj_c2_lj_1m_counters.md"):
    """Per pair-kernel launch, from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source (hash recorded in the summary): HBM bytes and executed FP32 / FP64
    operations (64 lanes x (add + mul + 2 fma + trans) per VALU instruction counted); else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in kernel_sources:
        h.update(open(os.path.join(ROOT, "paper_1408_4599_amd", "csrc", f), "rb").read())
    out, src = {}, None
    for line in open(path).read().splitlines():
        key, _, val = line.partition(":")
        if key == "source_sha256":
            src = val.strip()
        elif key in ("traffic_bytes_per_launch", "executed_fp32_flop_per_launch", "executed_fp64_flop_per_launch"):
            out[key] = float(val.strip())
    return out if src == h.hexdigest() else None


def measure_extra(md, W, torch, name, evals, steps, adjoint=False, half_shell=False, subcells=False):
    """Forces-only and md_step throughput of one more workload (FP32 and FP64); half_shell selects
    the half-shell pair kernel for a single-site model (MD_HALF_SHELL), subcells the half-edge
    cell order and walk (MD_SUBCELLS)."""
    cfg = W.make(name)
    N = cfg["pos"].shape[0]
    dev = lambda a, dt=torch.float64: None if a is None else torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    model = md.Model(cfg["model"], half_shell=half_shell, subcells=subcells)
    cells = md.Cells()
    multi = cfg["quat"] is not None
    md.build_cells(model, cells, dev(cfg["pos"]), dev(cfg["quat"]), None, cfg["box"])
    out = {"N": N, "box": cfg["box"].tolist(), "rc": cfg["model"]["rc"]}
    ref = md.forces(model, cells, "fp64", torque=multi, per_molecule=False)
    torch.cuda.synchronize()
    P = int(ref["npairs"].item())
    out["interacting_pairs"] = P
    v = cells.view()
    D = distance_tests(np.diff(v["cell_start"].cpu().numpy()).reshape(v["nc"][2], v["nc"][1], v["nc"][0]))
    W_alg = DIST_TEST_FLOP * D + pair_flops(cfg["model"]) * P
    out["algorithmic_flop_per_evaluation"] = W_alg
    out["flop_per_pair"] = pair_flops(cfg["model"])
    if model.single_site and not half_shell:
        out["walk_distance_tests"] = walk_tests(v)
        out["half_edge_cells"] = subcells
    for prec in ("fp32", "fp64"):
        buf = {"force": torch.empty((N, 3), dtype=torch.float64, device="cuda"),
               "uw": torch.empty(5, dtype=torch.float64, device="cuda"),
               "npairs": torch.empty(1, dtype=torch.int64, device="cuda")}
        if multi:
            buf["torque"] = torch.empty((N, 3), dtype=torch.float64, device="cuda")
        md.forces_into(model, cells, prec, buf)
        torch.cuda.synchronize()
        model.profile(True)
        t = time.perf_counter()
        for _ in range(evals):
            md.forces_into(model, cells, prec, buf)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / evals
        ms, k = model.profile_read("pair")
        model.profile(False)
        e = {"forces_interactions_per_s": P / wall, "forces_ms": 1e3 * wall, "pair_kernel_ms": ms / k}
        e["roofline_frac"] = W_alg / (ms / k / 1e3) / (PEAK_FP32 if prec == "fp32" else PEAK_FP64)
        if prec == "fp32":
            F32, F64 = buf["force"], ref["force"]
            e["force_rel_rms_vs_fp64"] = float(torch.linalg.norm(F32 - F64) / torch.linalg.norm(F64))
            e["energy_rel_vs_fp64"] = abs(float(buf["uw"][0]) - float(ref["uw"][0])) / abs(float(ref["uw"][0]))
        pos, vel, quat, ang = dev(cfg["pos"]), dev(cfg["vel"]), dev(cfg["quat"]), dev(cfg["angmom"])
        md.step(model, cells, pos, vel, quat, ang, None, cfg["box"], cfg["dt"], 2, prec)
        torch.cuda.synchronize()
        t = time.perf_counter()
        md.step(model, cells, pos, vel, quat, ang, None, cfg["box"], cfg["dt"], steps, prec)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t
        e.update({"steps_per_s": steps / ts, "step_interactions_per_s": P * steps / ts})
        if adjoint:
            # with the parameter gradients (dpos, dquat, dparams), then dpos and dquat only
            md.build_cells(model, cells, dev(cfg["pos"]), dev(cfg["quat"]), None, cfg["box"])
            for params, key in ((True, ""), (False, "_pos_quat_only")):
                md.forces_adjoint(model, cells, prec, 1.0, want_quat=multi, want_params=params)
                torch.cuda.synchronize()
                model.profile(True)
                t = time.perf_counter()
                for _ in range(evals):
                    md.forces_adjoint(model, cells, prec, 1.0, want_quat=multi, want_params=params)
                torch.cuda.synchronize()
                wall = (time.perf_counter() - t) / evals
                ms, k = model.profile_read("adjoint")
                model.profile(False)
                e.update({"adjoint_ms" + key: 1e3 * wall, "adjoint_kernel_ms" + key: ms / k,
                          "adjoint_interactions_per_s" + key: P / wall})
        out[prec] = e
    out["fp32_speedup_forces"] = out["fp64"]["forces_ms"] / out["fp32"]["forces_ms"]
    return out


def start_table_bytes(ncell, subcells):
    """Bytes of the start tables a build writes: one int32 per bin plus the total, and with
    half-edge cells (8 bins per cell) also the cell starts."""
    return 4.0 * (8 * ncell + 1) + 4.0 * (ncell + 1) if subcells else 4.0 * (ncell + 1)


def build_sweep(md, W, torch, nbuild=10, subcells=True):
    """Cell build (wrap, bin, stable counting sort, sorted gather) of homogeneous LJ fluids from 2^14
    to 2^26 molecules: rebuilds of the same configuration (as in md_step), timed with HIP events;
    algorithmic bytes 56 per molecule + the start tables (single-site)."""
    model = md.Model(W.lj_model(2.5), subcells=subcells)
    rows = []
    for n in (16, 32, 64, 128, 256):
        pos, box = W.fcc_positions_device(n, 0.75, 14084599 + n, "cuda")
        N = pos.shape[0]
        cells = md.Cells()
        for _ in range(2):
            md.build_cells(model, cells, pos, None, None, box)
        torch.cuda.synchronize()
        model.profile(True)
        for _ in range(nbuild):
            md.build_cells(model, cells, pos, None, None, box)
        ms, k = model.profile_read("build")
        model.profile(False)
        v = cells.view()
        ncell = int(np.prod(v["nc"]))
        s = ms / k / 1e3
        byts = 56.0 * N + start_table_bytes(ncell, subcells)
        rows.append({"N": N, "log2N": round(math.log2(N), 3), "cells": ncell, "ms_per_build": 1e3 * s,
                     "algorithmic_bytes": byts, "GB_per_s": byts / s / 1e9, "frac_of_hbm_peak": byts / s / PEAK_HBM})
        print(f"[bench] build N={N}: {1e3 * s:.4f} ms, {byts / s / 1e9:.0f} GB/s", file=sys.stderr, flush=True)
        cells.close()
        del pos
        torch.cuda.empty_cache()
    print(json.dumps({"build_sweep": rows, "peak_hbm_GB_per_s": PEAK_HBM / 1e9, "half_edge_cells": subcells,
                      "accounting": "56 B per molecule (COM read 24, cell id 4, permutation 4, sorted COM "
                                    "24) + 4 B per start-table entry (8 half-cells + 1 cell entry per cell "
                                    "with half-edge cells)"}), flush=True)


def step_sweep(md, W, torch):
    """md_step throughput of homogeneous LJTS fluids (rho = 0.75, T = 0.9, r_c = 2.5, the C2
    configuration) from 16 384 to 8 388 608 molecules on one GPU: FP32 path, half-edge cells, an
    energies row every step, as in the benchmark's timed steps.  The GPU is first kept busy for
    about 0.3 s (its first steps in a process run a few per cent slower); each size then takes 10
    untimed steps and 50 to 500 timed ones."""
    model = md.Model(W.lj_model(2.5, shift=True), subcells=True)
    pos, box = W.fcc_positions_device(64, 0.75, 24084599, "cuda")
    vel = torch.zeros_like(pos)
    cells = md.Cells()
    md.step(model, cells, pos, vel, None, None, None, box, 0.002, 700, "fp32")
    torch.cuda.synchronize()
    cells.close()
    del pos, vel
    rows = []
    for n in (16, 24, 32, 48, 64, 96, 128):
        pos, box = W.fcc_positions_device(n, 0.75, 24084599 + n, "cuda")
        N = pos.shape[0]
        g = torch.Generator(device="cuda")
        g.manual_seed(n)
        vel = torch.randn((N, 3), generator=g, device="cuda", dtype=torch.float64) * math.sqrt(0.9)
        vel -= vel.mean(dim=0)
        cells = md.Cells()
        md.build_cells(model, cells, pos, None, None, box)
        P = int(md.forces(model, cells, "fp32", torque=False, per_molecule=False)["npairs"].item())
        nsteps = max(50, min(500, int(1e8 / N)))
        en = torch.empty((nsteps, 4), dtype=torch.float64, device="cuda")
        md.step(model, cells, pos, vel, None, None, None, box, 0.002, 10, "fp32", en)
        torch.cuda.synchronize()
        t = time.perf_counter()
        md.step(model, cells, pos, vel, None, None, None, box, 0.002, nsteps, "fp32", en)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / nsteps
        rows.append({"N": N, "cells": int(np.prod(cells.view()["nc"])), "interacting_pairs": P, "steps": nsteps,
                     "ms_per_step": 1e3 * dt, "interactions_per_s": P / dt, "molecule_steps_per_s": N / dt})
        print(f"[bench] step N={N}: {1e3 * dt:.4f} ms, {P / dt:.3e} interactions/s", file=sys.stderr, flush=True)
        cells.close()
        del pos, vel, en
        torch.cuda.empty_cache()
    print(json.dumps({"step_sweep": rows, "precision": "fp32", "half_edge_cells": True,
                      "note": "LJTS rho = 0.75, T = 0.9, r_c = 2.5, dt = 0.002; md_step with cell rebuild, "
                              "forces, leapfrog and an energies row every step; rates from the wall time"}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--force-evals", type=int, default=100)
    ap.add_argument("--workload", default="c2_lj_1m")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle rows timed (0: auto)")
    ap.add_argument("--quick", action="store_true", help="short run for profilers: few steps, no extras")
    ap.add_argument("--step-sweep", action="store_true", help="md_step throughput from 2^14 to 2^23 molecules")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="also run 3 plain device copies of this many MiB (HBM byte-counter calibration)")
    ap.add_argument("--no-extra", action="store_true", help="skip the other workloads")
    ap.add_argument("--no-subcells", action="store_true",
                    help="single-site models: plain cell order and 27-cell walk instead of half-edge cells")
    ap.add_argument("--build-sweep", action="store_true",
                    help="only time the cell build of homogeneous LJ fluids (rho = 0.75, r_c = 2.5) for "
                         "N = 2^14, 2^17, 2^20, 2^23, 2^26 and print one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    if args.quick:
        args.steps, args.warmup, args.force_evals = min(args.steps, 5), min(args.warmup, 2), 5
        args.no_fp64 = args.no_cpu_baseline = args.no_extra = True

    import torch
    from paper_1408_4599_amd import md, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.build_sweep:
        build_sweep(md, W, torch, subcells=not args.no_subcells)
        return
    if args.step_sweep:
        step_sweep(md, W, torch)
        return
    t0 = time.time()
    cfg = W.make(args.workload)
    gen_s = time.time() - t0
    N = cfg["pos"].shape[0]
    dev = lambda a, dt=torch.float64: None if a is None else torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    multi = cfg["quat"] is not None
    ncomp = len(cfg["model"]["components"])
    comp_t = dev(cfg["comp"], torch.int32) if ncomp > 1 else None
    single = cfg["quat"] is None and ncomp == 1
    subcells = single and not args.no_subcells
    model = md.Model(cfg["model"], subcells=subcells)
    cells = md.Cells()
    print(f"[bench] workload {args.workload}: N={N}, box={cfg['box'].tolist()}, generated in {gen_s:.1f}s", file=sys.stderr, flush=True)

    if args.copy_calib:
        a = torch.ones(args.copy_calib * 262144, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # ---- one reference evaluation of the start configuration (both precisions) ----
    pos0 = dev(cfg["pos"])
    quat0 = dev(cfg["quat"])
    md.build_cells(model, cells, pos0, quat0, comp_t, cfg["box"])
    r64 = md.forces(model, cells, "fp64", torque=multi, per_molecule=False)
    r32 = md.forces(model, cells, "fp32", torque=multi, per_molecule=False)
    torch.cuda.synchronize()
    P = int(r64["npairs"].item())
    assert P == int(r32["npairs"].item())
    v = cells.view()
    counts = np.diff(v["cell_start"].cpu().numpy()).reshape(v["nc"][2], v["nc"][1], v["nc"][0])
    D = distance_tests(counts)
    F64, F32 = r64["force"].double(), r32["force"].double()
    eF = float(torch.linalg.norm(F32 - F64) / torch.linalg.norm(F64))
    U64, U32 = float(r64["uw"][0]), float(r32["uw"][0])
    eU = abs(U32 - U64) / abs(U64)
    errors = {"fp32_vs_fp64_gpu": {"force_rel_rms": eF, "energy_rel": eU,
                                   "virial_rel": abs(float(r32["uw"][1]) - float(r64["uw"][1])) / abs(float(r64["uw"][1]))}}
    if multi:
        T64, T32 = r64["torque"], r32["torque"]
        errors["fp32_vs_fp64_gpu"]["torque_rel_rms"] = float(torch.linalg.norm(T32 - T64) / torch.linalg.norm(T64))
    print(f"[bench] P={P} D={D:.4g} eps_F={eF:.2e} eps_U={eU:.2e}", file=sys.stderr, flush=True)

    # ---- forces-only timing: pair kernel with HIP events on its stream ----
    def time_forces(prec, n):
        out = {"force": torch.empty((N, 3), dtype=torch.float64, device="cuda"),
               "uw": torch.empty(5, dtype=torch.float64, device="cuda"),
               "npairs": torch.empty(1, dtype=torch.int64, device="cuda")}
        if multi:
            out["torque"] = torch.empty((N, 3), dtype=torch.float64, device="cuda")
        for _ in range(3):
            md.forces_into(model, cells, prec, out)
        torch.cuda.synchronize()
        model.profile(True)
        t = time.perf_counter()
        for _ in range(n):
            md.forces_into(model, cells, prec, out)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / n
        ms, k = model.profile_read("pair")
        model.profile(False)
        return wall, ms / k / 1e3

    # ---- cell build (wrap, bin, stable counting sort, sorted gather), HBM-bound ----
    def time_builds(n):
        for _ in range(2):
            md.build_cells(model, cells, pos0, quat0, comp_t, cfg["box"])
        torch.cuda.synchronize()
        model.profile(True)
        for _ in range(n):
            md.build_cells(model, cells, pos0, quat0, comp_t, cfg["box"])
        torch.cuda.synchronize()
        ms, k = model.profile_read("build")
        model.profile(False)
        return ms / k / 1e3

    build_s = time_builds(max(5, args.force_evals // 5))
    ncell_total = int(np.prod(v["nc"]))
    # algorithmic bytes: read the COM (24 B); write cell id (4 B), permutation (4 B) and the sorted
    # FP64 COM copy (24 B) per molecule, the cell start table (4 B per cell); multi-site models add
    # the quaternion (32 B) and component id (4 B) read and the component id (4 B) and world-frame
    # site vectors (24 B each) written
    build_bytes_mol = 56.0
    if multi:
        kinds = [[st["kind"] for st in c_["sites"]] for c_ in cfg["model"]["components"]]
        nv = sum(max(k.count(kind) for k in kinds) * w for kind, w in
                 (("lj", 1), ("charge", 1), ("dipole", 2), ("quadrupole", 2)))
        build_bytes_mol += 40.0 + 24.0 * nv
    build_bytes = build_bytes_mol * N + start_table_bytes(ncell_total, subcells)

    f32_wall, f32_pair = time_forces("fp32", args.force_evals)
    f64_wall, f64_pair = (None, None) if args.no_fp64 else time_forces("fp64", args.force_evals)

    # ---- the same evaluation with plain cells (27-cell walk), for the half-edge cells' gain ----
    plain = None
    if subcells and not args.quick:
        pm, pc = md.Model(cfg["model"]), md.Cells()
        md.build_cells(pm, pc, pos0, quat0, comp_t, cfg["box"])
        buf = {"force": torch.empty((N, 3), dtype=torch.float64, device="cuda"),
               "uw": torch.empty(5, dtype=torch.float64, device="cuda"),
               "npairs": torch.empty(1, dtype=torch.int64, device="cuda")}
        plain = {}
        for prec in ("fp32", "fp64"):
            for _ in range(3):
                md.forces_into(pm, pc, prec, buf)
            torch.cuda.synchronize()
            pm.profile(True)
            for _ in range(args.force_evals):
                md.forces_into(pm, pc, prec, buf)
            torch.cuda.synchronize()
            ms, k = pm.profile_read("pair")
            pm.profile(False)
            plain[prec + "_pair_kernel_ms"] = ms / k
        pm.profile(True)
        for _ in range(max(5, args.force_evals // 5)):
            md.build_cells(pm, pc, pos0, quat0, comp_t, cfg["box"])
        torch.cuda.synchronize()
        ms, k = pm.profile_read("build")
        pm.profile(False)
        plain["ms_per_build"] = ms / k
        plain["walk_distance_tests"] = walk_tests(pc.view())["full_27_cells"]
        pc.close()
        pm.close()

    # ---- full steps ----
    def run_steps(prec, nsteps=None):
        nsteps = args.steps if nsteps is None else nsteps
        pos = dev(cfg["pos"])
        vel = dev(cfg["vel"])
        quat = dev(cfg["quat"])
        ang = dev(cfg["angmom"])
        en = torch.empty((max(nsteps, args.warmup, 1), 4), dtype=torch.float64, device="cuda")
        if args.warmup:
            md.step(model, cells, pos, vel, quat, ang, comp_t, cfg["box"], cfg["dt"], args.warmup, prec, en)
        torch.cuda.synchronize()
        t = time.perf_counter()
        md.step(model, cells, pos, vel, quat, ang, comp_t, cfg["box"], cfg["dt"], nsteps, prec, en)
        torch.cuda.synchronize()
        dt_ = time.perf_counter() - t
        e = en[:nsteps].cpu().numpy()
        return dt_, e

    t32, e32 = run_steps("fp32")
    print(f"[bench] fp32 steps: {args.steps} in {t32:.3f}s", file=sys.stderr, flush=True)
    t64 = e64 = None
    if not args.no_fp64:
        t64, e64 = run_steps("fp64")
        print(f"[bench] fp64 steps: {args.steps} in {t64:.3f}s", file=sys.stderr, flush=True)

    # NVT: the same steps with velocity rescaling to the workload temperature (extra kernel and
    # the kinetic reduction every step)
    n_nvt = max(1, args.steps // 4)
    model.set_thermostat(cfg["T"])
    tnvt, envt = run_steps("fp32", n_nvt)
    model.set_thermostat(0.0)
    f_dof = 3 * N + (0 if cfg["quat"] is None else
                     sum(int(np.sum(np.asarray(cfg["model"]["components"][c]["inertia"]) > 0))
                         for c in (np.zeros(N, dtype=np.int64) if cfg["comp"] is None else cfg["comp"])))
    print(f"[bench] fp32 NVT steps: {n_nvt} in {tnvt:.3f}s", file=sys.stderr, flush=True)

    ms_per_step = 1e3 * t32 / args.steps
    value = P * args.steps / t32
    E = e32[:, 0] + e32[:, 1] + e32[:, 2]
    W_alg = DIST_TEST_FLOP * D + pair_flops(cfg["model"]) * P
    counters = pair_counters(["md_pair.hip", "md_device.h", "md_internal.h"]) if model.single_site else None
    traffic = counters.get("traffic_bytes_per_launch") if counters else None
    ex32 = counters.get("executed_fp32_flop_per_launch") if counters else None
    ex64 = counters.get("executed_fp64_flop_per_launch") if counters else None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": N, "box": cfg["box"].tolist(), "rc": cfg["model"]["rc"],
                   "lj_shift": cfg["model"]["lj_shift"], "dt": cfg["dt"], "T": cfg["T"],
                   "cells": list(v["nc"]), "interacting_pairs": P, "distance_tests_half_shell": D,
                   "half_edge_cells": subcells,
                   "walk_distance_tests": walk_tests(v) if model.single_site else None,
                   "note": "interactions/s = unique COM-cutoff pairs x steps / wall time of md_step (cell rebuild, "
                           "forces and leapfrog every step); FP32 cutoff test with guard band and FP32 force "
                           "algebra, FP64 pair decisions, energies and sums; single-site models with the "
                           "half-edge (r_c/2) cell order and z-culled walk"},
        "steps_per_s": args.steps / t32,
        "forces_only": {"fp32_interactions_per_s": P / f32_wall, "fp32_ms": 1e3 * f32_wall,
                        "fp32_pair_kernel_ms": 1e3 * f32_pair},
        "errors": errors,
        "nve_rel_energy_spread_fp32": float(np.abs(E - E[0]).max() / abs(E[0])),
        "nvt_fp32": {"steps": n_nvt, "steps_per_s": n_nvt / tnvt, "ms_per_step": 1e3 * tnvt / n_nvt,
                     "T_target": cfg["T"], "T_kin_last_step": float(2.0 * (envt[-1, 1] + envt[-1, 2]) / f_dof)},
        "roofline": {"bound": "alu", "achieved": W_alg / f32_pair / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": W_alg / f32_pair / PEAK_FP32,
                     "traffic": traffic,
                     # the last template argument (waves per SIMD: 4, or 5 where the LDS of a block
                     # leaves room for 5 blocks per CU) is chosen at launch; C2 takes 4
                     "kernel": ("k_pair_lj<float, true, 4|5>" if subcells else "k_pair_lj<float, false, 4|5>")
                               if model.single_site else "k_pair_ms<float>",
                     "algorithmic_flop_per_launch": W_alg,
                     "accounting": f"{DIST_TEST_FLOP} FLOP per half-shell distance test (D) + "
                                   f"{pair_flops(cfg['model'])} FLOP per unique interacting pair (P)",
                     "frac_of_nonpacked_fp32_issue": W_alg / f32_pair / (PEAK_FP32 / 2),
                     # executed operations from the committed counter summary (None once the kernel
                     # source has changed since it was taken), each precision against its own peak
                     "executed_fp32_flop_per_launch": ex32,
                     "executed_fp32_frac": None if ex32 is None else ex32 / f32_pair / PEAK_FP32,
                     "executed_fp64_flop_per_launch": ex64,
                     "executed_fp64_frac": None if ex64 is None else ex64 / f32_pair / PEAK_FP64},
        "plain_cells": None if plain is None else {
            **plain, "fp32_pair_kernel_ms_half_edge": 1e3 * f32_pair,
            "fp64_pair_kernel_ms_half_edge": None if f64_pair is None else 1e3 * f64_pair,
            "ms_per_build_half_edge": 1e3 * build_s,
            "note": "the same configuration with plain cells (MD_SUBCELLS off): pair kernel (HIP events), "
                    "build and the 27-cell walk's distance tests, beside the half-edge figures"},
        "cell_sort_roofline": {"bound": "hbm", "achieved": build_bytes / build_s / 1e9, "peak": PEAK_HBM / 1e9,
                               "unit": "GB/s", "frac": build_bytes / build_s / PEAK_HBM,
                               "ms_per_build": 1e3 * build_s, "algorithmic_bytes_per_build": build_bytes,
                               "accounting": f"{build_bytes_mol:.0f} B per molecule + 4 B per start-table entry "
                                             f"({'8 half-cells + 1 cell' if subcells else '1'} per cell)",
                               "kernels": "k_bin, k_scan_local, k_scan_top, k_scatter, k_rank_gather"},
    }
    if not args.no_fp64:
        out["fp64"] = {"interactions_per_s": P * args.steps / t64, "ms_per_step": 1e3 * t64 / args.steps,
                       "steps_per_s": args.steps / t64, "forces_only_interactions_per_s": P / f64_wall,
                       "pair_kernel_ms": 1e3 * f64_pair,
                       "roofline_frac_fp64_peak": W_alg / f64_pair / PEAK_FP64}
        out["fp32_speedup_over_fp64"] = {"step": t64 / t32, "pair_kernel": f64_pair / f32_pair}

    # the paper's own figures (CPU runs of single-site LJ / LJTS, Sec. 5): context, not a target
    out["paper_context"] = {
        "this_run_molecule_steps_per_s": N * args.steps / t32,
        "paper_sequential": {"molecule_steps_per_s": 102400 * 1000 / 530.9,
                             "hardware": "1 core, AMD Opteron 6276 @ 2.3 GHz",
                             "workload": "LJTS planar interface, N = 102 400, r_c = 2.5, 1000 steps in 530.9 s"},
        "paper_full_machine": {"molecule_steps_per_s": 4.125e12 / 40.0,
                               "hardware": "SuperMUC, 147 456 Sandy Bridge cores, FP32 AVX128",
                               "workload": "single-site LJ, 4.125e12 molecules, r_c = 3.5, about 40 s per step"},
    }

    if not args.no_extra:
        extra = {}
        for key, name, ev, st, adj, hs, sc in (
                ("c3_lj_slab_2m", "c3_lj_slab_2m", 20, 20, False, False, not args.no_subcells),
                ("c3_lj_slab_2m_half_shell", "c3_lj_slab_2m", 20, 20, False, True, False),
                ("c4_2cljq_500k", "c4_2cljq_500k", 10, 10, False, False, False),
                ("c5_4site_200k", "c5_4site_200k", 10, 10, True, False, False)):
            print(f"[bench] extra workload {key}", file=sys.stderr, flush=True)
            extra[key] = measure_extra(md, W, torch, name, ev, st, adj, hs, sc)
        out["workloads"] = extra

    # ---- oracle rows: FP32 errors on a sample and the CPU baseline ----
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        rng = np.random.default_rng(7)
        ns = args.cpu_sample or max(64, int(2.0e10 / N))
        idx = np.sort(rng.choice(N, size=min(ns, N), replace=False))
        t = time.perf_counter()
        ref = O.rows(cfg["model"], cfg["pos"], cfg["quat"], cfg["comp"], cfg["box"], idx)
        tcpu = time.perf_counter() - t
        F32s = F32.cpu().numpy()[idx]
        errors["fp32_vs_oracle_rows"] = {
            "rows": int(len(idx)),
            "force_rel_rms": float(np.linalg.norm(F32s - ref["F"]) / np.linalg.norm(ref["F"])),
            "fp64_force_rel_rms": float(np.linalg.norm(F64.cpu().numpy()[idx] - ref["F"]) / np.linalg.norm(ref["F"]))}
        t_full = tcpu * N / len(idx)
        cpu_model = None
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        out["cpu_baseline"] = {"value": P / t_full, "unit": "interactions/s", "cores": O.num_threads(),
                               "cpu_model": cpu_model, "kind": "oracle",
                               "sample": f"{len(idx)} of {N} molecules: full O(N) rows of the FP64 brute-force "
                                         f"oracle in {tcpu:.1f}s; rate scaled to all N rows (each pair visited "
                                         f"from both ends)"}
        # the oracle timing protocol on these cores: the small LJTS fluid (N = 4000) evaluated in full
        # and integrated for 100 steps; the full-size evaluations as recorded with the stored values
        c1 = W.make("c1_ljts_4000")
        t = time.perf_counter()
        r1 = O.forces(c1["model"], c1["pos"], c1["quat"], c1["comp"], c1["box"])
        t_c1 = time.perf_counter() - t
        t = time.perf_counter()
        O.step(c1["model"], c1["pos"], c1["vel"], c1["quat"], c1["angmom"], c1["comp"], c1["box"], c1["dt"], 100)
        t_c1s = time.perf_counter() - t
        n1 = c1["pos"].shape[0]
        golden_path = os.path.join(ROOT, "tests", "golden", "full_size.json")
        full = json.load(open(golden_path)) if os.path.exists(golden_path) else {}
        out["oracle_protocol"] = {
            "cores": O.num_threads(), "cpu_model": cpu_model,
            "c1_ljts_4000": {"full_evaluation_s": t_c1, "pair_tests_per_s": n1 * (n1 - 1) / 2 / t_c1,
                             "interactions_per_s": r1["npairs"] / t_c1, "steps": 100, "steps_s": t_c1s,
                             "steps_per_s": 100 / t_c1s},
            "full_size_evaluations": {k: {"seconds": v["oracle_seconds"], "threads": v["threads"],
                                          "interactions_per_s": v["npairs"] / v["oracle_seconds"],
                                          "pair_tests_per_s": v["N"] * (v["N"] - 1) / 2 / v["oracle_seconds"]}
                                      for k, v in full.items()},
            "note": "full-size evaluations: the brute-force oracle over all N^2 pairs, timed when the stored "
                    "energies were written (tests/golden/make_full_size.py, in the build container, threads "
                    "as stated); the C1 figures are measured here, on the cores above"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
