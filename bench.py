#!/usr/bin/env python3
"""Benchmark: SIPG assembly throughput on one MI355X.

Workload: 2D diffusion-advection-reaction, 16,384-cell seeded Voronoi mesh of
the unit square, p = 2 (6 dofs per cell), a = 1 + 0.5 sin(2 pi x) cos(2 pi y),
b = (1, 0.5), c = 1, upwinded advection faces; contraction and output in FP32,
geometry, weights and penalty in FP64.

One step = the whole path on the device: block sparsity pattern, geometry,
assembly of every block row and the right-hand side (one asynchronous dgp_run,
issued back to back; the same step replayed from a captured HIP graph is
reported beside it).  The mesh is resident in HBM before the timed region.
Prints one JSON line.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


# the headline kernel's sources, and the runtime, which builds the row orders
# of its launch configurations (the committed counters hold for these only)
KERNEL_SOURCES = ["assemble_f32.hip", "row_f32.h", "row_common.h", "asm_common.h", "dgp_common.h", "rules_data.h", "wave.h",
                  "runtime.hip", "ctx.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_row2d_f32_p2_voronoi16384.json")


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2007_04881_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _traffic_entry(cfg):
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_digest():
        return None
    return t.get("by_config", {}).get(str(cfg))


# vector issue rate: 1,024 SIMDs x 2.4 GHz, one wave64 VALU instruction per 4 cycles
VALU_ISSUE_PER_S = 1024 * 2.4e9 / 4


def valu_issue(cfg, kernel_ms):
    """The assembly kernel's VALU instructions per launch (SQ_INSTS_VALU of the
    committed counter run, same sources and launch configuration) against the
    chip's vector issue rate over the measured launch time; None if the sources
    changed."""
    v = _traffic_entry(cfg)
    if not v or "valu_insts" not in v:
        return None
    issue_ms = v["valu_insts"] / VALU_ISSUE_PER_S * 1e3
    return {"valu_insts_per_launch": v["valu_insts"], "issue_ms": issue_ms, "frac": issue_ms / kernel_ms}


def measured_traffic(cfg):
    """HBM bytes per launch of the assembly kernel in launch configuration cfg
    from the committed counter runs (FETCH_SIZE + WRITE_SIZE, scaled by a copy
    kernel of known size), or None if the kernel sources changed since they
    were taken."""
    v = _traffic_entry(cfg)
    return v.get("bytes_per_launch") if v else None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(mesh, info, val_bytes, with_pattern=False):
    """Bytes the 2D assembly kernel must move at least once in the launch that is
    timed (values only: the timing re-launch leaves the pattern arrays alone):
    mesh connectivity and coordinates, the per-cell geometry records, and the
    values and right-hand side it writes; with_pattern adds the pattern arrays
    a pattern-writing launch stores."""
    V, N, F = mesh.n_vertices, mesh.n_cells, mesh.n_faces
    nv = int(mesh.cell_ptr[-1])
    reads = 16 * V + 8 * (N + 1) + 4 * nv + 4 * nv + 8 * F + F + 64 * N
    writes = val_bytes * (info.n_vals + info.n_dofs)
    if with_pattern:
        writes += 8 * (N + 1) + 4 * info.nnzb + 8 * (info.nnzb + 1) + 8 * (N + 1)
    return reads + writes


def algorithmic_bytes_3d(mesh, info, val_bytes):
    """The same for polyhedra: tetrahedron ids, vertex coordinates, face arrays
    (vertices, cells, code, opposite vertex), cell-face lists, values and load."""
    V, N, F = mesh.n_vertices, mesh.n_cells, mesh.n_faces
    nt = int(mesh.cell_ptr[-1]) // 4
    ncf = int(mesh.cell_face_ptr[-1])
    reads = 24 * V + 16 * nt + 8 * (N + 1) * 2 + (12 + 8 + 1 + 4) * F + 4 * ncf + 144 * N
    return reads + val_bytes * (info.n_vals + info.n_dofs)


def flops_3d(mesh, info, nb=10, q_tet=11, q_tri=6):
    """Algorithmic FLOPs of one 3D assembly: the contraction Phi^T diag(w) Phi of
    every element and face block counted once, 2 K n_b n_b' per block, K = 3 Q
    (diffusion, d = 3) for the element block, K = 2 q per face block (two
    self and two cross blocks per interior face, one self block per boundary face)."""
    nt = int(mesh.cell_ptr[-1]) // 4
    interior = int((mesh.face_cell[1::2] >= 0).sum())
    boundary = mesh.n_faces - interior
    vol = 2 * (3 * q_tet * nt) * nb * nb
    face = (4 * interior + boundary) * 2 * (2 * q_tri) * nb * nb
    return vol + face


def roofline_hbm(abytes, kernel_ms, kernel, traffic=None):
    achieved = abytes / (kernel_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel, "algorithmic_bytes": abytes}


def hbm_copy_gbs(torch, mib=1024):
    """Device-to-device copy of a mib-MiB buffer (read + write), the achievable HBM rate."""
    x = torch.empty(mib * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        y.copy_(x)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / 10
    return 2 * x.numel() * 4 / (ms * 1e-3) / 1e9


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_rate(mesh, prob, parallel, budget_s):
    """Median over passes (pattern + full assembly) of the oracle on the mesh."""
    import oracle
    times, nnzb = [], 0
    t_total = 0.0
    while (t_total < budget_s or len(times) < 5) and len(times) < 200:
        t0 = time.perf_counter()
        pat = oracle.pattern(mesh)
        oracle.assemble(mesh, prob, pat=pat, parallel=parallel)
        dt = time.perf_counter() - t0
        times.append(dt)
        t_total += dt
        nnzb = pat.nnzb
    med = sorted(times)[len(times) // 2]
    return nnzb / med, mesh.n_cells / med, len(times), t_total


def cpu_baseline(mesh, params, budget_s=8.0):
    """The oracle as it stands (FP64 C) on the same mesh, pattern + full assembly,
    median of the passes that fit in about budget_s seconds each: the OpenMP
    build with rows over all the threads OpenMP is given (the headline figure),
    and the single-threaded canonical build."""
    import oracle
    prob = oracle.Problem.from_params(params)
    v_par, e_par, n_par, t_par = _oracle_rate(mesh, prob, True, budget_s)
    v_one, e_one, n_one, t_one = _oracle_rate(mesh, prob, False, budget_s)
    cores = oracle.threads(parallel=True)
    return dict(value=v_par, unit="block-nnz/s", cores=cores, kind="oracle",
                sample=f"median of {n_par} full passes (pattern + assembly) over the same 16,384-cell mesh, "
                       f"{t_par:.1f} s, OpenMP over rows on {cores} threads",
                elements_per_s=e_par, nproc=os.cpu_count(), cpu_model=_cpu_model(),
                single_thread={"value": v_one, "elements_per_s": e_one, "cores": 1,
                               "sample": f"median of {n_one} passes, {t_one:.1f} s"})


TRAIN_SEED = 2007048815  # key of the training polygon stream


def _replay_ms(ctx, D, torch, steps, warmup):
    for _ in range(warmup):
        ctx.graph_launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.graph_launch()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def reduced_rule_study(D, torch, steps, warmup, train_polygons, train_epochs):
    """Reduced volume rules on the 262,144-cell Voronoi mesh at p = 3 (Poisson):
    network training, rule construction from the network and from the untrained
    4 x 4 Gauss template, and the assembly with plain and with reduced rules."""
    from meshgen import config_mesh, problem_params
    log("reduced rules: 262,144-cell mesh")
    mesh = config_mesh(5)
    params = problem_params(5)
    ctx = D.Context(0)
    ctx.upload(mesh)
    info = ctx.pattern()
    log(f"training on {train_polygons} polygons, {train_epochs} epochs")
    t0 = time.perf_counter()
    _, losses, tst = ctx.mlp_train(train_polygons, TRAIN_SEED, init_seed=1, epochs=train_epochs, batch=4096,
                                   lr=2e-3)
    train_s = time.perf_counter() - t0

    def build(init):
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = ctx.qrule_build(init, 8, 1e-10)
        ms = (time.perf_counter() - t) * 1e3
        n_acc = max(st.n_accepted, 1)
        mean_it = sum(k * st.iters_hist[k] for k in range(16)) / n_acc
        return dict(wall_ms=ms, features_ms=st.ms_features, network_ms=st.ms_network, refine_ms=st.ms_refine,
                    eligible=st.n_eligible, accepted=st.n_accepted, accepted_frac=st.n_accepted / max(st.n_eligible, 1),
                    mean_steps=mean_it, steps_hist=list(st.iters_hist), max_residual=st.max_residual_accepted)

    log(f"trained in {time.perf_counter() - t0:.1f} s; building rules")
    tmpl = build(D.INIT_TEMPLATE)
    net = build(D.INIT_NETWORK)
    log("timing plain and reduced assembly")
    vals, rhs = ctx.outputs(D.F32)
    t = {}
    kern = {}
    for mode, name in ((D.RULE_PLAIN, "plain"), (D.RULE_REDUCED, "reduced")):
        ctx.graph_capture(1, params, D.F32, vals, rhs, rule_mode=mode)
        t[name] = _replay_ms(ctx, D, torch, steps, warmup)
        ctx.assemble(params, D.F32, vals, rhs, rule_mode=mode)
        kern[name] = ctx.time_kernels(10)[1]
    gain = kern["plain"] - kern["reduced"]
    rulegen = net["features_ms"] + net["network_ms"] + net["refine_ms"]
    ctx.close()
    return {"workload": "262144-cell seeded Voronoi, p=3, Poisson, FP32 assembly",
            "cells": mesh.n_cells, "nnzb": info.nnzb,
            "training": {"polygons": train_polygons, "epochs": train_epochs, "steps": tst.steps, "seconds": train_s,
                         "loss_first_epoch": float(losses[0]), "loss_last_epoch": float(losses[-1])},
            "rules_network_init": net, "rules_template_init": tmpl,
            "assemble_ms": t, "assemble_kernel_ms": kern,
            "roofline_plain": roofline_hbm(algorithmic_bytes(mesh, info, 4), kern["plain"],
                                           "k_row2d<float,3,3,false,false,*>"),
            "kernel_speedup": kern["plain"] / kern["reduced"],
            "rulegen_ms": rulegen,
            "break_even_assemblies": (rulegen / gain) if gain > 0 else None}


def mixed_degree_study(D, torch, steps, warmup):
    """262,144-cell Voronoi mesh with degrees drawn from {1, 2, 3, 4} (Poisson):
    whole-path graph replays and per-launch kernel times, FP32 and FP64."""
    from meshgen import config_mesh, problem_params
    log("mixed degrees: 262,144-cell mesh, p in 1..4")
    mesh = config_mesh(3)
    params = problem_params(3)
    ctx = D.Context(0)
    ctx.upload(mesh)
    info = ctx.pattern()
    out = {"workload": "2D Poisson, 262144-cell seeded Voronoi, p drawn from {1,2,3,4}",
           "cells": mesh.n_cells, "nnzb": info.nnzb, "n_vals": info.n_vals, "n_dofs": info.n_dofs}
    for prec, name in ((D.F32, "f32"), (D.F64, "f64")):
        vals, rhs = ctx.outputs(prec)
        ctx.graph_capture(0, params, prec, vals, rhs)
        ms = _replay_ms(ctx, D, torch, steps, warmup)
        ctx.run(params, prec, vals, rhs)
        prep_ms, asm_ms = ctx.time_kernels(10)
        # per-degree register budgets tuned on this workload, then timed again
        choice = ctx.autotune(400)
        ctx.graph_capture(0, params, prec, vals, rhs)
        ms_t = _replay_ms(ctx, D, torch, steps, warmup)
        ctx.run(params, prec, vals, rhs)
        asm_t = ctx.time_kernels(10)[1]
        vb = 4 if prec == D.F32 else 8
        tname = "float" if prec == D.F32 else "double"
        row = choice[1 if prec == D.F32 else 0]
        fused = bool(row[0])
        per_degree = (f"k_row2d_f32<p,false,*,true> (p = 1, 2) + k_row2d<float,p,4,true,false,*> (p = 3, 4)"
                      if prec == D.F32 else "k_row2d<double,p,4,true,false,*>")
        kname = (f"k_row2d_fused<{tname},false> (one persistent launch over every bin)" if fused else
                 f"{per_degree} (one launch per degree, summed)")
        out[name] = {"ms_per_step": ms, "block_nnz_per_s": info.nnzb / (ms * 1e-3),
                     "kernel_ms": {"prep": prep_ms, "assemble": asm_ms},
                     "autotuned": {"single_launch": fused, "launch_cfg_by_degree": row[1:],
                                   "ms_per_step": ms_t, "assemble_kernel_ms": asm_t},
                     "roofline": roofline_hbm(algorithmic_bytes(mesh, info, vb), asm_t, kname)}
        del vals, rhs
    ctx.close()
    return out


def polyhedra_study(D, torch, steps, warmup):
    """3D Poisson (A = I) on the 128^3-cube Kuhn mesh agglomerated into 32,768
    polyhedra (about 384 tetrahedra each), p = 2 (10 dofs per cell): the whole
    path replayed from a graph, and the per-launch kernel times, FP32 and FP64."""
    from meshgen import config_mesh, problem_params
    log("polyhedra: 128^3 Kuhn cubes, 32,768 cells")
    t0 = time.perf_counter()
    mesh = config_mesh(4)
    gen_s = time.perf_counter() - t0
    params = problem_params(4)
    ctx = D.Context(0)
    ctx.upload(mesh)
    info = ctx.pattern()
    out = {"workload": "3D Poisson, 128^3 Kuhn tetrahedra agglomerated into 32768 polyhedra, p=2",
           "cells": mesh.n_cells, "tetrahedra": int(mesh.cell_ptr[-1] // 4), "faces": mesh.n_faces,
           "nnzb": info.nnzb, "n_vals": info.n_vals, "n_dofs": info.n_dofs, "mesh_generation_s": gen_s}
    for prec, name in ((D.F32, "f32"), (D.F64, "f64")):
        vals, rhs = ctx.outputs(prec)
        ctx.graph_capture(0, params, prec, vals, rhs)
        ms = _replay_ms(ctx, D, torch, steps, warmup)
        ctx.run(params, prec, vals, rhs)
        prep_ms, asm_ms = ctx.time_kernels(10)
        vb = 4 if prec == D.F32 else 8
        fl = flops_3d(mesh, info)
        peak = 157.3 if prec == D.F32 else 78.6
        tf = fl / (asm_ms * 1e-3) / 1e12
        out[name] = {"ms_per_step": ms, "block_nnz_per_s": info.nnzb / (ms * 1e-3),
                     "kernel_ms": {"prep": prep_ms, "assemble": asm_ms},
                     "roofline": {"bound": "alu", "achieved": tf, "peak": peak, "unit": "TFLOP/s",
                                  "frac": tf / peak, "traffic": None, "algorithmic_flops": fl,
                                  "kernel": "k_vol3d + k_face3d",
                                  "hbm": roofline_hbm(algorithmic_bytes_3d(mesh, info, vb), asm_ms,
                                                      "k_vol3d + k_face3d")}}
        del vals, rhs
    ctx.close()
    return out


def approach1_study(D, torch, steps, warmup):
    """Approach 1 of Section 3.3 (COO records with duplicates, radix sort,
    segmented sums) against the pattern-first row-owner path on the 16,384-cell
    FP32 workload: device time per whole assembly, pattern included."""
    from meshgen import config_mesh, problem_params
    log("Approach 1 ablation: 16,384-cell mesh")
    mesh, params = config_mesh(2), problem_params(2)
    ctx = D.Context(0)
    ctx.upload(mesh)
    info = ctx.pattern()
    out = {}
    ctx.assemble_coo(params, D.F32)
    torch.cuda.synchronize()
    for _ in range(warmup):
        ctx.assemble_coo(params, D.F32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.assemble_coo(params, D.F32)
    torch.cuda.synchronize()
    a1 = (time.perf_counter() - t0) * 1e3 / steps
    vals, rhs = ctx.outputs(D.F32)
    for _ in range(warmup):
        ctx.run(params, D.F32, vals, rhs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.run(params, D.F32, vals, rhs)
    torch.cuda.synchronize()
    a2 = (time.perf_counter() - t0) * 1e3 / steps
    ctx.close()
    records = mesh.n_cells + 4 * mesh.n_faces
    return {"workload": "2D DAR, 16384-cell seeded Voronoi, p=2, FP32", "nnzb": info.nnzb, "coo_records": records,
            "approach1_ms_per_step": a1, "approach2_ms_per_step": a2, "approach2_speedup": a1 / a2,
            "approach1_block_nnz_per_s": info.nnzb / (a1 * 1e-3)}


def spacetime_study(D, torch, steps, warmup):
    """One space-time slab (Section 2.3) of the parabolic benchmark's kind (a = 1,
    w = 0, c = 1) on prisms over the 16,384-cell Voronoi mesh, p = 1..3, FP64
    and FP32: device time per slab, block nonzeros and seconds per million
    degrees of freedom (the unit of the paper's tables)."""
    from meshgen import voronoi_mesh
    log("space-time slabs: 16,384 prisms")
    heat = dict(a0=1.0, a1=0.0, b=(0.0, 0.0, 0.0), c=1.0, c_sigma=10.0, u="sin")
    out = {"workload": "space-time slab, prisms over a 16384-cell seeded Voronoi mesh, a=1, w=0, c=1"}
    for p in (1, 2, 3):
        mesh = voronoi_mesh(16384, 2007048812, lloyd=0, p=p)
        ctx = D.Context(0)
        ctx.upload(mesh)
        info = ctx.pattern()
        nb = (p + 1) * (p + 2) * (p + 3) // 6
        for prec, name in ((D.F64, "f64"), (D.F32, "f32")):
            outs = ctx.assemble_st(heat, prec, 0.0, 0.01)
            for _ in range(warmup):
                ctx.assemble_st(heat, prec, 0.0, 0.01, out=outs)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                ctx.assemble_st(heat, prec, 0.0, 0.01, out=outs)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            mdof = mesh.n_cells * nb / 1e6
            out[f"p{p}_{name}"] = {"ms_per_slab": ms, "dofs": mesh.n_cells * nb,
                                   "block_nnz_per_s": info.nnzb / (ms * 1e-3), "s_per_mdof": ms * 1e-3 / mdof}
            del outs
        ctx.close()
    return out


def traffic_probe(D, torch, which="voronoi16384"):
    """A short program for rocprofv3 --pmc: a workload's assembly dispatches and
    a copy of known size to scale the counters by.
      voronoi16384  10 steps (FP32) of the 16,384-cell workload, 10 more in each
                    of the four launch configurations (cfg = r + 2 s: register
                    budget r, row order s);
      mixed262144   the 262,144-cell mixed-degree mesh, FP32: 5 steps with one
                    launch per degree, then 5 with the single persistent launch;
      kuhn128       the 32,768-polyhedron mesh, 5 FP32 steps, then 5 FP64."""
    from meshgen import config_mesh, problem_params
    k = {"voronoi16384": 2, "mixed262144": 3, "kuhn128": 4}[which]
    mesh, params = config_mesh(k), problem_params(k)
    ctx = D.Context(0)
    ctx.upload(mesh)
    ctx.pattern()
    if which == "voronoi16384":
        vals, rhs = ctx.outputs(D.F32)
        for _ in range(10):
            ctx.run(params, D.F32, vals, rhs)
        for cfg in range(4):
            ctx.set_launch(D.F32, 2, cfg)
            for _ in range(10):
                ctx.run(params, D.F32, vals, rhs)
    elif which == "mixed262144":
        vals, rhs = ctx.outputs(D.F32)
        for fused in (0, 1):
            ctx.set_launch(D.F32, 0, fused)
            for _ in range(5):
                ctx.run(params, D.F32, vals, rhs)
    else:
        for prec in (D.F32, D.F64):
            vals, rhs = ctx.outputs(prec)
            for _ in range(5):
                ctx.run(params, prec, vals, rhs)
    torch.cuda.synchronize()
    del vals, rhs
    x = torch.empty(16 * 1024 * 1024, dtype=torch.float32, device="cuda")  # 64 MiB
    y = torch.empty_like(x)
    x.fill_(1.0)
    for _ in range(10):
        y.copy_(x)
    torch.cuda.synchronize()
    ctx.close()
    log(f"traffic probe {which} done")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-reduced", action="store_true", help="skip the reduced-rule study")
    ap.add_argument("--no-3d", action="store_true", help="skip the polyhedral (3D) workload")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-degree 262,144-cell workload")
    ap.add_argument("--no-extras", action="store_true", help="skip the Approach-1 and space-time studies")
    ap.add_argument("--traffic-probe", nargs="?", const="voronoi16384", default=None,
                    choices=["voronoi16384", "mixed262144", "kuhn128"],
                    help="for HBM counter runs: a few whole steps of one workload (default the headline one, "
                         "in each of its four launch configurations), then 10 copies of a "
                         "64 MiB tensor (the copy calibrates FETCH_SIZE / WRITE_SIZE); prints no JSON")
    ap.add_argument("--train-polygons", type=int, default=1_000_000)
    ap.add_argument("--train-epochs", type=int, default=30)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build assembles on exactly one GPU (the method needs no communication; "
              "the multi-GPU layout is described in the design notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2007_04881_amd as D
    from meshgen import config_mesh, problem_params

    if args.traffic_probe:
        traffic_probe(D, torch, args.traffic_probe)
        return

    log("16,384-cell mesh")
    mesh = config_mesh(2)
    params = problem_params(2)
    ctx = D.Context(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.upload(mesh)  # host checks + copy of the host arrays to the device
    upload_ms = (time.perf_counter() - t0) * 1e3
    info = ctx.pattern()
    vals, rhs = ctx.outputs(D.F32)

    # single-shot latency of the eager path (pattern + geometry + assembly)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.run(params, D.F32, vals, rhs)
    torch.cuda.synchronize()
    single_ms = (time.perf_counter() - t0) * 1e3

    # launch tuning (outside the timed region): the row kernel's register budget
    cfg = ctx.autotune(200)[1][2]
    alt = cfg & 1

    # the timed steps: the whole path, one asynchronous dgp_run per step, back to
    # back on the context stream (the host enqueues a step in ~10 us, well
    # inside a step's device time)
    for _ in range(args.warmup):
        ctx.run(params, D.F32, vals, rhs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.run(params, D.F32, vals, rhs)
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    ms_per_step = t_steps * 1e3 / args.steps

    # the same step replayed from a captured HIP graph
    ctx.graph_capture(0, params, D.F32, vals, rhs)
    ms_graph = _replay_ms(ctx, D, torch, args.steps, args.warmup)

    # values only (pattern reused), as in time stepping with changing coefficients
    for _ in range(args.warmup):
        ctx.assemble(params, D.F32, vals, rhs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.assemble(params, D.F32, vals, rhs)
    torch.cuda.synchronize()
    ms_values = (time.perf_counter() - t0) * 1e3 / args.steps

    # per-launch device time of the kernels: HIP events on the context stream
    # around 50 back-to-back re-launches of the last step's kernels
    ctx.run(params, D.F32, vals, rhs)
    prep_ms, asm_ms = ctx.time_kernels(50)
    avg = {"prep": prep_ms, "assemble": asm_ms}
    abytes = algorithmic_bytes(mesh, info, 4)
    achieved = abytes / (avg["assemble"] * 1e-3) / 1e9
    copy_gbs = hbm_copy_gbs(torch)

    out = {
        "metric": "assembled block-nnz/s, 2D Voronoi p=2 (whole path: geometry + pattern + assembly)",
        "value": info.nnzb * args.steps / t_steps,
        "unit": "block-nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Voronoi mesh, manufactured solution)",
        "config": {"workload": "2D DAR, 16384-cell seeded Voronoi, p=2, FP32 contraction with FP64 geometry",
                   "cells": mesh.n_cells, "nnzb": info.nnzb, "n_vals": info.n_vals, "n_dofs": info.n_dofs,
                   "parallelism": "single GPU"},
        "elements_per_s": mesh.n_cells * args.steps / t_steps,
        "values_only": {"ms_per_step": ms_values, "block_nnz_per_s": info.nnzb / (ms_values * 1e-3)},
        "graph_replay": {"ms_per_step": ms_graph, "block_nnz_per_s": info.nnzb / (ms_graph * 1e-3)},
        "single_shot_ms": single_ms,
        "kernel_ms": avg,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(cfg),
                     "kernel": f"k_row2d_f32<2,true,{alt}>", "algorithmic_bytes": abytes,
                     "measured_copy_gbs": copy_gbs, "frac_of_measured_copy": achieved / copy_gbs,
                     "valu_issue": valu_issue(cfg, avg["assemble"])},
        "upload_ms": upload_ms,
        "launch_config": {"cfg": cfg, "register_budget": "one more wave per SIMD" if alt else "default",
                          "row_order": "per XCD range, most sub-triangles first" if cfg & 2 else "cell id"},
    }
    ctx.close()
    if not args.no_reduced:
        out["reduced_rules"] = reduced_rule_study(D, torch, 20, 3, args.train_polygons, args.train_epochs)
    if not args.no_mixed:
        out["mixed_degrees"] = mixed_degree_study(D, torch, 20, 3)
    if not args.no_3d:
        out["polyhedra"] = polyhedra_study(D, torch, 20, 3)
    if not args.no_extras:
        out["approach1"] = approach1_study(D, torch, 20, 3)
        out["spacetime"] = spacetime_study(D, torch, 10, 2)
    if not args.no_cpu:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(mesh, params)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
