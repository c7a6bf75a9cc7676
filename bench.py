#!/usr/bin/env python3
"""Benchmark of the matrix-free stabilized Navier-Stokes Jacobian with mortar
faces on one MI355X.

Timed region: K applications of the FP64 Jacobian (the metric's unit of work)
on the 3D Q2 annular rotor/stator workload (64 x 8 x 32 cells per domain,
1,131,520 DoFs), inputs resident in HBM, bracketed by device synchronization.
The other rows of the hot path are timed in the same run and reported beside
the metric: rotor rotation + mortar setup, linearization, the FP32 Jacobian,
the diagonal, and the FGMRES solve (plain FP64 vs FP32-preconditioned).

Prints one JSON line.  `--gpus N` with N > 1 exits: the library runs on one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DoFs/s of stabilized NS Jacobian vmult (FP64 vs FP32) + GMRES solve time to 1e-8"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# FP64 flops that the quad-layout volume kernel executes per 3D Q2 cell, from
# its SQ_INSTS_VALU_{FMA,MUL,ADD}_F64 counters on the 32,768-cell mesh
# (64 lanes x (2 FMA + MUL + ADD) per dispatch / cells); the fourth lane of a
# quad repeats the third slice, so a quarter of them is duplicate work
QUAD_Q2_FLOP_PER_CELL = 19160


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="annulus3d_q2_64x8x32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--solve-maxit", type=int, default=4000)
    ap.add_argument("--solve-dt", type=float, default=0.01,
                    help="time step of the BDF2 Jacobian solved on degree-3 workloads")
    ap.add_argument("--solve-restart", type=int, default=30)
    ap.add_argument("--cheb-degree", type=int, default=12)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--fused", type=int, default=-1,
                    help="-1: automatic; 1: volume and mortar in one launch; 2: mortar on a second stream; 0: sequential")
    ap.add_argument("--volume-layout", type=int, default=1, help="1: lane quad per cell (3D, k = 2, 3); 0: LDS planes")
    ap.add_argument("--no-batch", action="store_true", help="skip the batching leg (48 uneven instances)")
    ap.add_argument("--no-iso", action="store_true", help="skip the curved-mesh (iso-parametric) leg")
    ap.add_argument("--no-copy-bandwidth", action="store_true", help="skip the device-copy bandwidth measurement")
    ap.add_argument("--transient", action="store_true",
                    help="also time one BDF2 + Newton step (transient workloads; rotor advances omega * dt)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 7.3M- and 68M-DoF legs (vmults, degree-3 multigrid solve, 68M-DoF time step)")
    return ap.parse_args()


def algorithmic_bytes_volume(mesh, n_dofs, real_bytes, lin_source=0):
    """Minimum HBM bytes of one application: read src once, write dst once,
    read the per-point linearization data once (source B: 16 values per point
    in 3D, 9 in 2D; source C: tau and tau R, 4 values per point, plus the
    state's velocity once, 3/4 of a vector)."""
    dim, k = mesh["dim"], mesh["degree"]
    n = k + 1
    nz = mesh["n_z"] if dim == 3 else 1
    cells = mesh["n_theta"] * (mesh["n_r_rotor"] + mesh["n_r_stator"]) * nz
    if lin_source == 1:
        return (2.75 * n_dofs + 4 * n ** dim * cells) * real_bytes, cells
    lin = (16 if dim == 3 else 9) * n ** dim * cells
    return (2 * n_dofs + lin) * real_bytes, cells


def has_source_c(mesh, real="double"):
    """Linearization source C exists with the quad layout: 3D degree 2 in
    both precisions, degree 3 in FP32."""
    return mesh["dim"] == 3 and (mesh["degree"] == 2 or (mesh["degree"] == 3 and real == "float"))


def dominant_kernel(mesh, fused, layout, real="double", lin_source=0):
    """Name of the launch that the volume timer brackets."""
    dim, k = mesh["dim"], mesh["degree"]
    quad = layout == 1 and dim == 3 and k in (2, 3)
    c = "true" if (lin_source == 1 and has_source_c(mesh, real)) else "false"
    if fused < 0:
        cells = mesh["n_theta"] * (mesh["n_r_rotor"] + mesh["n_r_stator"]) * (mesh["n_z"] if dim == 3 else 1)
        fused = 2 if cells >= (1 << 18) else 1
    fused = 1 if fused == 1 else 0
    if quad and fused and real == "double" and k == 2:
        return f"mns::k_jacobian_fused_quad_lds<3, {c}>"
    if quad:
        return f"mns::k_jacobian_{'fused' if fused else 'volume'}_quad<{real}, {k + 1}, {c}>"
    return f"mns::k_jacobian_{'fused' if fused else 'volume'}<{real}, {dim}, {k + 1}>"


def source_c_leg(op, mesh, x, sync, steps, warmup=5):
    """The vmult with linearization source C (tau and tau R per point, a and
    grad u evaluated from the state) next to source B, both precisions, in
    the automatic launch mode: HIP-event time per application and the HBM
    rate against each source's own algorithmic bytes."""
    import torch

    n = x.numel()
    cfg = op.get_kernel_config()
    out = {}
    for label, xx, real, rb in (("fp64", x, "double", 8), ("fp32", x.float(), "float", 4)):
        if not has_source_c(mesh, real):
            continue
        y = torch.empty_like(xx)
        rec = {}
        for src in (0, 1):
            op.set_kernel_config(lin_source_f64=src, lin_source_f32=src)
            for _ in range(warmup):
                op.apply_jacobian(xx, y)
            sync()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                op.apply_jacobian(xx, y)
            e1.record()
            sync()
            ms = e0.elapsed_time(e1) / steps
            nbytes, _ = algorithmic_bytes_volume(mesh, n, rb, src)
            rec["BC"[src]] = {"ms_per_vmult": ms, "algorithmic_bytes": nbytes,
                              "frac_of_8TBs": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "kernel": dominant_kernel(mesh, cfg["fused_launch"], 1, real, src)}
        rec["faster"] = "C" if rec["C"]["ms_per_vmult"] < rec["B"]["ms_per_vmult"] else "B"
        rec["speedup_C_over_B"] = rec["B"]["ms_per_vmult"] / rec["C"]["ms_per_vmult"]
        out[label] = rec
        del y
    op.set_kernel_config(**cfg)
    return out


def kernel_source_digest():
    import hashlib

    path = os.path.join(ROOT, "paper_2608_27423_amd", "csrc", "mns_kernels.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def measured_traffic(workload, kernel):
    """HBM bytes of one FP64 vmult (all its launches) and of `kernel` alone,
    from the committed counter summary of this workload (FETCH_SIZE and
    WRITE_SIZE passes scaled by a plain copy): (vmult bytes, kernel bytes),
    each None when missing or when the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None, None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith((" ", "#", "|")):
            key, val = line.rsplit(":", 1)  # kernel names in the keys hold "::"
            rec[key.strip()] = val.strip()
    if rec.get("kernel_source_sha256") != kernel_source_digest():
        return None, None

    def num(key):
        try:
            return float(rec[key])
        except (KeyError, ValueError):
            return None

    return num("vmult_bytes_per_call"), num(f"bytes_per_launch {kernel}")


def batch_leg(args, dev, sync):
    """48 uneven rotor/stator instances (half 2D, half 3D Q2; angles and
    Reynolds numbers seeded) in one batch: FP64 Jacobian of every instance,
    once as one batched call (one volume + mortar launch and one gather launch
    per dimension) and once as one mns_apply_jacobian per instance; 30
    FGMRES iterations of every instance as one batched solve (one graph per
    lockstep iteration over all 48) and as one solve per instance; the same
    with the multigrid V-cycle as preconditioner (10 iterations)."""
    import torch

    from paper_2608_27423_amd import binding, inputs

    insts = inputs.batch_instances()
    ops = []
    for mesh_i, th, om, seed in insts:
        o = binding.Operator(mesh_i)
        o.rotate_rotor(th, om)
        o.set_linearization(torch.from_numpy(inputs.uniform(o.n_dofs, seed)).to(dev))
        ops.append(o)
    groups = [[o for o in ops if o.mesh["dim"] == d] for d in (2, 3)]
    batches = [binding.Batch(ops)]
    xs = [torch.from_numpy(inputs.uniform(b.n_dofs, 7 + i)).to(dev) for i, b in enumerate(batches)]
    ys = [torch.empty_like(x) for x in xs]
    total = sum(b.n_dofs for b in batches)
    reps = max(args.steps // 2, 10)

    def t_batched(dtype):
        xx = [x.to(dtype) for x in xs]
        yy = [y.to(dtype) for y in ys]
        for _ in range(3):
            for b, x, y in zip(batches, xx, yy):
                b.apply_jacobian(x, y)
        sync()
        t0 = time.perf_counter()
        for _ in range(reps):
            for b, x, y in zip(batches, xx, yy):
                b.apply_jacobian(x, y)
        sync()
        return (time.perf_counter() - t0) / reps, yy

    def t_single():
        sl = []
        for b, x, y in zip(batches, xs, ys):
            for o, off in zip(b._ops, b.offsets):
                sl.append((o, x[off:off + o.n_dofs], y[off:off + o.n_dofs]))
        for _ in range(3):
            for o, x, y in sl:
                o.apply_jacobian(x, y)
        sync()
        t0 = time.perf_counter()
        for _ in range(reps):
            for o, x, y in sl:
                o.apply_jacobian(x, y)
        sync()
        return (time.perf_counter() - t0) / reps

    tb, yb = t_batched(torch.float64)
    ref = [y.clone() for y in yb]
    ts = t_single()
    same = all(bool(torch.equal(a, b)) for a, b in zip(ref, ys))
    tb32, _ = t_batched(torch.float32)

    # 30 FGMRES iterations (one restart cycle, FP32 Jacobi-Chebyshev degree 4)
    # of every instance: two batched solves against one solve per instance
    sopts = dict(rtol=1e-14, restart=30, maxit=30, precond="f32", cheb_degree=4)
    rhs = [torch.from_numpy(inputs.uniform(b.n_dofs, 31 + i)).to(dev) for i, b in enumerate(batches)]
    for b, r in zip(batches, rhs):
        b.solve(r, check=False, **dict(sopts, maxit=1))
    for b, r in zip(batches, rhs):
        for o, off in zip(b._ops, b.offsets):
            o.solve(r[off:off + o.n_dofs], check=False, **dict(sopts, maxit=1))
    sync()
    t0 = time.perf_counter()
    batch_its = []
    for b, r in zip(batches, rhs):
        _, _, reps = b.solve(r, check=False, **sopts)
        batch_its += [rp["iterations"] for rp in reps]
    sync()
    t_bsolve = time.perf_counter() - t0
    t0 = time.perf_counter()
    single_its = []
    for b, r in zip(batches, rhs):
        for o, off in zip(b._ops, b.offsets):
            _, rp = o.solve(r[off:off + o.n_dofs], check=False, **sopts)
            single_its.append(rp["iterations"])
    sync()
    t_ssolve = time.perf_counter() - t0

    # 10 FGMRES iterations with the multigrid V-cycle (FP32 smoothing, FP64
    # direct coarsest level) as preconditioner: every level batched over the
    # instances (inside the iteration graph) against one solve per instance;
    # the hierarchies are set up by an untimed one-iteration solve first
    mopts = dict(rtol=1e-14, restart=30, maxit=10, precond="mg")
    for b, r in zip(batches, rhs):
        b.solve(r, check=False, **dict(mopts, maxit=1))
        for o, off in zip(b._ops, b.offsets):
            o.solve(r[off:off + o.n_dofs], check=False, **dict(mopts, maxit=1))
    sync()
    t0 = time.perf_counter()
    mg_its, mg_rc = [], set()
    for b, r in zip(batches, rhs):
        _, rc, reps = b.solve(r, check=False, **mopts)
        mg_rc.add(rc)
        mg_its += [rp["iterations"] for rp in reps]
    sync()
    t_bmg = time.perf_counter() - t0
    t0 = time.perf_counter()
    mg_single_its, mg_single_rc = [], set()
    for b, r in zip(batches, rhs):
        for o, off in zip(b._ops, b.offsets):
            _, rp = o.solve(r[off:off + o.n_dofs], check=False, **mopts)
            mg_single_rc.add(rp["rc"])
            mg_single_its.append(rp["iterations"])
    sync()
    t_smg = time.perf_counter() - t0
    out = {
        "instances": len(ops), "instances_2d": len(groups[0]), "instances_3d": len(groups[1]), "dofs": total,
        "dofs_2d": sum(o.n_dofs for o in groups[0]), "dofs_3d": sum(o.n_dofs for o in groups[1]),
        "batches": "one batch of all instances (launch groups: 2D Q2, 3D Q2)",
        "batched_ms": 1e3 * tb, "batched_dofs_per_s": total / tb,
        "single_launches_ms": 1e3 * ts, "single_launches_dofs_per_s": total / ts,
        "speedup_batched_over_single": ts / tb,
        "batched_fp32_ms": 1e3 * tb32, "batched_fp32_dofs_per_s": total / tb32,
        "batched_equals_single": same,
        "fgmres_30_iterations": {
            "batched_s": t_bsolve, "single_solves_s": t_ssolve, "speedup_batched_over_single": t_ssolve / t_bsolve,
            "iterations_batched": sum(batch_its), "iterations_single": sum(single_its),
            "solver": "FGMRES(30) FP64, Jacobi-Chebyshev degree 4 in FP32, 30 iterations per instance (rtol 1e-14)"},
        "fgmres_10_iterations_multigrid": {
            "batched_s": t_bmg, "single_solves_s": t_smg, "speedup_batched_over_single": t_smg / t_bmg,
            "iterations_batched": sum(mg_its), "iterations_single": sum(mg_single_its),
            "return_codes_batched": sorted(mg_rc), "return_codes_single": sorted(mg_single_rc),
            "solver": "FGMRES(30) FP64, V-cycle with FP32 Chebyshev smoothing (degree 2) and FP64 direct coarsest "
                      "level, 10 iterations per instance (rtol 1e-14: return code -4, not converged, expected)"},
        "recipe": "inputs.batch_instances(): 2D Q2 32x4..256x32, 3D Q2 16x4x8..64x8x16 per domain, "
                  "angles U[0, 2pi), Re log-uniform in [1, 2000], steady, nodal-uniform states",
    }
    for b in batches:
        b.close()
    for o in ops:
        o.close()
    return out


def copy_bandwidth(dev, sync, nbytes=1 << 30, reps=20):
    """Device-to-device copy rate (bytes read + written per second) of a
    buffer far larger than the 256 MB Infinity Cache: the practical HBM
    ceiling beside the 8 TB/s spec figure."""
    import torch

    a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sync()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    sync()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / t / 1e9


def degree3_solve_leg(args, mesh, name, theta, omega, dev, sync):
    """Solve leg of the degree-3 workload: the Jacobian of one BDF2 time step
    (dt = --solve-dt, history of a state at rest in time, so that the
    point residual is the steady one) at the smooth state, FGMRES(30) to 1e-8
    with the V-cycle (degree 3 -> 2 on the same mesh, then halved meshes;
    Picard coarse levels) in FP32 against FP64.  The steady degree-3
    operator is not solved by Jacobi-type polynomial smoothing (neither
    V-cycle nor single-level polynomial), so the steady solve is not timed."""
    import numpy as np
    import torch

    from paper_2608_27423_amd import binding, inputs

    dt = args.solve_dt
    tmesh = dict(mesh, steady=0, dt=dt)
    out = {}
    with binding.Operator(tmesh) as sop:
        sop.rotate_rotor(theta, omega)
        s = inputs.smooth_field(tmesh, inputs.STATE_SEED[name])
        s /= np.abs(s).max()
        st = torch.from_numpy(s).to(dev)
        sop.set_linearization(st, hist=-1.5 / dt * st)
        xstar = torch.from_numpy(inputs.uniform(sop.n_dofs, inputs.SOLUTION_SEED[name])).to(dev)
        rhs = sop.apply_jacobian(xstar)
        mgo = dict(rtol=1e-8, restart=30, maxit=args.solve_maxit, mg_coarse_linearization="picard", eig_iters=60)
        sop.solve(rhs, torch.zeros_like(rhs), check=False, precond="mg", **dict(mgo, maxit=1))
        for label, prec in (("plain_fp64", "mg64"), ("mixed_fp32", "mg")):
            xs = torch.zeros_like(rhs)
            sync()
            _, info = sop.solve(rhs, xs, check=False, precond=prec, **mgo)
            chk = sop.apply_jacobian(xs)
            sync()
            out[label] = {"seconds": info["seconds"], "iterations": info["iterations"], "converged": info["rc"] == 0,
                          "true_rel_residual": float((rhs - chk).norm() / rhs.norm()),
                          "vmults_f64": info["vmults_f64"], "vmults_f32": info["vmults_f32"]}
        out["levels"] = sop.mg_levels()
    p, m = out["plain_fp64"], out["mixed_fp32"]
    out["speedup_mixed_over_plain"] = p["seconds"] / m["seconds"] if m["seconds"] > 0 else None
    out["operator"] = (f"Jacobian of one BDF2 step, dt = {dt}, history of a state at rest in time (not the "
                       f"steady operator: see steady_attempt)")
    out["state"] = "smooth manufactured field scaled to max |u| = 1"
    out["preconditioner"] = ("geometric/polynomial multigrid V-cycle (degree 3 -> 2, then halved meshes), "
                             "Picard-linearized coarse levels, Jacobi-Chebyshev smoothing degree 2 on "
                             "[1.05 lambda/5, 1.05 lambda] (lambda by 60 power iterations) in FP32 (mixed) or FP64 "
                             "(plain), FGMRES(30)")
    return {"multigrid": out}


def vmult_leg(name, dev, sync, steps=100, warmup=10):
    """FP64 and FP32 Jacobian of a workload: per-application time from HIP
    events on the launch stream over `steps` back-to-back applications, the
    dominant launch's time from its own dispatch events, and the HBM roofline
    of the whole application (algorithmic bytes over its time)."""
    import torch

    from paper_2608_27423_amd import binding, inputs

    mesh = inputs.mesh(name)
    theta = inputs.rotor_angle(name)
    op = binding.Operator(mesh)
    op.rotate_rotor(theta, mesh["omega"])
    op.set_linearization(torch.from_numpy(inputs.state_for(name)).to(dev))
    x = torch.from_numpy(inputs.vector_for(name)).to(dev)
    n = x.numel()
    out = {"workload": name, "dofs": n}
    for label, xx in (("fp64", x), ("fp32", x.float())):
        y = torch.empty_like(xx)
        for _ in range(warmup):
            op.apply_jacobian(xx, y)
        sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            op.apply_jacobian(xx, y)
        e1.record()
        sync()
        ms = e0.elapsed_time(e1) / steps
        op.enable_timing(steps)
        for _ in range(steps):
            op.apply_jacobian(xx, y)
        sync()
        t = op.read_timing()
        op.enable_timing(0)
        nbytes, _ = algorithmic_bytes_volume(mesh, n, 8 if label == "fp64" else 4)
        vol_ms = t["ms_volume"] / max(1, t["n_volume"])
        out[label] = {"ms_per_vmult": ms, "dofs_per_s": n / (ms * 1e-3), "volume_kernel_ms": vol_ms,
                      "mortar_kernel_ms": t["ms_mortar"] / max(1, t["n_mortar"]),
                      "algorithmic_bytes": nbytes, "achieved_GBs": nbytes / (ms * 1e-3) / 1e9,
                      "frac_of_8TBs": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "volume_launch_frac_of_8TBs": nbytes / (vol_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "volume_kernel": dominant_kernel(mesh, -1, 1, "double" if label == "fp64" else "float")}
        del y
    out["fp32_speedup_over_fp64"] = out["fp64"]["ms_per_vmult"] / out["fp32"]["ms_per_vmult"]
    out["lin_source_c"] = source_c_leg(op, mesh, x, sync, steps // 2 or 1)
    return op, mesh, theta, out


ISO_PERTURB = 0.1  # interior node displacement of the curved mesh, in cell sizes


def algorithmic_bytes_iso(mesh, n_dofs, real_bytes):
    """Minimum HBM bytes of one application on iso-parametric cells: src read
    and dst written once, per point the linearization data (16 values in 3D,
    9 in 2D) and the metric (inverse Jacobian, JxW and the mapping term of
    the Laplacian: 13 values in 3D, 7 in 2D) read once."""
    dim, k = mesh["dim"], mesh["degree"]
    nz = mesh["n_z"] if dim == 3 else 1
    cells = mesh["n_theta"] * (mesh["n_r_rotor"] + mesh["n_r_stator"]) * nz
    per_point = (16 + 13) if dim == 3 else (9 + 7)
    return (2 * n_dofs + per_point * (k + 1) ** dim * cells) * real_bytes, cells


def iso_leg(name, dev, sync, steps=100, warmup=10):
    """The workload on a curved mesh (every interior node moved by up to
    ISO_PERTURB cells, inputs.iso_node_positions; cells are the Q_k
    interpolants of their nodes): set-up times, FP64 and FP32 vmult with the
    HIP-event time per application and per kernel class, the HBM roofline
    against the iso algorithmic bytes, and a mixed-precision Jacobi-Chebyshev
    FGMRES solve to 1e-8 next to the same solve on the polar mesh."""
    import numpy as np
    import torch

    from paper_2608_27423_amd import binding, inputs

    mesh = inputs.mesh(name)
    theta = inputs.rotor_angle(name)
    xyz = inputs.iso_node_positions(mesh, ISO_PERTURB)
    op = binding.Operator(mesh)
    out = {"workload": name, "perturb_cells": ISO_PERTURB}
    _, t = timed(lambda: op.set_node_positions(xyz), sync)
    out["set_node_positions_ms"] = 1e3 * t
    state = torch.from_numpy(inputs.state_for(name)).to(dev)
    op.rotate_rotor(theta, mesh["omega"])
    op.set_linearization(state)
    _, t = timed(lambda: op.rotate_rotor(theta, mesh["omega"]), sync)
    out["rotate_rotor_ms"] = 1e3 * t
    _, t = timed(lambda: op.set_linearization(state), sync)
    out["set_linearization_ms"] = 1e3 * t
    x = torch.from_numpy(inputs.vector_for(name)).to(dev)
    n = x.numel()
    for label, xx in (("fp64", x), ("fp32", x.float())):
        y = torch.empty_like(xx)
        for _ in range(warmup):
            op.apply_jacobian(xx, y)
        sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            op.apply_jacobian(xx, y)
        e1.record()
        sync()
        ms = e0.elapsed_time(e1) / steps
        op.enable_timing(steps)
        for _ in range(steps):
            op.apply_jacobian(xx, y)
        sync()
        tt = op.read_timing()
        op.enable_timing(0)
        real = "double" if label == "fp64" else "float"
        nbytes, _ = algorithmic_bytes_iso(mesh, n, 8 if label == "fp64" else 4)
        vol_ms = tt["ms_volume"] / max(1, tt["n_volume"])
        out[label] = {"ms_per_vmult": ms, "dofs_per_s": n / (ms * 1e-3), "volume_kernel_ms": vol_ms,
                      "mortar_kernel_ms": tt["ms_mortar"] / max(1, tt["n_mortar"]),
                      "algorithmic_bytes": nbytes, "achieved_GBs": nbytes / (ms * 1e-3) / 1e9,
                      "frac_of_8TBs": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "volume_launch_frac_of_8TBs": nbytes / (vol_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "volume_kernel": f"mns::k_jacobian_fused<{real}, {mesh['dim']}, {mesh['degree'] + 1}, true>"}
        del y
    out["fp32_speedup_over_fp64"] = out["fp64"]["ms_per_vmult"] / out["fp32"]["ms_per_vmult"]
    # HBM bytes of the FP64 application from the committed counter summary
    # (profile_vmult.py --iso), when it matches the current kernel source
    tb, tk = measured_traffic("curved_" + name, out["fp64"]["volume_kernel"])
    if tb is not None:
        ms = out["fp64"]["ms_per_vmult"]
        out["fp64"]["measured_bytes_per_vmult"] = tb
        out["fp64"]["measured_GBs"] = tb / (ms * 1e-3) / 1e9
        out["fp64"]["measured_over_algorithmic"] = tb / out["fp64"]["algorithmic_bytes"]
        out["fp64"]["dominant_launch_measured_bytes"] = tk
    # mixed-precision solve on the curved and on the polar mesh
    sstate = inputs.smooth_field(mesh, inputs.STATE_SEED[name])
    sstate = torch.from_numpy(sstate / np.abs(sstate).max()).to(dev)
    xstar = torch.from_numpy(inputs.uniform(n, inputs.SOLUTION_SEED[name])).to(dev)
    solves = {}
    for label in ("curved", "polar"):
        if label == "polar":
            op.set_node_positions(None)
            op.rotate_rotor(theta, mesh["omega"])
        op.set_linearization(sstate)
        rhs = op.apply_jacobian(xstar)
        xs = torch.zeros_like(rhs)
        sync()
        _, info = op.solve(rhs, xs, check=False, rtol=1e-8, restart=50, maxit=2000, precond="f32", cheb_degree=6)
        chk = op.apply_jacobian(xs)
        sync()
        solves[label] = {"seconds": info["seconds"], "iterations": info["iterations"], "converged": info["rc"] == 0,
                         "true_rel_residual": float((rhs - chk).norm() / rhs.norm())}
    solves["preconditioner"] = "Jacobi-Chebyshev degree 6 in FP32, FGMRES(50) in FP64"
    out["solve"] = solves
    op.close()
    return out


def transient_leg(op, mesh, name, theta, dev, sync):
    """Two implicit time steps of a spin-up: fluid at rest, a smooth body
    force (the workload's smooth field, max 1) switched on, the rotor
    advancing omega dt per step; the second step is timed with the FP32 and
    with the FP64 V-cycle."""
    import torch

    from paper_2608_27423_amd import inputs

    omega, dt = mesh["omega"], mesh["dt"]
    force = torch.from_numpy(inputs.transient_start(mesh, inputs.STATE_SEED[name])).to(dev)
    u0 = torch.zeros_like(force)
    u1 = u0.clone()
    lin_opts = dict(rtol=1e-6, restart=30, maxit=600, precond="mg")
    op.bdf2_step(theta + omega * dt, omega, u0, u1, u_nm1=None, force=force, newton_rtol=1e-8, max_newton=10,
                 linear=lin_opts)
    steps = {}
    for label, prec in (("mixed_fp32_multigrid", "mg"), ("plain_fp64_multigrid", "mg64")):
        u = u1.clone()
        sync()
        info = op.bdf2_step(theta + 2 * omega * dt, omega, u1, u, u_nm1=u0, force=force, check=False,
                            newton_rtol=1e-8, max_newton=10, linear=dict(lin_opts, precond=prec))
        steps[label] = {"seconds": info["seconds"], "newton_iterations": info["newton_iterations"],
                        "linear_iterations": info["linear_iterations"], "converged": info["rc"] == 0,
                        "residual0": info["residual0"], "residual": info["residual"],
                        "line_search_halvings": info["line_search_halvings"]}
        del u
    m_, p_ = steps["mixed_fp32_multigrid"], steps["plain_fp64_multigrid"]
    del force, u0, u1
    return {**steps, "speedup_mixed_over_plain": p_["seconds"] / m_["seconds"] if m_["seconds"] > 0 else None,
            "dt": dt, "rotation_rad": omega * dt,
            "scenario": "spin-up from rest under a smooth body force; second BDF2 step timed",
            "newton_rtol": 1e-8,
            "linear": "FGMRES(30) FP64 to 1e-6, geometric multigrid V-cycle with an FP64 direct coarse solve, "
                      "Jacobi-Chebyshev smoothing in FP32 (mixed) or FP64 (plain)"}


def steady_degree3_attempt(mesh, name, theta, dev, sync, maxit=300):
    """The steady degree-3 operator itself (Re = 1/nu, no time derivative) at
    the smooth state: FGMRES(30) with the FP32 V-cycle (Picard coarse levels,
    FP64 direct coarse solve), stopped at `maxit` iterations; the reached
    relative residual is reported whether or not 1e-8 is met."""
    import numpy as np
    import torch

    from paper_2608_27423_amd import binding, inputs

    with binding.Operator(mesh) as sop:
        sop.rotate_rotor(theta, mesh["omega"])
        s = inputs.smooth_field(mesh, inputs.STATE_SEED[name])
        s /= np.abs(s).max()
        sop.set_linearization(torch.from_numpy(s).to(dev))
        rhs = sop.apply_jacobian(torch.from_numpy(inputs.uniform(sop.n_dofs, inputs.SOLUTION_SEED[name])).to(dev))
        xs = torch.zeros_like(rhs)
        sync()
        _, info = sop.solve(rhs, xs, check=False, rtol=1e-8, restart=30, maxit=maxit, precond="mg",
                            mg_coarse_linearization="picard", mg_fine_linearization="picard", eig_iters=60,
                            mg_smooth_degree=3, mg_smooth_range=10.0)
        chk = sop.apply_jacobian(xs)
        sync()
        return {"converged": info["rc"] == 0, "iterations": info["iterations"], "seconds": info["seconds"],
                "true_rel_residual": float((rhs - chk).norm() / rhs.norm()), "maxit": maxit,
                "operator": f"steady Jacobian, nu = {mesh['nu']}, smooth state (max |u| = 1)",
                "preconditioner": "FGMRES(30), FP32 V-cycle: Picard levels, smoothing degree 3 on "
                                  "[1.05 lambda/10, 1.05 lambda], FP64 direct solve on the coarsest level"}


def large_workloads_leg(args, dev, sync):
    """The degree-3 7.3M-DoF and degree-2 68M-DoF workloads in the default run:
    vmults in FP64 and FP32, the degree-3 multigrid solve (and the steady
    degree-3 attempt), one BDF2 + Newton step at 68M DoFs."""
    import torch

    out = {}
    name = "annulus3d_q3_64x16x32"
    op, mesh, theta, rec = vmult_leg(name, dev, sync)
    op.close()
    rec.update(degree3_solve_leg(args, mesh, name, theta, mesh["omega"], dev, sync))
    rec["steady_attempt"] = steady_degree3_attempt(mesh, name, theta, dev, sync)
    out[name] = rec
    torch.cuda.empty_cache()
    name = "annulus3d_q2_256x32x128"
    op, mesh, theta, rec = vmult_leg(name, dev, sync, steps=50, warmup=5)
    rec["transient_step"] = transient_leg(op, mesh, name, theta, dev, sync)
    op.close()
    out[name] = rec
    torch.cuda.empty_cache()
    return out


def timed(fn, sync):
    sync()
    t0 = time.perf_counter()
    out = fn()
    sync()
    return out, time.perf_counter() - t0


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; multi-GPU sharding is design-only "
                                   "(axial slabs, see the design notes)", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2608_27423_amd import binding, inputs

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    sync = torch.cuda.synchronize
    name = args.workload
    mesh = inputs.mesh(name)
    theta = inputs.rotor_angle(name)
    omega = mesh["omega"]
    state_np = inputs.state_for(name)
    x_np = inputs.vector_for(name)
    n = x_np.size
    state = torch.from_numpy(state_np).to(dev)
    x64 = torch.from_numpy(x_np).to(dev)
    x32 = x64.float()
    y64 = torch.empty_like(x64)
    y32 = torch.empty_like(x32)
    rec = {}
    op = binding.Operator(mesh)
    op.set_kernel_config(fused_launch=args.fused, volume_layout=args.volume_layout)
    _, t_rot = timed(lambda: op.rotate_rotor(theta, omega), sync)
    _, t_lin1 = timed(lambda: op.set_linearization(state), sync)  # first call allocates the per-point store
    _, t_rot2 = timed(lambda: op.rotate_rotor(theta, omega), sync)
    _, t_lin = timed(lambda: op.set_linearization(state), sync)
    rec["rotate_rotor_first_ms"] = 1e3 * t_rot
    rec["rotate_rotor_ms"] = 1e3 * t_rot2
    rec["set_linearization_first_ms"] = 1e3 * t_lin1
    rec["set_linearization_ms"] = 1e3 * t_lin

    def run(src, dst, steps, warmup):
        """Timed region: `steps` back-to-back applications bracketed by device
        synchronization and by two HIP events on the launch stream (no events
        between the kernels).  A second pass of the same length records HIP
        events around every kernel class on the launch stream, for the
        per-kernel durations."""
        for _ in range(warmup):
            op.apply_jacobian(src, dst)
        sync()
        # HIP events on the launch stream (torch's current stream, which the
        # binding hands to the library) bracket the timed region
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            op.apply_jacobian(src, dst)
        e1.record()
        sync()
        ms = e0.elapsed_time(e1) / steps
        op.enable_timing(steps)
        for _ in range(steps):
            op.apply_jacobian(src, dst)
        sync()
        t = op.read_timing()
        op.enable_timing(0)
        return ms, t

    ms64, t64 = run(x64, y64, args.steps, args.warmup)
    ms32, t32 = run(x32, y32, args.steps, args.warmup)

    def distribution(src, dst, calls):
        """Per-call FP64 vmult times (events around each call): median, p10, p90."""
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
        sync()
        for a, b in ev:
            a.record()
            op.apply_jacobian(src, dst)
            b.record()
        sync()
        t = sorted(a.elapsed_time(b) for a, b in ev)
        return {"median_ms": t[len(t) // 2], "p10_ms": t[len(t) // 10], "p90_ms": t[(9 * len(t)) // 10],
                "calls": calls}

    rec["fp64_per_call"] = distribution(x64, y64, max(args.steps, 20))
    sync()
    err32 = float((y32.double() - y64).abs().max() / y64.abs().max())
    _, t_diag = timed(lambda: op.compute_diagonal(torch.float64), sync)
    rec["diagonal_ms"] = 1e3 * t_diag

    vol_ms64 = t64["ms_volume"] / max(1, t64["n_volume"])
    vol_ms32 = t32["ms_volume"] / max(1, t32["n_volume"])
    bytes64, cells = algorithmic_bytes_volume(mesh, n, 8)
    bytes32, _ = algorithmic_bytes_volume(mesh, n, 4)
    # headline roofline: the whole FP64 vmult (every launch of one
    # application: volume + mortar, gather) against the algorithmic bytes of
    # the application, over its event-timed duration per call
    achieved = bytes64 / (ms64 * 1e-3) / 1e9
    kname = dominant_kernel(mesh, args.fused, args.volume_layout)
    tb, tk = measured_traffic(name, kname)
    traffic = None if tb is None else tb / (ms64 * 1e-3) / 1e9
    # the dominant launch alone: the same algorithmic bytes over its own
    # duration (it does not write the result vector: the gather launch does)
    achieved_kernel = bytes64 / (vol_ms64 * 1e-3) / 1e9
    copy_gbs = None if args.no_copy_bandwidth else copy_bandwidth(dev, sync)
    # the practical ceiling: the library's own read-dominated stream kernel
    # (2 GiB read, 1/6 of it written, as the Jacobian's read:write mix)
    stream_gbs = None if args.no_copy_bandwidth else binding.stream_bandwidth(1 << 31, 6, 20)
    valu = None
    if "_quad" in kname and mesh["dim"] == 3 and mesh["degree"] == 2:
        tflops = QUAD_Q2_FLOP_PER_CELL * cells / (vol_ms64 * 1e-3) / 1e12
        alg = 0.75 * tflops  # without the fourth lane of each quad, which repeats the third
        valu = {"fp64_flop_per_cell_executed": QUAD_Q2_FLOP_PER_CELL, "executed_TFLOPs": tflops,
                "algorithmic_TFLOPs": alg, "peak_TFLOPs": FP64_PEAK_TFLOPS, "frac": alg / FP64_PEAK_TFLOPS,
                "frac_executed": tflops / FP64_PEAK_TFLOPS,
                "note": "FP64 VALU flops of the volume part (counters) over the dominant launch's time; "
                        "frac counts three of the four lanes of each cell (the fourth duplicates the third)"}
    rec["fp64"] = {"ms_per_vmult": ms64, "dofs_per_s": n / (ms64 * 1e-3), "volume_kernel_ms": vol_ms64,
                   "mortar_kernel_ms": t64["ms_mortar"] / max(1, t64["n_mortar"]),
                   "other_kernels_ms": t64["ms_other"] / max(1, t64["n_volume"])}
    rec["fp32"] = {"ms_per_vmult": ms32, "dofs_per_s": n / (ms32 * 1e-3), "volume_kernel_ms": vol_ms32,
                   "mortar_kernel_ms": t32["ms_mortar"] / max(1, t32["n_mortar"]),
                   "algorithmic_GBs": bytes32 / (vol_ms32 * 1e-3) / 1e9,
                   "rel_maxnorm_err_vs_fp64": err32}

    # FGMRES(FP64) solve to 1e-8: plain (FP64 Chebyshev) vs mixed (FP32 Chebyshev)
    if not args.no_solve and mesh["degree"] == 3:
        rec["solve"] = degree3_solve_leg(args, mesh, name, theta, omega, dev, sync)
    elif not args.no_solve:
        sstate = inputs.smooth_field(mesh, inputs.STATE_SEED[name])
        sstate /= np.abs(sstate).max()
        op.set_linearization(torch.from_numpy(sstate).to(dev))
        xstar = torch.from_numpy(inputs.uniform(n, inputs.SOLUTION_SEED[name])).to(dev)
        rhs = op.apply_jacobian(xstar)
        solves = {}
        for label, prec in (("plain_fp64", "f64"), ("mixed_fp32", "f32")):
            xs = torch.zeros_like(rhs)
            sync()
            _, info = op.solve(rhs, xs, check=False, rtol=1e-8, restart=args.solve_restart,
                               maxit=args.solve_maxit, precond=prec, cheb_degree=args.cheb_degree)
            chk = op.apply_jacobian(xs)
            sync()
            true_rel = float((rhs - chk).norm() / rhs.norm())
            solves[label] = {"seconds": info["seconds"], "iterations": info["iterations"],
                             "converged": info["rc"] == 0, "true_rel_residual": true_rel,
                             "vmults_f64": info["vmults_f64"], "vmults_f32": info["vmults_f32"],
                             "lambda_max": info["lambda_max"]}
        p, m = solves["plain_fp64"], solves["mixed_fp32"]
        solves["speedup_mixed_over_plain"] = (p["seconds"] / m["seconds"]) if m["seconds"] > 0 else None
        solves["state"] = "smooth manufactured field scaled to max |u| = 1"
        solves["preconditioner"] = f"Jacobi-Chebyshev degree {args.cheb_degree}, FGMRES({args.solve_restart})"
        if mesh["degree"] == 2:
            # the same solves with the multigrid V-cycle (Picard levels); one
            # untimed solve builds and linearizes the hierarchy first
            mgo = dict(rtol=1e-8, restart=60, maxit=args.solve_maxit, mg_coarse_linearization="picard",
                       mg_fine_linearization="picard", mg_smooth_degree=3, mg_smooth_range=10.0)
            op.solve(rhs, torch.zeros_like(rhs), check=False, precond="mg", **dict(mgo, maxit=1))
            mg = {}
            for label, prec in (("plain_fp64", "mg64"), ("mixed_fp32", "mg")):
                xs = torch.zeros_like(rhs)
                sync()
                _, info = op.solve(rhs, xs, check=False, precond=prec, **mgo)
                chk = op.apply_jacobian(xs)
                sync()
                mg[label] = {"seconds": info["seconds"], "iterations": info["iterations"],
                             "converged": info["rc"] == 0, "true_rel_residual": float((rhs - chk).norm() / rhs.norm())}
            mg["speedup_mixed_over_plain"] = (mg["plain_fp64"]["seconds"] / mg["mixed_fp32"]["seconds"]
                                              if mg["mixed_fp32"]["seconds"] > 0 else None)
            mg["levels"] = op.mg_levels()
            mg["preconditioner"] = ("geometric multigrid V-cycle, Picard-linearized levels, Jacobi-Chebyshev smoothing "
                                    "degree 3 on [1.05 lambda/10, 1.05 lambda] in FP32 (mixed) or FP64 (plain), FGMRES(60)")
            solves["multigrid"] = mg
        rec["solve"] = solves

    # linearization source C next to B (the timed region above used B)
    op.set_linearization(state)
    if has_source_c(mesh):
        rec["lin_source_c"] = source_c_leg(op, mesh, x64, sync, max(args.steps // 2, 10))
    # launch configuration chosen by the library's autotuner on this mesh
    # (the timed region above used the automatic default)
    default_cfg = op.get_kernel_config()
    chosen = op.autotune_kernel_config(20)
    ms_tuned, _ = run(x64, y64, max(args.steps // 2, 10), 3)
    rec["autotune"] = {"default": default_cfg, "chosen": chosen, "ms_per_vmult_chosen": ms_tuned}
    op.set_kernel_config(**default_cfg)

    # the volume kernel on its own (separate launches, fused_launch = 0): its
    # roofline without the mortar blocks that share the fused launch
    if mesh["dim"] == 3 and args.fused < 0:
        op.set_kernel_config(fused_launch=0, volume_layout=args.volume_layout)
        ms_sep, t_sep = run(x64, y64, args.steps, min(args.warmup, 20))
        op.set_kernel_config(**default_cfg)
        vol_sep = t_sep["ms_volume"] / max(1, t_sep["n_volume"])
        ach_sep = bytes64 / (vol_sep * 1e-3) / 1e9
        rec["separate_volume_launch"] = {
            "kernel": dominant_kernel(mesh, 0, args.volume_layout), "ms_per_vmult": ms_sep, "kernel_ms": vol_sep,
            "achieved_GBs": ach_sep, "frac_of_8TBs": ach_sep / HBM_PEAK_GBS,
            "frac_of_measured_copy": ach_sep / copy_gbs if copy_gbs else None,
            "mortar_kernel_ms": t_sep["ms_mortar"] / max(1, t_sep["n_mortar"])}

    if not args.no_iso and mesh["dim"] == 3:
        rec["iso_parametric"] = iso_leg(name, dev, sync, max(args.steps, 20), min(args.warmup, 10))

    if not args.no_batch:
        rec["batch"] = batch_leg(args, dev, sync)

    if not args.no_large and name == "annulus3d_q2_64x8x32":
        # free the 1.1M-DoF handle's Krylov workspace first
        rec["large_workloads"] = large_workloads_leg(args, dev, sync)

    if args.transient and not mesh.get("steady", 1):
        # two implicit time steps of a spin-up: fluid at rest, a smooth body
        # force (the smooth field, max 1) switched on, the rotor advancing by
        # omega dt per step; the second step is timed
        dt = mesh["dt"]
        force = torch.from_numpy(inputs.transient_start(mesh, inputs.STATE_SEED[name])).to(dev)
        u0 = torch.zeros_like(force)
        u1 = u0.clone()
        lin_opts = dict(rtol=1e-6, restart=30, maxit=600, precond="mg")
        op.bdf2_step(theta + omega * dt, omega, u0, u1, u_nm1=None, force=force, newton_rtol=1e-8, max_newton=10,
                     linear=lin_opts)
        steps = {}
        for label, prec in (("mixed_fp32_multigrid", "mg"), ("plain_fp64_multigrid", "mg64")):
            u = u1.clone()
            sync()
            info = op.bdf2_step(theta + 2 * omega * dt, omega, u1, u, u_nm1=u0, force=force, check=False,
                                newton_rtol=1e-8, max_newton=10, linear=dict(lin_opts, precond=prec))
            steps[label] = {"seconds": info["seconds"], "newton_iterations": info["newton_iterations"],
                            "linear_iterations": info["linear_iterations"], "converged": info["rc"] == 0,
                            "residual0": info["residual0"], "residual": info["residual"],
                            "line_search_halvings": info["line_search_halvings"]}
        m_, p_ = steps["mixed_fp32_multigrid"], steps["plain_fp64_multigrid"]
        rec["transient_step"] = {
            **steps, "speedup_mixed_over_plain": p_["seconds"] / m_["seconds"] if m_["seconds"] > 0 else None,
            "dt": dt, "rotation_rad": omega * dt,
            "scenario": "spin-up from rest under a smooth body force; second BDF2 step timed",
            "newton_rtol": 1e-8,
            "linear": "FGMRES(30) FP64 to 1e-6, geometric multigrid V-cycle, Jacobi-Chebyshev smoothing in FP32 (mixed) "
                      "or FP64 (plain)",
        }
        del force, u0, u1, u

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        ocfg = oracle.params(**{k: mesh[k] for k in ("dim", "degree", "r_in", "r_if", "r_out", "height",
                                                    "n_theta", "n_r_rotor", "n_r_stator", "n_z", "nu",
                                                    "steady", "dt")}, theta_rot=theta, omega=omega)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        reps, t_cpu, yo = 0, 0.0, None
        while t_cpu < args.cpu_seconds and reps < 50:
            t0 = time.perf_counter()
            yo = oracle.apply_jacobian(ocfg, state_np, x_np)
            t_cpu += time.perf_counter() - t0
            reps += 1
        cpu = {"value": n * reps / t_cpu, "unit": "DoFs/s", "cores": threads, "kind": "oracle",
               "sample": f"{reps} full FP64 Jacobian applications of {name} ({n} DoFs) by the C oracle "
                         f"(element by element, full basis tables, OpenMP over 8 cell colours)"}
        rec["fp64"]["rel_maxnorm_err_vs_oracle"] = float(np.abs(y64.cpu().numpy() - yo).max() / np.abs(yo).max())

    line = {
        "metric": METRIC,
        "value": n / (ms64 * 1e-3),
        "unit": "DoFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms64,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": name, "dofs": n, "cells": cells, "degree": mesh["degree"], "dim": mesh["dim"],
                   "rotor_angle": theta, "nu": mesh["nu"], "step": "one FP64 Jacobian application"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_bytes_per_call": tb, "traffic_source": f"profiles/traffic_{name}.txt" if tb else None,
                     "kernel": f"whole FP64 vmult ({kname} + gather)", "kernel_ms": ms64,
                     "algorithmic_bytes_per_launch": bytes64,
                     "measured_stream_GBs": stream_gbs,
                     "frac_of_measured_stream": achieved / stream_gbs if stream_gbs else None,
                     "measured_copy_GBs": copy_gbs, "frac_of_measured_copy": achieved / copy_gbs if copy_gbs else None,
                     "dominant_launch": {"kernel": kname, "kernel_ms": vol_ms64, "achieved_GBs": achieved_kernel,
                                         "frac_of_8TBs": achieved_kernel / HBM_PEAK_GBS,
                                         "traffic_bytes_per_launch": tk,
                                         "note": "the vmult's algorithmic bytes over this launch alone; "
                                                 "the result vector is written by the gather launch"},
                     "fp64_valu": valu},
        "cpu_baseline": cpu,
        "hot_path": rec,
    }
    op.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
