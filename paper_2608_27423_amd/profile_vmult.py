#!/usr/bin/env python3
"""Small driver for hardware-counter runs of the Jacobian vmult.

Run under a profiler, it first copies one 512 MiB buffer (the calibration
dispatch: 512 MiB read, 512 MiB written), then applies the FP64 (or FP32)
Jacobian of a named workload a few times.  The counter totals of the copy
dispatch give the scale from FETCH_SIZE / WRITE_SIZE to bytes.

    rocprofv3 --pmc FETCH_SIZE -f csv -d OUT -o p -- python paper_2608_27423_amd/profile_vmult.py \
        --workload annulus3d_q2_64x8x32

`--iso PERTURB` runs the workload on the curved mesh of
inputs.iso_node_positions (cells are the Q_k interpolants of their nodes).

`--summarize DIR_FETCH DIR_WRITE` reads the two counter CSV files and prints
the per-dispatch bytes of every kernel of the run (scaled by the copy); with
`--traffic-out FILE` it also writes the summary that bench.py reads: the
bytes of every kernel dispatched once per vmult (`--reps` dispatches) and
their sum per vmult, tagged with the digest of the kernel source.
"""
import argparse
import csv
import glob
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

COPY_BYTES = 1 << 29


def run(args):
    import torch

    from paper_2608_27423_amd import binding, inputs

    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    name = args.workload
    mesh = inputs.mesh(name)
    dtype = torch.float64 if args.precision == "f64" else torch.float32
    state = torch.from_numpy(inputs.state_for(name)).cuda()
    x = torch.from_numpy(inputs.vector_for(name)).cuda().to(dtype)
    with binding.Operator(mesh) as op:
        op.set_kernel_config(fused_launch=args.fused, volume_layout=args.volume_layout,
                             lin_source_f64=args.lin_source, lin_source_f32=args.lin_source)
        if args.iso is not None:
            op.set_node_positions(inputs.iso_node_positions(mesh, args.iso))
        op.rotate_rotor(inputs.rotor_angle(name), mesh["omega"])
        op.set_linearization(state)
        y = torch.empty_like(x)
        for _ in range(args.reps):
            op.apply_jacobian(x, y)
        torch.cuda.synchronize()
    print(f"done: {args.reps} vmults of {name} ({args.precision})", flush=True)


def _totals(path):
    """{dispatch: (kernel, counter, value)} summed over the counter's instances."""
    out = {}
    for f in glob.glob(os.path.join(path, "*counter_collection.csv")):
        for r in csv.DictReader(open(f)):
            key = int(r["Dispatch_Id"])
            k, c, v = r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])
            if key in out:
                out[key] = (k, c, out[key][2] + v)
            else:
                out[key] = (k, c, v)
    return out


def summarize(dfetch, dwrite, traffic_out=None, reps=3, workload=""):
    f, w = _totals(dfetch), _totals(dwrite)
    copy_f = [v for k, c, v in f.values() if "copyBuffer" in k and v > 1e5]
    copy_w = [v for k, c, v in w.values() if "copyBuffer" in k and v > 1e5]
    if not copy_f or not copy_w:
        raise SystemExit("calibration copy dispatch not found")
    sf = COPY_BYTES / (copy_f[0] * 1024.0)
    sw = COPY_BYTES / (copy_w[0] * 1024.0)
    print(f"calibration: FETCH_SIZE {copy_f[0]:.0f} KiB and WRITE_SIZE {copy_w[0]:.0f} KiB for a "
          f"{COPY_BYTES >> 20} MiB copy -> scale {sf:.4f} (fetch), {sw:.4f} (write)")
    per = {}
    for d in sorted(set(f) & set(w)):
        k = f[d][0]
        if "copyBuffer" in k or "elementwise" in k:
            continue
        short = k.split("(")[0].replace("void ", "")
        per.setdefault(short, []).append((f[d][2] * 1024 * sf, w[d][2] * 1024 * sw))
    print("| kernel | dispatches | read MB / dispatch | write MB / dispatch | total MB / dispatch |")
    print("|---|---|---|---|---|")
    rows = []
    for k, v in per.items():
        rd = sum(a for a, _ in v) / len(v)
        wr = sum(b for _, b in v) / len(v)
        rows.append((k, len(v), rd, wr))
        print(f"| `{k}` | {len(v)} | {rd / 1e6:.2f} | {wr / 1e6:.2f} | {(rd + wr) / 1e6:.2f} |")
    if traffic_out:
        import hashlib

        src = os.path.join(HERE, "csrc", "mns_kernels.hip")
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        vm = [r for r in rows if r[1] % reps == 0 and r[1] // reps >= 1 and "k_state" not in r[0]
              and "k_cast" not in r[0] and "k_rotate" not in r[0] and "k_iso_" not in r[0]]
        with open(traffic_out, "w") as f:
            f.write(f"# HBM bytes of the FP64 vmult kernels, {workload} (read by bench.py); FETCH_SIZE and\n"
                    f"# WRITE_SIZE passes of profile_vmult.py, scaled by the {COPY_BYTES >> 20} MiB copy "
                    f"calibration (fetch x {sf:.4f}, write x {sw:.4f})\n")
            f.write(f"kernel_source_sha256: {digest}\n")
            tot_r = tot_w = 0.0
            for k, cnt, rd, wr in vm:
                per_call = cnt // reps
                tot_r += per_call * rd
                tot_w += per_call * wr
                f.write(f"bytes_per_launch {k}: {rd + wr:.0f}\n")
                f.write(f"read_write_per_launch {k}: {rd:.0f} {wr:.0f}\n")
            f.write(f"vmult_read_bytes_per_call: {tot_r:.0f}\n")
            f.write(f"vmult_write_bytes_per_call: {tot_w:.0f}\n")
            f.write(f"vmult_bytes_per_call: {tot_r + tot_w:.0f}\n")
        print(f"wrote {traffic_out}")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", default="annulus3d_q2_64x8x32")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--fused", type=int, default=-1)
    ap.add_argument("--volume-layout", type=int, default=1)
    ap.add_argument("--lin-source", type=int, default=0, choices=[0, 1],
                    help="linearization source of the quad volume kernels: 0 = B (full per-point store), "
                         "1 = C (tau and tau R per point, a and grad u from the state)")
    ap.add_argument("--iso", type=float, default=None, metavar="PERTURB",
                    help="curved mesh: inputs.iso_node_positions with this interior displacement (in cells)")
    ap.add_argument("--summarize", nargs=2, metavar=("DIR_FETCH", "DIR_WRITE"))
    ap.add_argument("--traffic-out", default=None)
    args = ap.parse_args()
    if args.summarize:
        summarize(*args.summarize, traffic_out=args.traffic_out, reps=args.reps, workload=args.workload)
    else:
        run(args)


if __name__ == "__main__":
    main()
