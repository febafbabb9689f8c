"""Benchmark of the polyenergetic cone-beam projector on one MI355X.

A step is one fcat_project call over the whole contrast-phantom workload:
1024x1024x10 labelled voxels (0.15625 mm, 8 materials), 200 energy bins
(0.01-6 MeV), 1024x64 detector at 0.392 mm, 360 angles, per-angle scatter
maps and 8 energy-group 15x15 optical spread kernels.  Inputs are seeded
synthetic stand-ins, resident in HBM before timing starts.

Prints one JSON line: rays x energy-bins per second, the roofline of the
dominant kernel (timed live with HIP events on the library's stream), HBM
GB/s of the compulsory traffic, and the FP64 oracle timed on the host on a
bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_HBM_GBPS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="plain", choices=["plain", "split_bf16", "surrogate"])
    ap.add_argument("--cpu-angles", type=int, default=24,
                    help="angles of the workload the FP64 oracle is timed on (0: skip)")
    ap.add_argument("--variant", default="", help="'z' for the 1.5625 mm slab variant")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this projector benchmark runs on one GPU only; "
                                   "angles would be sharded across GPUs with no exchange "
                                   f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})"}))
        sys.exit(2)

    import torch
    import paper_2011_04736_amd as fc
    import synth

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    cfg = synth.make_config(2, variant=args.variant)
    g, s = cfg.geometry, cfg.spectral
    pb = fc.upload(cfg, device=dev)
    out = torch.empty((g.n_angles, g.nv, g.nu), dtype=torch.float32, device=dev)
    ws_bytes = fc.fcat_project_workspace_bytes(pb, args.mode)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        fc.fcat_project(pb, mode=args.mode, out=out, workspace=ws, stream=stream)
    torch.cuda.synchronize()

    fc.fcat_timing_enable(True)
    fc.fcat_timing_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fc.fcat_project(pb, mode=args.mode, out=out, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = fc.fcat_timing_read(reset=True)
    fc.fcat_timing_enable(False)

    rays = g.n_angles * g.nu * g.nv
    ray_e = rays * s.n_energy
    ms_per_step = 1e3 * elapsed / args.steps
    value = ray_e * args.steps / elapsed

    # dominant kernel and its roofline
    G, K = s.n_groups, cfg.psf.k
    dominant = max(("trace", "psf"), key=lambda k: stages[k][0])
    psf_ms, psf_n = stages["psf"]
    trace_ms, trace_n = stages["trace"]
    psf_flops_total = 2.0 * G * K * K * rays * args.steps
    roof = {
        "kernel": "k_psf (optical spread + group sum)" if dominant == "psf" else "k_project_rows (traversal + spectral)",
        "bound": "alu",
        "unit": "TFLOP/s",
        "peak": PEAK_FP32_VECTOR_TFLOPS,
        "traffic": None,
    }
    if dominant == "psf":
        ach = psf_flops_total / (psf_ms * 1e-3) / 1e12
        roof.update(achieved=round(ach, 3), frac=round(ach / PEAK_FP32_VECTOR_TFLOPS, 4),
                    avg_launch_ms=round(psf_ms / max(psf_n, 1), 4), launches=psf_n)
    else:
        roof.update(achieved=None, frac=None, avg_launch_ms=round(trace_ms / max(trace_n, 1), 4),
                    launches=trace_n)

    # compulsory HBM traffic per step: labels + scatter maps in, projections out
    comp_bytes = cfg.phantom.labels.size + 2 * rays * 4
    hbm = comp_bytes / (ms_per_step * 1e-3) / 1e9

    result = {
        "metric": "rays*energy_bins/s",
        "value": value,
        "unit": "ray*E/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded stand-in for the Catphan-like contrast phantom, MV spectrum, scatter and OSFs)",
        "config": {
            "workload": "contrast phantom 1024x1024x10 @0.15625 mm, 8 materials, 200 bins 0.01-6 MeV, "
                        "1024x64 detector @0.392 mm, 360 angles, scatter + 8 groups 15x15 PSF"
                        + (" (dz=1.5625 variant)" if args.variant == "z" else ""),
            "mode": args.mode,
            "rays": rays,
            "energy_bins": s.n_energy,
        },
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items() if v[1]},
        "hbm_compulsory_GBps": round(hbm, 2),
        "roofline": roof,
    }

    if args.cpu_angles > 0:
        result["cpu_baseline"] = cpu_baseline(cfg, args.cpu_angles, ray_e / g.n_angles)

    print(json.dumps(result))


def cpu_baseline(cfg, n_angles: int, ray_e_per_angle: float) -> dict:
    """The FP64 oracle on an evenly spaced sample of the workload's angles."""
    import oracle
    A = cfg.geometry.n_angles
    angles = np.unique(np.linspace(0, A - 1, n_angles).round().astype(int))
    S = cfg.scatter.maps(angles)
    t0 = time.perf_counter()
    oracle.project(cfg, angles, scatter_maps=S)
    dt = time.perf_counter() - t0
    return {"value": len(angles) * ray_e_per_angle / dt, "unit": "ray*E/s", "cores": oracle.max_threads(),
            "kind": "oracle", "seconds": round(dt, 2),
            "sample": f"{len(angles)} of {A} angles (evenly spaced), full detector, all bins, scatter and PSF"}


if __name__ == "__main__":
    main()
