"""Benchmark of the polyenergetic cone-beam projector on one MI355X.

A step is one fcat_project call over the whole head workload, the largest
single-GPU configuration: 512x512x256 labelled voxels (0.5 mm, 10
materials), a 120 kVp spectrum in 120 bins of 1 keV, a 1024x768 detector at
0.4 mm, 720 angles, per-angle scatter maps and 8 energy-group 15x15 optical
spread kernels.  Inputs are seeded synthetic stand-ins, resident in HBM
before timing starts.

Prints one JSON line: rays x energy-bins per second of the plain FP32 form on
that workload, the roofline of its dominant kernel (timed live with HIP
events on the library's stream) priced by two work units (the Siddon voxel
segments of the method and the steps the walk actually takes, both counted
on the GPU by fcat_walk_stats), the FP64 oracle timed on the host on 16 of
the 720 angles; then the contrast phantom and its thick-slab variant as
secondary workloads, the other two forms of the projector (BF16 hi/lo split
on the matrix cores; the learned surrogate trained here by the library's own
kernels) with their errors against the plain form and their rooflines, the
stages after the projector on the contrast workload, the device-ceiling
microbenchmark, and the oracle's single-thread time on the tiny case.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks.
PEAK_FP32_VECTOR_TFLOPS = 157.3               # FP32 vector, counted with packed FMA (2 FP32 FMAs per lane per cycle)
PEAK_BF16_MFMA_TFLOPS = 2500.0                # dense BF16 matrix
PEAK_HBM_GBPS = 8000.0
# Lane-operation peak for plain-ALU rows: the published FP32 rate in FMAs,
# 157.3e12 FLOP/s / 2 FLOP per FMA = 78.65e12 lane-operations/s.  That rate
# assumes packed FP32, which this library never emits; one unpacked vector
# instruction per SIMD per cycle over 16 lanes gives 256 CUs x 4 SIMDs x 16 x
# 2.4 GHz = 39.32e12, reported beside it.
PEAK_LANE_OPS = PEAK_FP32_VECTOR_TFLOPS * 1e12 / 2
SINGLE_ISSUE_LANE_OPS = 256 * 4 * 16 * 2.4e9
PEAK_NOTE = ("peak: published FP32 157.3 TFLOP/s / 2 FLOP per FMA = 78.65e12 lane-ops/s (packed issue); "
             "peak_single_issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.32e12")

# Algorithmic work per unit (vector lane-operations).
OPS_PER_SEGMENT = 12          # one voxel segment of the incremental Siddon walk: next crossing as the
                              # min of three, segment length, accumulation, advance of one axis's crossing
                              # and index, label address and load, exit test
EXP_SLOTS = 4                 # lane-operations counted for the dose sum's 1 - exp(-P) (a half-rate exp2 plus its
                              # argument reduction)
EXP2_SLOTS = 2                # the spectral sum's exponential: one hardware exp2, half rate


EXECUTED_UNIT = (f"{OPS_PER_SEGMENT} lane-ops per walk step taken (brick steps + voxel steps in mixed bricks) "
                 f"+ the same spectral work")


def spectral_ops_per_bin(M: int) -> int:
    """Lane-operations of the spectral sum per hit ray and bin: M FMAs of the
    base-2 optical depth (mu log2 e tabulated), one exp2 at half rate and the
    weight FMA."""
    return M + 1 + EXP2_SLOTS

WORKLOADS = {
    "head": (3, "", "head phantom 512x512x256 @0.5 mm, 10 materials, 120 bins 1-120 keV, 1024x768 detector "
                    "@0.4 mm, 720 angles, scatter + 8 groups 15x15 PSF"),
    "contrast": (2, "", "contrast phantom 1024x1024x10 @0.15625 mm, 8 materials, 200 bins 0.01-6 MeV, "
                        "1024x64 detector @0.392 mm, 360 angles, scatter + 8 groups 15x15 PSF"),
    "contrast_dz": (2, "z", "contrast phantom 1024x1024x10 @0.15625 x 0.15625 x 1.5625 mm (thick-slab variant), "
                            "8 materials, 200 bins 0.01-6 MeV, 1024x64 detector @0.392 mm, 360 angles, scatter + "
                            "8 groups 15x15 PSF"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="head", choices=sorted(WORKLOADS),
                    help="the headline workload (default: the largest, head)")
    ap.add_argument("--secondary", default="contrast,contrast_dz",
                    help="comma list of further workloads timed in the plain form ('' for none)")
    ap.add_argument("--secondary-steps", type=int, default=10)
    ap.add_argument("--cpu-angles", type=int, default=16,
                    help="angles of the headline workload the FP64 oracle is timed on (0: skip)")
    ap.add_argument("--tiny-oracle", type=int, default=1, help="1: time the oracle single-threaded on the tiny case")
    ap.add_argument("--noise-counts", type=float, default=1.0e5,
                    help="H of Eq. 5 (flood counts per open pixel) for the noise stage; 0 skips it")
    ap.add_argument("--dose", type=int, default=1, help="1: time the dose estimate of Eqs. 6-7 (0 skips it)")
    ap.add_argument("--fdk", type=int, default=1, help="1: time the FDK reconstruction of the projections (0 skips it)")
    ap.add_argument("--image-projector", type=int, default=1,
                    help="1: time the image projector and its transpose on the contrast grid (0 skips them)")
    ap.add_argument("--rl-iterations", type=int, default=10,
                    help="Richardson-Lucy iterations on the detected profiles (0 skips the optics stage)")
    ap.add_argument("--spectral", type=int, default=1, help="1: time steps a3-a4 alone on the hit rays' path lengths")
    ap.add_argument("--ceilings", type=int, default=1,
                    help="1: run the device-ceiling microbenchmark and add fractions of the measured ceilings")
    ap.add_argument("--forms", default="split_bf16,surrogate",
                    help="comma list of extra forms to measure beside the plain one ('' for none)")
    ap.add_argument("--form-steps", type=int, default=3, help="timed steps of the extra forms and stages")
    ap.add_argument("--surrogate-samples", type=int, default=4_000_000)
    ap.add_argument("--surrogate-epochs", type=int, default=120)
    ap.add_argument("--surrogate-fine", type=int, default=8,
                    help="also time plain and surrogate projectors on the head spectrum cut into this many times "
                         "finer bins (0 or 1 skips)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this size first (scale reference for HBM counters)")
    return ap.parse_args()


# -------------------------------------------------------------- traffic

def source_digest(files) -> str:
    hsh = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2011_04736_amd", "csrc", f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()[:16]


TRACE_SOURCES = ["fcat_kernels.hip", "fcat_device.h", "fcat_internal.h"]
SPLIT_SOURCES = ["fcat_split.hip", "fcat_device.h", "fcat_internal.h"]
NOISE_SOURCES = ["fcat_noise.hip", "fcat_internal.h"]
DOSE_SOURCES = ["fcat_dose.hip", "fcat_internal.h"]
FDK_SOURCES = ["fcat_fdk.hip", "fcat_recon.h"]
BP_OPS_PER_VOXEL_ANGLE = 10   # axial position 1, floor and fraction 2, four-tap bilinear 6, weighted add 1


def profiled_traffic(kernel: str, digest: str, workload: str = "contrast"):
    """HBM bytes per step (all launches of the kernel in one step) of ``kernel``
    from the committed counter summary of the workload, or None when the
    summary is missing or was taken on other sources."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^sources:\s*(\S+)", text, re.M)
    t = re.search(r"^traffic_bytes_per_step:\s*(\S+)", text, re.M) or \
        re.search(r"^traffic_bytes_per_launch:\s*(\S+)", text, re.M)
    if not m or not t or m.group(1) != digest:
        return None
    return float(t.group(1))


def profiled_counters(kernel: str, digest: str, workload: str) -> dict:
    """Derived counter figures (issue rate, MFMA busy, L2 hit ...) of ``kernel``
    from the committed counter summary of the workload, if it was taken on
    the current sources."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.txt")
    if not os.path.exists(path):
        return {}
    text = open(path).read()
    for b in re.split(r"\n(?=\S)", text):
        # the kernel's block: its name, then a template list, a space or an argument list
        if re.match(re.escape(kernel) + r"[<\s(]", b):
            m = re.search(r"^\s*sources:\s*(\S+)", b, re.M)
            if not m or m.group(1) != digest:
                return {}
            out = {}
            for key, name in (("VALU issue rate", "valu_issue_vs_16_lane_rate"), ("MFMA busy", "mfma_busy"),
                              ("L2 hit rate", "l2_hit"), ("LDS bank-conflict share", "lds_bank_conflict_share"),
                              ("wait share of wave cycles", "wait_share"),
                              ("ACTIVE_INST_VALU2 / VALU", "valu2_share"),
                              ("VALU lane-slots per segment", "valu_lane_slots_per_segment")):
                mm = re.search(rf"^\s+{re.escape(key)}\s+([0-9.eE+-]+)", b, re.M)
                if mm:
                    out[name] = float(mm.group(1))
            return out
    return {}


def alu_roof(kernel: str, ops: float, ms: float, launches: float = 1, **extra) -> dict:
    """Roofline entry of a plain-ALU kernel: ``ops`` algorithmic lane-operations
    per step in ``ms`` per step over ``launches`` launches."""
    ach = ops / (ms * 1e-3)
    e = {"kernel": kernel, "bound": "alu", "achieved": round(ach / 1e12, 3), "peak": round(PEAK_LANE_OPS / 1e12, 2),
         "unit": "Top/s", "frac": round(ach / PEAK_LANE_OPS, 4),
         "peak_single_issue": round(SINGLE_ISSUE_LANE_OPS / 1e12, 2),
         "frac_single_issue": round(ach / SINGLE_ISSUE_LANE_OPS, 4),
         "stage_ms_per_step": round(ms, 4), "launches_per_step": launches,
         "avg_launch_ms": round(ms / max(launches, 1), 4), "algorithmic_ops_per_step": ops}
    e.update(extra)
    return e


# ----------------------------------------------------------------- forms

def optics_stage(pb, cfg, args, torch, fc):
    """Effective PSF and its presampled MTF from a 0.3 mm slit tilted by 2.5
    degrees (Sec. II.B), then Richardson-Lucy deconvolution of the workload's
    360 detected profiles with it (two 15 x 15 convolutions per iteration)."""
    g = cfg.geometry
    out = fc.fcat_project(pb)
    K = fc.fcat_effective_psf(pb.spectral, pb.psf)
    freqs = np.linspace(0.0, 1.0 / g.du, 65)
    mtf, _, _, _ = fc.fcat_slit_mtf(K, g.du, 0.3, 2.5, 256, 64, 10, freqs)
    m = mtf.cpu().numpy()
    f50 = float(np.interp(0.5, m[::-1], freqs[::-1])) if m.min() < 0.5 else None
    k = int(K.shape[0])
    ws = torch.empty(fc.fcat_richardson_lucy_workspace_bytes(g.n_angles, g.nv, g.nu, k), dtype=torch.uint8,
                     device=out.device)
    dec = torch.empty_like(out)
    stream = torch.cuda.current_stream()
    elapsed, stages = timed_steps(lambda: fc.fcat_richardson_lucy(out, K, args.rl_iterations, out=dec, workspace=ws,
                                                                  stream=stream), 1, args.form_steps, torch)
    psf_ms = stages["psf"][0] / args.form_steps
    flops = 2.0 * 2 * k * k * g.n_angles * g.nv * g.nu * args.rl_iterations
    ach = flops / (psf_ms * 1e-3) / 1e12
    finite = bool(torch.isfinite(dec).all().item())
    del ws, dec, out
    return {
        "ms_per_step": round(1e3 * elapsed / args.form_steps, 4),
        "steps": args.form_steps,
        "iterations": args.rl_iterations,
        "stages_ms_per_step": {kk: round(v[0] / args.form_steps, 4) for kk, v in stages.items() if v[1]},
        "mtf50_per_mm": f50,
        "finite": finite,
        "roofline": {"kernel": "k_psf4<15,8> (one group)", "bound": "alu", "achieved": round(ach, 3),
                     "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_VECTOR_TFLOPS, 4),
                     "stage_ms": round(psf_ms, 4), "algorithmic_flops_per_step": flops, "traffic": None},
    }


# v_exp_f32 issues at half the 16-lane rate (measured by the ceiling probe)
EXP_RATE = SINGLE_ISSUE_LANE_OPS / 2


def spectral_stage(pb, cfg, args, torch, fc):
    """Steps a3-a4 on their own: the exact spectral sum (Eq. 3) over the
    path lengths of the workload's rays that meet the phantom, timed as
    k_spectral (E exps and E (M + 1) FMAs per ray)."""
    s = cfg.spectral
    M, E = s.n_mat, s.n_energy
    L = fc.fcat_pathlengths(pb, M).reshape(-1, M)
    Lh = L[L.sum(dim=1) > 0].contiguous()
    del L
    n = int(Lh.shape[0])
    Y = torch.empty((s.n_groups, n), dtype=torch.float32, device=Lh.device)
    ws = torch.empty(max(fc.fcat_spectral_workspace_bytes(pb.spectral), 1), dtype=torch.uint8, device=Lh.device)
    stream = torch.cuda.current_stream()
    elapsed, stages = timed_steps(lambda: fc.fcat_spectral(Lh, pb.spectral, out=Y, workspace=ws, stream=stream),
                                  1, args.form_steps, torch)
    t = stages["trace"][0] / args.form_steps
    exps = float(n) * E
    ops = exps * spectral_ops_per_bin(M)
    ach = ops / (t * 1e-3)
    del Lh, Y, ws
    return {
        "rays": n,
        "energy_bins": E,
        "ms": round(t, 4),
        "exp_per_s": exps / (t * 1e-3),
        "exp_rate_frac": round(exps / (t * 1e-3) / EXP_RATE, 4),
        "roofline": {"kernel": "k_spectral", "bound": "alu", "achieved": round(ach / 1e12, 3),
                     "peak": round(PEAK_LANE_OPS / 1e12, 2), "unit": "Top/s", "frac": round(ach / PEAK_LANE_OPS, 4),
                     "frac_single_issue": round(ach / SINGLE_ISSUE_LANE_OPS, 4),
                     "note": "per hit ray and bin M FMAs, the weight FMA and an exp2 counted as "
                             "EXP2_SLOTS lane-operations; the exp unit itself is far from busy (exp_rate_frac)"},
    }


def fdk_stage(pb, cfg, args, torch, fc):
    """FDK reconstruction of the workload's noiseless projections into the
    phantom's own grid (1024 x 1024 x 10): ramp filter (nu/2 FMAs per output,
    the even taps being zero) and back-projection (every voxel from every
    angle)."""
    import synth
    g, ph = cfg.geometry, cfg.phantom
    proj = fc.fcat_projections(pb, None)
    grid = synth.Grid(nx=ph.nx, ny=ph.ny, nz=ph.nz, dx=ph.dx, dy=ph.dy, dz=ph.dz)
    vol = torch.empty((grid.nz, grid.ny, grid.nx), dtype=torch.float32, device=proj.device)
    ws = torch.empty(fc.fcat_fdk_workspace_bytes(pb.geometry), dtype=torch.uint8, device=proj.device)
    stream = torch.cuda.current_stream()
    elapsed, stages = timed_steps(lambda: fc.fcat_fdk(pb.geometry, proj, grid, volume=vol, workspace=ws,
                                                      stream=stream), 1, args.form_steps, torch)
    bp_ms = stages["backproject"][0] / args.form_steps
    fl_ms = stages["filter"][0] / args.form_steps
    vox_ang = float(grid.nx) * grid.ny * grid.nz * g.n_angles
    bp_ops = BP_OPS_PER_VOXEL_ANGLE * vox_ang
    bp_ach = bp_ops / (bp_ms * 1e-3) / 1e12
    fl_flops = 2.0 * g.n_angles * g.nv * g.nu * ((g.nu + 1) // 2)
    fl_ach = fl_flops / (fl_ms * 1e-3) / 1e12
    # the sample quads: each padded plane read once, its quads written once
    su = max(g.nu, 2)
    ly_bytes = g.n_angles * (4.0 * (g.nv + 3) * su + 16.0 * (g.nv + 2) * (su - 1))
    ly_ms = stages["layout"][0] / args.form_steps
    finite = bool(torch.isfinite(vol).all().item())
    del ws, vol, proj
    return {
        "ms_per_step": round(1e3 * elapsed / args.form_steps, 4),
        "steps": args.form_steps,
        "grid": [grid.nx, grid.ny, grid.nz],
        "stages_ms_per_step": {k: round(v[0] / args.form_steps, 4) for k, v in stages.items() if v[1]},
        "voxel_angle_updates_per_s": vox_ang / (bp_ms * 1e-3),
        "finite": finite,
        "roofline": {"kernel": "k_fdk_backproject", "bound": "alu", "achieved": round(bp_ach, 3),
                     "peak": round(PEAK_LANE_OPS / 1e12, 2), "unit": "Top/s",
                     "frac": round(bp_ach * 1e12 / PEAK_LANE_OPS, 4),
                     "frac_single_issue": round(bp_ach * 1e12 / SINGLE_ISSUE_LANE_OPS, 4), "stage_ms": round(bp_ms, 4),
                     "algorithmic_ops_per_step": bp_ops,
                     "traffic": profiled_traffic("k_fdk_backproject", source_digest(FDK_SOURCES))},
        "filter": {"kernel": "k_fdk_filter", "bound": "alu", "achieved": round(fl_ach, 3),
                   "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                   "frac": round(fl_ach / PEAK_FP32_VECTOR_TFLOPS, 4), "stage_ms": round(fl_ms, 4),
                   "algorithmic_flops_per_step": fl_flops},
        "layout": {"kernel": "k_fdk_quads (+ k_fdk_pad)", "bound": "hbm",
                   "achieved": round(ly_bytes / (ly_ms * 1e-3) / 1e9, 2), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                   "frac": round(ly_bytes / (ly_ms * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4), "stage_ms": round(ly_ms, 4),
                   "algorithmic_bytes_per_step": ly_bytes},
    }


def image_projector_stage(pb, cfg, args, torch, fc, counts):
    """The image projector A and its transpose on the workload's grid and
    detector (every angle): A of the phantom's mean-attenuation image, then
    A^T of those projections.  Work: the Siddon voxel segments of every ray
    (fcat_walk_stats), one FMA-accumulation (A) or one atomic add (A^T) each."""
    import synth
    g, ph, s = cfg.geometry, cfg.phantom, cfg.spectral
    grid = synth.Grid(nx=ph.nx, ny=ph.ny, nz=ph.nz, dx=ph.dx, dy=ph.dy, dz=ph.dz, cx=ph.cx, cy=ph.cy, cz=ph.cz)
    w = (s.phi * s.eta).astype(np.float64)
    mbar = torch.as_tensor((s.mu @ w / w.sum()).astype(np.float32), device=pb.phantom.labels.device)
    image = mbar[pb.phantom.labels.long()].contiguous()
    proj = torch.empty((g.n_angles, g.nv, g.nu), dtype=torch.float32, device=image.device)
    back = torch.empty_like(image)
    stream = torch.cuda.current_stream()
    tf, st_f = timed_steps(lambda: fc.fcat_image_project(pb.geometry, grid, image, out=proj, stream=stream),
                           1, args.form_steps, torch)
    tb, st_b = timed_steps(lambda: fc.fcat_image_backproject(pb.geometry, grid, proj, image=back, stream=stream),
                           1, args.form_steps, torch)
    K = args.form_steps
    segs = float(counts["siddon_segments"])
    f_ms, b_ms = st_f["trace"][0] / K, st_b["backproject"][0] / K
    finite = bool(torch.isfinite(proj).all().item() and torch.isfinite(back).all().item())
    del image, proj, back
    return {
        "grid": [grid.nx, grid.ny, grid.nz], "angles": g.n_angles, "voxel_segments": segs, "finite": finite,
        "project": {"ms_per_step": round(1e3 * tf / K, 4), "segments_per_s": segs / (f_ms * 1e-3),
                    "roofline": alu_roof("k_image_rays<false>", OPS_PER_SEGMENT * segs, f_ms,
                                         work_unit=f"{OPS_PER_SEGMENT} lane-ops per Siddon voxel segment")},
        "backproject": {"ms_per_step": round(1e3 * tb / K, 4), "segments_per_s": segs / (b_ms * 1e-3),
                        # one FP32 atomic add to the image per segment: priced against the
                        # measured atomic-add ceiling (there is no published figure)
                        "roofline": {"kernel": "k_image_rays<true>", "bound": "atomic",
                                     "achieved": round(segs / (b_ms * 1e-3) / 1e9, 2), "peak": None,
                                     "unit": "Gatomic/s", "frac": None,
                                     "work_unit": "one FP32 atomic add per Siddon voxel segment",
                                     "alu_view": alu_roof("k_image_rays<true>", OPS_PER_SEGMENT * segs, b_ms,
                                                          work_unit=f"{OPS_PER_SEGMENT} lane-ops per Siddon voxel "
                                                                    "segment"),
                                     # the same adds against the ceiling of adds whose lanes
                                     # each fall on a line of their own
                                     "scattered_view": {"kernel": "k_image_rays<true>", "bound": "atomic_scattered",
                                                        "achieved": round(segs / (b_ms * 1e-3) / 1e9, 2),
                                                        "peak": None, "unit": "Gatomic/s", "frac": None}}},
    }


def dose_stage(pb, cfg, args, torch, fc, hit_rays):
    """Dose per particle (Eqs. 6-7) over all angles of the workload: the walk
    writes path lengths, k_dose_rays sums 1 - exp(-P) per bin over the rays
    that meet the phantom (M FMAs, the negated expm1 as a transcendental of
    EXP_SLOTS and two operations more per hit ray and bin)."""
    import synth
    s = cfg.spectral
    ratio = synth.energy_absorption_ratio(np.random.default_rng(2011), s.energies, 1.0)
    energy = torch.as_tensor(s.energies.astype(np.float32)).cuda()
    ratio = torch.as_tensor(ratio).cuda()
    mass = synth.phantom_mass_kg(cfg.phantom, synth.material_densities(s.material_names))
    ws = torch.empty(fc.fcat_dose_workspace_bytes(pb), dtype=torch.uint8, device=energy.device)
    stream = torch.cuda.current_stream()
    res = {}

    def step():
        res["d"] = fc.fcat_dose(pb, energy, ratio, mass, workspace=ws, stream=stream)

    elapsed, stages = timed_steps(step, 1, args.form_steps, torch)
    dose_ms, dose_n = stages["dose"]
    # the dose stage launches k_dose_rays and k_dose_sum per chunk and k_dose_final once;
    # the kernel-trace summary gives k_dose_rays alone, the stage time bounds it from above
    ops = hit_rays * s.n_energy * (s.n_mat + 2 + EXP_SLOTS)
    per_step = dose_ms / args.form_steps
    ach = ops / (per_step * 1e-3) / 1e12
    D0, Dp = res["d"]
    del ws
    return {
        "ms_per_step": round(1e3 * elapsed / args.form_steps, 4),
        "steps": args.form_steps,
        "stages_ms_per_step": {k: round(v[0] / args.form_steps, 4) for k, v in stages.items() if v[1]},
        "mass_kg": mass,
        "Dp_MeV_per_kg_per_particle": float(Dp.item()),
        "roofline": {"kernel": "k_dose_rays (+ k_dose_sum)", "bound": "alu", "achieved": round(ach, 3),
                     "peak": round(PEAK_LANE_OPS / 1e12, 2), "unit": "Top/s",
                     "frac": round(ach * 1e12 / PEAK_LANE_OPS, 4),
                     "frac_single_issue": round(ach * 1e12 / SINGLE_ISSUE_LANE_OPS, 4), "stage_ms": round(per_step, 4),
                     "algorithmic_ops_per_step": ops,
                     "traffic": profiled_traffic("k_dose_rays", source_digest(DOSE_SOURCES))},
    }


def noise_stage(pb, cfg, args, torch, fc):
    """Projections with Poisson noise (Eq. 5) on the same workload: the whole
    fcat_projections call per step, and the roofline of the Poisson kernel
    (4 B read and 4 B written per draw, one draw per pixel, group and angle)."""
    g, s = cfg.geometry, cfg.spectral
    proj = torch.empty((g.n_angles, g.nv, g.nu), dtype=torch.float32, device=pb.phantom.labels.device)
    ws = torch.empty(fc.fcat_projections_workspace_bytes(pb, "plain"), dtype=torch.uint8, device=proj.device)
    noise = fc.Noise(counts_per_pixel=args.noise_counts, seed=2011)
    stream = torch.cuda.current_stream()
    elapsed, stages = timed_steps(lambda: fc.fcat_projections(pb, noise, out=proj, workspace=ws, stream=stream),
                                  1, args.form_steps, torch)
    draws = g.n_angles * s.n_groups * g.nu * g.nv
    nz_ms, nz_n = stages["noise"]
    per_launch = draws / max(nz_n / args.form_steps, 1)
    avg = nz_ms / max(nz_n, 1)
    ach = 8.0 * per_launch / (avg * 1e-3) / 1e9
    finite = bool(torch.isfinite(proj).all().item())
    del ws, proj
    return {
        "ms_per_step": round(1e3 * elapsed / args.form_steps, 4),
        "steps": args.form_steps,
        "counts_per_pixel": args.noise_counts,
        "draws_per_step": draws,
        "draws_per_s": per_launch / (avg * 1e-3),
        "stages_ms_per_step": {k: round(v[0] / args.form_steps, 4) for k, v in stages.items() if v[1]},
        "finite": finite,
        "roofline": {"kernel": "k_poisson", "bound": "hbm", "achieved": round(ach, 2), "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBPS, 4), "avg_launch_ms": round(avg, 4),
                     "algorithmic_bytes_per_launch": 8.0 * per_launch,
                     "traffic": profiled_traffic("k_poisson", source_digest(NOISE_SOURCES))},
    }


def timed_steps(fn, warmup, steps, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    import paper_2011_04736_amd as fc
    fc.fcat_timing_enable(True)
    fc.fcat_timing_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = fc.fcat_timing_read(reset=True)
    fc.fcat_timing_enable(False)
    return elapsed, stages


def rel_errors(x, ref, torch):
    """Max and RMS of |x - ref| / max(|ref|, 1e-12 max|ref| of the angle), over all pixels."""
    mx, ss, n = 0.0, 0.0, 0
    for a0 in range(0, ref.shape[0], 64):
        r = ref[a0:a0 + 64]
        floor = 1e-12 * r.abs().amax(dim=(1, 2), keepdim=True)
        e = (x[a0:a0 + 64] - r).abs() / torch.maximum(r.abs(), floor)
        mx = max(mx, float(e.max()))
        ss += float(e.double().pow(2).sum())
        n += e.numel()
    return mx, (ss / n) ** 0.5


def walk_work(counts: dict, M: int, E: int) -> tuple[float, float]:
    """(model, executed) lane-operations of the fused walk + spectral kernel:
    OPS_PER_SEGMENT per Siddon voxel segment (the unit of the method's
    work) or per step the two-level walk takes (brick steps plus
    voxel steps inside mixed bricks), plus the spectral sum of every hit ray
    (spectral_ops_per_bin: M FMAs, the weight FMA and an exp2 per bin)."""
    spectral = counts["hit_rays"] * E * spectral_ops_per_bin(M)
    model = OPS_PER_SEGMENT * counts["siddon_segments"] + spectral
    executed = OPS_PER_SEGMENT * (counts["brick_steps"] + counts["voxel_steps"]) + spectral
    return float(model), float(executed)


def plain_workload(name, pb, cfg, warmup, steps, torch, fc):
    """The plain form on one workload: throughput, stage times, walk counts and
    the rooflines of its two kernels.  Returns (entry, out)."""
    g, s = cfg.geometry, cfg.spectral
    dev = pb.phantom.labels.device
    out = torch.empty((g.n_angles, g.nv, g.nu), dtype=torch.float32, device=dev)
    ws = torch.empty(fc.fcat_project_workspace_bytes(pb, "plain"), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    elapsed, stages = timed_steps(lambda: fc.fcat_project(pb, mode="plain", out=out, workspace=ws, stream=stream),
                                  warmup, steps, torch)
    del ws
    counts = fc.fcat_walk_stats(pb)
    rays = g.n_angles * g.nu * g.nv
    M, E, G, K = s.n_mat, s.n_energy, s.n_groups, cfg.psf.k
    mp = 8 if M <= 8 else (10 if M <= 10 else (12 if M <= 12 else (16 if M <= 16 else 32)))   # material slots
    model, executed = walk_work(counts, M, E)
    trace_ms, trace_n = (v / steps for v in stages["trace"])
    psf_ms, psf_n = (v / steps for v in stages["psf"])
    digest = source_digest(TRACE_SOURCES)
    walk = alu_roof(f"k_project_rows<{mp}>", model, trace_ms, trace_n,
                    traffic=profiled_traffic("k_project_rows", digest, name),
                    work_unit=f"{OPS_PER_SEGMENT} lane-ops per Siddon voxel segment + {spectral_ops_per_bin(M)} per hit "
                              f"ray and bin",
                    executed=alu_roof("same launches", executed, trace_ms, trace_n, work_unit=EXECUTED_UNIT),
                    counters=profiled_counters("k_project_rows", digest, name))
    psf_flops = 2.0 * G * K * K * rays
    psf_ach = psf_flops / (psf_ms * 1e-3) / 1e12
    psf = {"kernel": "k_psf4<15, 8, 0>", "bound": "alu", "achieved": round(psf_ach, 3),
           "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s", "frac": round(psf_ach / PEAK_FP32_VECTOR_TFLOPS, 4),
           "stage_ms_per_step": round(psf_ms, 4), "launches_per_step": psf_n,
           "avg_launch_ms": round(psf_ms / max(psf_n, 1), 4), "algorithmic_flops_per_step": psf_flops,
           "traffic": profiled_traffic("k_psf", digest, name),
           "counters": profiled_counters("k_psf4", digest, name)}
    kernels = {"k_project_rows": walk, "k_psf": psf}
    dom = kernels["k_project_rows"] if trace_ms >= psf_ms else kernels["k_psf"]
    roof = {k: dom.get(k) for k in ("kernel", "bound", "achieved", "peak", "unit", "frac", "traffic")}
    if "executed" in dom:
        roof["frac_executed"] = dom["executed"]["frac"]
    entry = {
        "workload": WORKLOADS[name][2],
        "value": rays * E * steps / elapsed, "unit": "ray*E/s",
        "ms_per_step": 1e3 * elapsed / steps, "steps": steps,
        "rays": rays, "energy_bins": E,
        "walk": counts,
        "stages_ms_per_step": {k: round(v[0] / steps, 4) for k, v in stages.items() if v[1]},
        "roofline": roof, "kernels": kernels,
    }
    return entry, out


def form_split(name, pb, cfg, plain_out, steps, torch, fc, counts):
    """The BF16 hi/lo form on a workload: throughput, error against the plain
    form, and the rooflines of its kernels (the walk as in the plain form;
    the contraction and the spread on the matrix cores)."""
    g, s = cfg.geometry, cfg.spectral
    out = torch.empty_like(plain_out)
    ws = torch.empty(fc.fcat_project_workspace_bytes(pb, "split_bf16"), dtype=torch.uint8, device=out.device)
    elapsed, stages = timed_steps(lambda: fc.fcat_project(pb, mode="split_bf16", out=out, workspace=ws),
                                  1, steps, torch)
    del ws
    mx, rms = rel_errors(out, plain_out, torch)
    del out
    rays = g.n_angles * g.nu * g.nv
    M, E, G, K = s.n_mat, s.n_energy, s.n_groups, cfg.psf.k
    model, executed = walk_work(counts, M, E)
    trace_ms, trace_n = (v / steps for v in stages["trace"])
    psf_ms, psf_n = (v / steps for v in stages["psf"])
    digest = source_digest(SPLIT_SOURCES)
    # useful matrix-core work: the three BF16 products (hi.hi, lo.hi, hi.lo)
    # of the contraction, M terms each per hit ray and bin; of the spread,
    # K^2 taps per group and pixel
    con_flops = 2.0 * 3 * M * E * counts["hit_rays"]
    psf_flops = 2.0 * 3 * G * K * K * rays
    mf = lambda f, ms: round(f / (ms * 1e-3) / 1e12, 3)
    kernels = {
        "k_project_rows_split": alu_roof("k_project_rows_split", model, trace_ms, trace_n,
                                         executed=alu_roof("same launches", executed, trace_ms, trace_n,
                                                           work_unit=EXECUTED_UNIT),
                                         counters=profiled_counters("k_project_rows_split", digest, name),
                                         mfma={"bound": "mfma", "achieved": mf(con_flops, trace_ms),
                                               "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
                                               "frac": round(mf(con_flops, trace_ms) / PEAK_BF16_MFMA_TFLOPS, 6),
                                               "algorithmic_flops_per_step": con_flops}),
        "k_psf_split": {"kernel": "k_psf_split", "bound": "mfma", "achieved": mf(psf_flops, psf_ms),
                        "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(mf(psf_flops, psf_ms) / PEAK_BF16_MFMA_TFLOPS, 5),
                        "stage_ms_per_step": round(psf_ms, 4), "launches_per_step": psf_n,
                        "algorithmic_flops_per_step": psf_flops,
                        "counters": profiled_counters("k_psf_split", digest, name)},
    }
    dom = kernels["k_project_rows_split"] if trace_ms >= psf_ms else kernels["k_psf_split"]
    return {"workload": WORKLOADS[name][2], "value": rays * E * steps / elapsed, "unit": "ray*E/s",
            "ms_per_step": 1e3 * elapsed / steps, "steps": steps,
            "stages_ms_per_step": {k: round(v[0] / steps, 4) for k, v in stages.items() if v[1]},
            "max_rel_err_vs_plain": mx, "rms_rel_err_vs_plain": rms,
            "roofline": dict({k: dom.get(k) for k in ("kernel", "bound", "achieved", "peak", "unit", "frac")},
                             **({"frac_executed": dom["executed"]["frac"]} if "executed" in dom else {})),
            "kernels": kernels,
            "note": "the plain form is within 1e-5 and the split form within 1e-3 of the FP64 oracle (parity tests)"}


def form_surrogate(pb, cfg, plain, args, torch, fc, counts):
    """The learned form on the head workload: the network trained here on 4M
    (L, signal) pairs by the library's kernels, then the projector with the
    network and the exact fallback, against the plain form's step."""
    from paper_2011_04736_amd import surrogate as sg
    g, s = cfg.geometry, cfg.spectral
    dev = pb.phantom.labels.device
    rays = g.n_angles * g.nu * g.nv
    ray_e = rays * s.n_energy
    K = args.form_steps
    t0 = time.perf_counter()
    sur, rep = sg.build_surrogate(pb, n_samples=args.surrogate_samples, epochs=args.surrogate_epochs)
    t_build = time.perf_counter() - t0
    out = torch.empty_like(plain["out"])
    ws = torch.empty(fc.fcat_project_workspace_bytes(pb, "surrogate"), dtype=torch.uint8, device=dev)
    sur.counts = torch.zeros(2, dtype=torch.int32, device=dev)
    fc.fcat_project(pb, mode="surrogate", surrogate=sur, out=out, workspace=ws)
    n_net, n_exact = (int(x) for x in sur.counts.cpu().numpy())
    sur.counts = None
    t_sur, st = timed_steps(lambda: fc.fcat_project(pb, mode="surrogate", surrogate=sur, out=out, workspace=ws),
                            0, K, torch)
    del ws
    mx, rms = rel_errors(out, plain["out"], torch)
    del out
    trace_ms, trace_n = (v / K for v in st["trace"])
    M, E = s.n_mat, s.n_energy
    mp = 8 if M <= 8 else (10 if M <= 10 else (12 if M <= 12 else 16))
    # network MACs per ray: n_in*64 + 64*64 + 64*n_out, each product as three BF16 MFMA terms
    macs = 64 * M + 64 * 64 + 64 * s.n_groups
    net_flops = 2.0 * 3 * macs * n_net
    net_ach = net_flops / (trace_ms * 1e-3) / 1e12
    # the fused kernel's vector work: the walk, and the exact spectral sum of the rays that fall back
    model = float(OPS_PER_SEGMENT * counts["siddon_segments"] + n_exact * E * spectral_ops_per_bin(M))
    executed = float(OPS_PER_SEGMENT * (counts["brick_steps"] + counts["voxel_steps"])
                     + n_exact * E * spectral_ops_per_bin(M))
    fused = alu_roof(f"k_project_rows_mlp<{mp}>", model, trace_ms, trace_n,
                     executed=alu_roof("same launches", executed, trace_ms, trace_n,
                                       work_unit=f"{OPS_PER_SEGMENT} lane-ops per walk step taken (brick steps + "
                                                 f"voxel steps in mixed bricks) + the same spectral work"),
                     work_unit=f"{OPS_PER_SEGMENT} lane-ops per Siddon voxel segment + {spectral_ops_per_bin(M)} per bin "
                               f"of each ray that falls back to the exact sum",
                     network={"bound": "mfma", "achieved": round(net_ach, 3), "peak": PEAK_BF16_MFMA_TFLOPS,
                              "unit": "TFLOP/s", "frac": round(net_ach / PEAK_BF16_MFMA_TFLOPS, 5),
                              "algorithmic_flops_per_step": net_flops,
                              "work_unit": "2 x 3 BF16 products x (n_in*64 + 64*64 + 64*n_out) MACs per ray the "
                                           "network takes, over the fused kernel's whole time (walk included)"})
    return {
        "workload": WORKLOADS["head"][2],
        "value": ray_e * K / t_sur, "unit": "ray*E/s", "ms_per_step": 1e3 * t_sur / K, "steps": K,
        "plain_ms_per_step": plain["ms_per_step"],
        "gain_vs_plain": plain["ms_per_step"] / (1e3 * t_sur / K),
        "stages_ms_per_step": {k: round(v[0] / K, 3) for k, v in st.items() if v[1]},
        "max_rel_err_vs_plain": mx, "rms_rel_err_vs_plain": rms,
        "rays_by_network": n_net, "rays_by_exact_sum": n_exact,
        "roofline": dict({k: fused.get(k) for k in ("kernel", "bound", "achieved", "peak", "unit", "frac")},
                         frac_executed=fused["executed"]["frac"]),
        "kernels": {"k_project_rows_mlp": fused},
        "training": {"samples": rep.n_train, "holdout": rep.n_holdout, "epochs": rep.epochs,
                     "train_seconds": round(rep.seconds, 2), "setup_seconds": round(t_build, 2),
                     "final_loss": rep.epoch_loss[-1], "validated_cells": int(rep.cell_ok.sum()),
                     "holdout_share_in_validated_cells": rep.holdout_in_ok_cells},
        "fine_bins": surrogate_fine_bins(pb, cfg, args, torch, fc) if args.surrogate_fine > 1 else None,
    }


def surrogate_fine_bins(pb, cfg, args, torch, fc):
    """Plain and surrogate projectors on the head workload with the same
    spectrum cut into args.surrogate_fine times finer bins: the exact sum's
    cost grows with the number of bins, the network's does not.  The network
    is trained anew on the finer spectrum, with the same sample count and
    schedule."""
    import dataclasses
    import synth
    from paper_2011_04736_amd import surrogate as sg
    spec = synth.refine_spectral(cfg.spectral, args.surrogate_fine)
    dev = pb.phantom.labels.device
    f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=dev)
    sp = fc.Spectral(f32(spec.mu), f32(spec.phi), f32(spec.eta), spec.n_groups, spec.group_of_bin)
    pbf = dataclasses.replace(pb, spectral=sp)
    g = cfg.geometry
    ray_e = g.n_angles * g.nu * g.nv * spec.n_energy
    K = args.form_steps
    out_p = torch.empty((g.n_angles, g.nv, g.nu), dtype=torch.float32, device=dev)
    ws = torch.empty(fc.fcat_project_workspace_bytes(pbf, "plain"), dtype=torch.uint8, device=dev)
    t_plain, st_p = timed_steps(lambda: fc.fcat_project(pbf, mode="plain", out=out_p, workspace=ws), 1, K, torch)
    del ws
    sur, rep = sg.build_surrogate(pbf, n_samples=args.surrogate_samples, epochs=args.surrogate_epochs)
    out = torch.empty_like(out_p)
    ws = torch.empty(fc.fcat_project_workspace_bytes(pbf, "surrogate"), dtype=torch.uint8, device=dev)
    sur.counts = torch.zeros(2, dtype=torch.int32, device=dev)
    fc.fcat_project(pbf, mode="surrogate", surrogate=sur, out=out, workspace=ws)
    n_net, n_exact = (int(x) for x in sur.counts.cpu().numpy())
    sur.counts = None
    t_sur, st_s = timed_steps(lambda: fc.fcat_project(pbf, mode="surrogate", surrogate=sur, out=out, workspace=ws),
                              0, K, torch)
    del ws
    mx, rms = rel_errors(out, out_p, torch)
    del out, out_p
    torch.cuda.empty_cache()
    return {"energy_bins": spec.n_energy, "steps": K,
            "plain": {"value": ray_e * K / t_plain, "unit": "ray*E/s", "ms_per_step": 1e3 * t_plain / K,
                      "stages_ms_per_step": {k: round(v[0] / K, 3) for k, v in st_p.items() if v[1]}},
            "surrogate": {"value": ray_e * K / t_sur, "unit": "ray*E/s", "ms_per_step": 1e3 * t_sur / K,
                          "stages_ms_per_step": {k: round(v[0] / K, 3) for k, v in st_s.items() if v[1]},
                          "max_rel_err_vs_plain": mx, "rms_rel_err_vs_plain": rms,
                          "rays_by_network": n_net, "rays_by_exact_sum": n_exact,
                          "validated_cells": int(rep.cell_ok.sum()),
                          "holdout_share_in_validated_cells": rep.holdout_in_ok_cells},
            "gain_vs_plain": t_plain / t_sur}


# ------------------------------------------------------------------ main

def progress(msg: str):
    """One line on stderr per finished stage (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


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

    if args.copy_probe_mib > 0:
        nel = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(nel, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    forms = [f for f in args.forms.split(",") if f]
    cfgn, variant, desc = WORKLOADS[args.workload]
    cfg = synth.make_config(cfgn, variant=variant)
    g, s = cfg.geometry, cfg.spectral
    pb = fc.upload(cfg, device=dev)
    head, out = plain_workload(args.workload, pb, cfg, args.warmup, args.steps, torch, fc)
    counts = head["walk"]
    progress(f"{args.workload}: plain form, {head['ms_per_step']:.3f} ms per step")

    result = {
        "metric": "rays*energy_bins/s",
        "value": head["value"],
        "unit": "ray*E/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded stand-ins for the paper's phantoms, spectra, scatter and OSFs)",
        "config": {
            "workload": desc,
            "mode": "plain",
            "rays": head["rays"],
            "energy_bins": s.n_energy,
            "hit_rays": counts["hit_rays"],
            "voxel_segments": counts["siddon_segments"],
            "walk_steps": counts["brick_steps"] + counts["voxel_steps"],
        },
        "stages_ms_per_step": head["stages_ms_per_step"],
        "roofline": head["roofline"],
        "roofline_peak_note": PEAK_NOTE,
        "kernels": head["kernels"],
        "walk": counts,
    }
    result["forms"] = {}
    if "split_bf16" in forms:
        result["forms"]["split_bf16"] = {args.workload: form_split(args.workload, pb, cfg, out, args.form_steps,
                                                                   torch, fc, counts)}
        progress(f"{args.workload}: split form")
    if "surrogate" in forms and args.workload == "head":
        result["forms"]["surrogate"] = form_surrogate(pb, cfg, {"out": out, "ms_per_step": head["ms_per_step"]},
                                                      args, torch, fc, counts)
        progress(f"{args.workload}: surrogate form")
    del pb, out
    torch.cuda.empty_cache()

    # secondary workloads; the contrast one also carries the split form of
    # its own configuration and the stages after the projector (run on it
    # as well when it is the primary workload)
    result["workloads"] = {}
    result["next"] = {}
    result["stages"] = {}

    def contrast_stages(p2, c2, walk):
        if args.spectral:
            result["stages"]["spectral"] = spectral_stage(p2, c2, args, torch, fc)
        if args.noise_counts > 0:
            result["next"]["noise_and_projections"] = noise_stage(p2, c2, args, torch, fc)
        if args.dose:
            result["next"]["dose"] = dose_stage(p2, c2, args, torch, fc, walk["hit_rays"])
        if args.fdk:
            result["next"]["fdk"] = fdk_stage(p2, c2, args, torch, fc)
        if args.image_projector:
            result["next"]["image_projector"] = image_projector_stage(p2, c2, args, torch, fc, walk)
        if args.rl_iterations > 0:
            result["next"]["optics"] = optics_stage(p2, c2, args, torch, fc)

    if args.workload == "contrast":
        pb = fc.upload(cfg, device=dev)
        contrast_stages(pb, cfg, counts)
        progress("contrast: the stages after the projector")
        del pb
        torch.cuda.empty_cache()
    for name in [w for w in args.secondary.split(",") if w and w != args.workload]:
        n2, var2, _ = WORKLOADS[name]
        c2 = synth.make_config(n2, variant=var2)
        p2 = fc.upload(c2, device=dev)
        entry, o2 = plain_workload(name, p2, c2, 2, args.secondary_steps, torch, fc)
        result["workloads"][name] = entry
        progress(f"{name}: plain form, {entry['ms_per_step']:.3f} ms per step")
        if name == "contrast":
            if "split_bf16" in forms:
                result["forms"]["split_bf16"][name] = form_split(name, p2, c2, o2, args.secondary_steps, torch, fc,
                                                                 entry["walk"])
            del o2
            torch.cuda.empty_cache()
            contrast_stages(p2, c2, entry["walk"])
            progress(f"{name}: split form and the stages after the projector")
        del p2
        torch.cuda.empty_cache()

    if args.ceilings:
        add_measured_ceilings(result)
    if args.cpu_angles > 0:
        result["cpu_baseline"] = cpu_baseline(cfg, args.cpu_angles, head["rays"] * s.n_energy / g.n_angles)
        progress("oracle on the host cores")
    if args.tiny_oracle:
        result["cpu_tiny_single_thread"] = tiny_oracle()

    print(json.dumps(result))


def measured_ceiling(entry: dict, ceil: dict):
    """The microbenchmark rate that bounds a roofline entry, in the entry's unit."""
    bound, unit = entry.get("bound"), entry.get("unit")
    if bound == "hbm" and unit == "GB/s":
        return ceil["copy_GBps"]
    if bound == "alu" and unit == "TFLOP/s":
        return ceil["fma_f32_TFLOPs"]
    if bound == "alu" and unit == "Top/s":
        return ceil["fma_f32_TFLOPs"] / 2.0        # one FMA is one lane-operation
    if bound == "mfma" and unit == "TFLOP/s":
        return ceil["mfma_bf16_TFLOPs"]
    if bound == "atomic" and unit == "Gatomic/s":
        return ceil.get("atomic_add_f32_Gps")
    if bound == "atomic_scattered" and unit == "Gatomic/s":
        return ceil.get("atomic_add_f32_scattered_Gps")
    return None


def _roofline_entries(node):
    """Every roofline-like dict (one with bound, unit and achieved) under node."""
    if isinstance(node, dict):
        if {"bound", "unit", "achieved"} <= node.keys():
            yield node
        for v in node.values():
            yield from _roofline_entries(v)
    elif isinstance(node, list):
        for v in node:
            yield from _roofline_entries(v)


def add_measured_ceilings(result: dict) -> None:
    """Run the ceiling microbenchmark (a child process) and add measured_peak / frac_measured
    beside every roofline entry whose bound it measures."""
    import subprocess
    exe = os.path.join(ROOT, "paper_2011_04736_amd", "fcat_ceilings")
    if not os.path.exists(exe):
        result["ceilings"] = {"error": "fcat_ceilings not built"}
        return
    try:
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        if r.returncode != 0:
            raise RuntimeError(r.stderr.strip()[-300:] or f"exit status {r.returncode}")
        ceil = json.loads(r.stdout.strip().splitlines()[-1])
    except (OSError, RuntimeError, ValueError, IndexError, subprocess.TimeoutExpired) as e:
        result["ceilings"] = {"error": str(e)[-300:]}
        return
    apply_measured_ceilings(result, ceil)


def apply_measured_ceilings(result: dict, ceil: dict) -> None:
    """Record the ceilings and price every roofline entry they bound against them."""
    result["ceilings"] = ceil
    for e in list(_roofline_entries(result)):
        if "executed" in e or "frac_executed" in e:
            # a walk priced by the model count (every Siddon segment) does less work than
            # it counts where it crosses uniform bricks in one step; its rate against a
            # measured ceiling is carried by the executed-steps entry beside it
            continue
        m = measured_ceiling(e, ceil)
        if m:
            e["measured_peak"] = round(m, 2)
            e["frac_measured"] = round(e["achieved"] / m, 4)
            if e.get("peak") is None:   # no published peak: the measured one stands in
                e["peak"], e["frac"] = e["measured_peak"], e["frac_measured"]


def cpu_baseline(cfg, n_angles: int, ray_e_per_angle: float) -> dict:
    """The FP64 oracle on an evenly spaced sample of the workload's angles,
    every thread of the host; its rate extrapolates linearly to all angles
    (angles are independent and alike in cost)."""
    import oracle
    A = cfg.geometry.n_angles
    angles = np.unique(np.linspace(0, A - 1, n_angles).round().astype(int))
    S = cfg.scatter.maps(angles)
    t0 = time.perf_counter()
    oracle.project(cfg, angles, scatter_maps=S)
    dt = time.perf_counter() - t0
    g = cfg.geometry
    return {"value": len(angles) * ray_e_per_angle / dt, "unit": "ray*E/s", "cores": oracle.max_threads(),
            "kind": "oracle", "seconds": round(dt, 2),
            "sample": (f"{len(angles)} of {A} angles (evenly spaced; linear extrapolation to all {A}: "
                       f"{dt * A / len(angles):.0f} s)" if len(angles) < A else "all angles")
                      + f", full {g.nu}x{g.nv} detector, all {cfg.spectral.n_energy} bins, scatter and PSF"}


def tiny_oracle() -> dict:
    """The FP64 oracle on the whole tiny case (45 angles of 128x16 rays, 32
    bins) on one thread and on every thread."""
    import oracle
    import synth
    cfg = synth.make_config(1)
    ray_e = cfg.ray_energy
    out = {"workload": "tiny phantom 64x64x16 @1 mm, 6 materials, 32 bins 20-120 keV, 128x16 detector, 45 angles",
           "kind": "oracle", "unit": "ray*E/s"}
    n_all = oracle.max_threads()
    for key, nt in (("single_thread", 1), ("all_threads", n_all)):
        t0 = time.perf_counter()
        oracle.project(cfg, list(range(cfg.geometry.n_angles)), n_threads=nt)
        dt = time.perf_counter() - t0
        out[key] = {"seconds": round(dt, 4), "value": ray_e / dt, "cores": nt}
    return out


if __name__ == "__main__":
    main()
