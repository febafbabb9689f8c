"""Benchmark of the polyenergetic cone-beam projector on one MI355X.

A step is one fcat_project call over the whole contrast-phantom workload:
1024x1024x10 labelled voxels (0.15625 mm, 8 materials), 200 energy bins
(0.01-6 MeV), 1024x64 detector at 0.392 mm, 360 angles, per-angle scatter
maps and 8 energy-group 15x15 optical spread kernels.  Inputs are seeded
synthetic stand-ins, resident in HBM before timing starts.

Prints one JSON line: rays x energy-bins per second of the plain FP32 form,
the roofline of the dominant kernel (timed live with HIP events on the
library's stream), the two other forms of the projector (BF16 hi/lo split on
the same workload; the learned surrogate on the head workload, trained here
by the library's own kernels) with their error against the plain form, the
noise and projection stage after the projector (Poisson counts of Eq. 5,
log conversion through the flood) on the same workload, and the FP64 oracle
timed on the host on a bounded sample of the workload.
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

# MI355X: 256 compute units x 4 SIMDs x 16 lanes at 2.4 GHz.
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9          # 3.93e13 vector lane-operations per second
PEAK_FP32_VECTOR_TFLOPS = 157.3               # published FP32 vector peak (packed FMA)
PEAK_BF16_MFMA_TFLOPS = 2500.0                # published dense BF16 matrix peak
PEAK_HBM_GBPS = 8000.0

# Algorithmic work per unit (vector lane-operations).
OPS_PER_SEGMENT = 12          # one voxel segment of the incremental Siddon walk
EXP_SLOTS = 4                 # lane-operations counted for one exp (the hardware exp2 is half rate; expf adds its reduction)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-angles", type=int, default=360,
                    help="angles of the workload the FP64 oracle is timed on (0: skip)")
    ap.add_argument("--variant", default="", help="'z' for the 1.5625 mm slab variant")
    ap.add_argument("--noise-counts", type=float, default=1.0e5,
                    help="H of Eq. 5 (flood counts per open pixel) for the noise stage; 0 skips it")
    ap.add_argument("--dose", type=int, default=1, help="1: time the dose estimate of Eqs. 6-7 (0 skips it)")
    ap.add_argument("--fdk", type=int, default=1, help="1: time the FDK reconstruction of the projections (0 skips it)")
    ap.add_argument("--rl-iterations", type=int, default=10,
                    help="Richardson-Lucy iterations on the detected profiles (0 skips the optics stage)")
    ap.add_argument("--spectral", type=int, default=1, help="1: time steps a3-a4 alone on the hit rays' path lengths")
    ap.add_argument("--ceilings", type=int, default=1,
                    help="1: run the device-ceiling microbenchmark and add fractions of the measured ceilings")
    ap.add_argument("--forms", default="split_bf16,surrogate",
                    help="comma list of extra forms to measure beside the plain one ('' for none)")
    ap.add_argument("--form-steps", type=int, default=3, help="timed steps of the head workload forms")
    ap.add_argument("--surrogate-samples", type=int, default=4_000_000)
    ap.add_argument("--surrogate-epochs", type=int, default=120)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this size first (scale reference for HBM counters)")
    return ap.parse_args()


# ----------------------------------------------------------------- counts

def workload_counts(cfg, angles=None) -> dict:
    """Rays, rays that cross the phantom and voxel segments of the exact walk
    (per-axis voxel-plane crossings inside the box, plus one), for the given
    angles; FP64 slab method in the conventions of the library."""
    g, p = cfg.geometry, cfg.phantom
    n = np.array([p.nx, p.ny, p.nz], np.float64)
    h = np.array([p.dx, p.dy, p.dz], np.float64)
    lo = np.array([p.cx, p.cy, p.cz], np.float64) - n * h / 2
    hi = lo + n * h
    th = g.angle_values()
    if angles is None:
        angles = np.arange(g.n_angles)
    pu = ((np.arange(g.nu) - (g.nu - 1) / 2) * g.du + g.off_u)[None, :]
    pv = ((np.arange(g.nv) - (g.nv - 1) / 2) * g.dv + g.off_v)[:, None]
    segs = hits = 0
    for a in angles:
        c, s = np.cos(th[a]), np.sin(th[a])
        src = np.array([g.sid * c, g.sid * s, 0.0])
        cen = -(g.sdd - g.sid) * np.array([c, s, 0.0])
        dst = np.stack(np.broadcast_arrays(cen[0] - pu * s, cen[1] + pu * c, pv + 0 * pu), -1)
        d = dst - src
        with np.errstate(divide="ignore", invalid="ignore"):
            a0, a1 = (lo - src) / d, (hi - src) / d
            amin = np.maximum(0.0, np.nanmax(np.minimum(a0, a1), -1))
            amax = np.minimum(1.0, np.nanmin(np.maximum(a0, a1), -1))
        hit = amax > amin
        i0 = np.clip(np.floor((src + amin[..., None] * d - lo) / h), 0, n - 1)
        i1 = np.clip(np.floor((src + amax[..., None] * d - lo) / h), 0, n - 1)
        segs += int((1 + np.abs(i1 - i0).sum(-1))[hit].sum())
        hits += int(hit.sum())
    return {"rays": len(angles) * g.nu * g.nv, "hit_rays": hits, "segments": segs}


# -------------------------------------------------------------- traffic

def source_digest(files) -> str:
    hsh = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2011_04736_amd", "csrc", f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()[:16]


TRACE_SOURCES = ["fcat_kernels.hip", "fcat_device.h", "fcat_internal.h"]
NOISE_SOURCES = ["fcat_noise.hip", "fcat_internal.h"]
DOSE_SOURCES = ["fcat_dose.hip", "fcat_internal.h"]
FDK_SOURCES = ["fcat_fdk.hip", "fcat_recon.h"]
BP_OPS_PER_VOXEL_ANGLE = 10   # axial position 1, floor and fraction 2, four-tap bilinear 6, weighted add 1


def profiled_traffic(kernel: str, digest: str):
    """HBM bytes per launch of ``kernel`` from the committed counter summary,
    or None when the summary is missing or was taken on other sources."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{kernel}_contrast.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^sources:\s*(\S+)", text, re.M)
    t = re.search(r"^traffic_bytes_per_launch:\s*(\S+)", text, re.M)
    if not m or not t or m.group(1) != digest:
        return None
    return float(t.group(1))


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
EXP_RATE = 256 * 4 * 16 * 2.4e9 / 2


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
    ops = exps * (M + 2 + EXP_SLOTS)
    ach = ops / (t * 1e-3)
    del Lh, Y, ws
    return {
        "rays": n,
        "energy_bins": E,
        "ms": round(t, 4),
        "exp_per_s": exps / (t * 1e-3),
        "exp_rate_frac": round(exps / (t * 1e-3) / EXP_RATE, 4),
        "roofline": {"kernel": "k_spectral", "bound": "alu", "achieved": round(ach / 1e12, 3),
                     "peak": round(VALU_LANE_OPS / 1e12, 2), "unit": "Top/s", "frac": round(ach / VALU_LANE_OPS, 4),
                     "note": "per hit ray and bin M FMAs, the weight FMA, the scale and an exp counted as "
                             "EXP_SLOTS lane-operations; the exp unit itself is far from busy (exp_rate_frac)"},
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
                     "peak": round(VALU_LANE_OPS / 1e12, 2), "unit": "Top/s",
                     "frac": round(bp_ach * 1e12 / VALU_LANE_OPS, 4), "stage_ms": round(bp_ms, 4),
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
                     "peak": round(VALU_LANE_OPS / 1e12, 2), "unit": "Top/s",
                     "frac": round(ach * 1e12 / VALU_LANE_OPS, 4), "stage_ms": round(per_step, 4),
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


def form_split(pb, cfg, plain_out, args, torch, fc):
    g, s = cfg.geometry, cfg.spectral
    out = torch.empty_like(plain_out)
    ws = torch.empty(fc.fcat_project_workspace_bytes(pb, "split_bf16"), dtype=torch.uint8, device=out.device)
    elapsed, stages = timed_steps(lambda: fc.fcat_project(pb, mode="split_bf16", out=out, workspace=ws),
                                  1, args.steps, torch)
    mx, rms = rel_errors(out, plain_out, torch)
    ray_e = g.n_angles * g.nu * g.nv * s.n_energy
    return {"workload": "contrast phantom (as the plain form)", "value": ray_e * args.steps / elapsed,
            "unit": "ray*E/s", "ms_per_step": 1e3 * elapsed / args.steps,
            "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items() if v[1]},
            "max_rel_err_vs_plain": mx, "rms_rel_err_vs_plain": rms,
            "note": "the plain form is within 1e-5 of the FP64 oracle (parity tests)"}


def form_surrogate(args, torch, fc):
    import synth
    from paper_2011_04736_amd import surrogate as sg
    cfg = synth.make_config(5)
    g, s = cfg.geometry, cfg.spectral
    pb = fc.upload(cfg)
    dev = pb.phantom.labels.device
    ray_e = g.n_angles * g.nu * g.nv * s.n_energy
    K = args.form_steps
    plain = torch.empty((g.n_angles, g.nv, g.nu), dtype=torch.float32, device=dev)
    ws = torch.empty(fc.fcat_project_workspace_bytes(pb, "plain"), dtype=torch.uint8, device=dev)
    t_plain, st_plain = timed_steps(lambda: fc.fcat_project(pb, mode="plain", out=plain, workspace=ws), 1, K, torch)
    del ws
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    sur, rep = sg.build_surrogate(pb, n_samples=args.surrogate_samples, epochs=args.surrogate_epochs)
    t_build = time.perf_counter() - t0
    out = torch.empty_like(plain)
    ws = torch.empty(fc.fcat_project_workspace_bytes(pb, "surrogate"), dtype=torch.uint8, device=dev)
    sur.counts = torch.zeros(2, dtype=torch.int32, device=dev)
    fc.fcat_project(pb, mode="surrogate", surrogate=sur, out=out, workspace=ws)
    counts = sur.counts.cpu().numpy().astype(np.int64)
    sur.counts = None
    t_sur, st_sur = timed_steps(lambda: fc.fcat_project(pb, mode="surrogate", surrogate=sur, out=out, workspace=ws),
                                0, K, torch)
    mx, rms = rel_errors(out, plain, torch)
    mlp_ms = st_sur["mlp"][0] / K
    # network MACs: n_in*64 + 64*64 + 64*n_out per ray that takes the network
    macs = 64 * s.n_mat + 64 * 64 + 64 * s.n_groups
    result = {
        "workload": "head phantom 512x512x256 @0.5 mm, 10 materials, 120 bins 1-120 keV, 1024x768 detector "
                    "@0.4 mm, 720 angles, scatter + 8 groups 15x15 PSF",
        "plain": {"value": ray_e * K / t_plain, "unit": "ray*E/s", "ms_per_step": 1e3 * t_plain / K,
                  "stages_ms_per_step": {k: round(v[0] / K, 3) for k, v in st_plain.items() if v[1]}},
        "surrogate": {"value": ray_e * K / t_sur, "unit": "ray*E/s", "ms_per_step": 1e3 * t_sur / K,
                      "stages_ms_per_step": {k: round(v[0] / K, 3) for k, v in st_sur.items() if v[1]},
                      "max_rel_err_vs_plain": mx, "rms_rel_err_vs_plain": rms,
                      "rays_by_network": int(counts[0]), "rays_by_exact_sum": int(counts[1]),
                      "mlp_stage_mfma_tflops": 2.0 * macs * counts[0] / (mlp_ms * 1e-3) / 1e12,
                      "mlp_stage_mfma_frac": 2.0 * macs * counts[0] / (mlp_ms * 1e-3) / 1e12 / PEAK_BF16_MFMA_TFLOPS},
        "gain_vs_plain": t_plain / t_sur,
        "training": {"samples": rep.n_train, "holdout": rep.n_holdout, "epochs": rep.epochs,
                     "train_seconds": round(rep.seconds, 2), "setup_seconds": round(t_build, 2),
                     "final_loss": rep.epoch_loss[-1], "validated_cells": int(rep.cell_ok.sum()),
                     "holdout_share_in_validated_cells": rep.holdout_in_ok_cells},
    }
    del pb, out, plain, ws
    torch.cuda.empty_cache()
    return result


# ------------------------------------------------------------------ main

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

    cfg = synth.make_config(2, variant=args.variant)
    g, s = cfg.geometry, cfg.spectral
    pb = fc.upload(cfg, device=dev)
    out = torch.empty((g.n_angles, g.nv, g.nu), dtype=torch.float32, device=dev)
    ws = torch.empty(fc.fcat_project_workspace_bytes(pb, "plain"), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    elapsed, stages = timed_steps(lambda: fc.fcat_project(pb, mode="plain", out=out, workspace=ws, stream=stream),
                                  args.warmup, args.steps, torch)

    rays = g.n_angles * g.nu * g.nv
    ray_e = rays * s.n_energy
    ms_per_step = 1e3 * elapsed / args.steps
    value = ray_e * args.steps / elapsed

    # rooflines of the two kernels of the step; the dominant one is reported
    cnt = workload_counts(cfg)
    G, K, M, E = s.n_groups, cfg.psf.k, s.n_mat, s.n_energy
    trace_ms, trace_n = stages["trace"]
    psf_ms, psf_n = stages["psf"]
    trace_ops = (OPS_PER_SEGMENT * cnt["segments"] + cnt["hit_rays"] * E * (M + 2 + EXP_SLOTS)) / max(trace_n
                                                                                                    / args.steps, 1)
    trace_avg = trace_ms / max(trace_n, 1)
    trace_ach = trace_ops / (trace_avg * 1e-3) / 1e12
    psf_flops = 2.0 * G * K * K * rays / max(psf_n / args.steps, 1)
    psf_avg = psf_ms / max(psf_n, 1)
    psf_ach = psf_flops / (psf_avg * 1e-3) / 1e12
    kernels = {
        "k_project_rows": {"bound": "alu", "achieved": round(trace_ach, 3), "peak": round(VALU_LANE_OPS / 1e12, 2),
                           "unit": "Top/s", "frac": round(trace_ach * 1e12 / VALU_LANE_OPS, 4),
                           "avg_launch_ms": round(trace_avg, 4), "launches_per_step": trace_n / args.steps,
                           "algorithmic_ops_per_launch": trace_ops,
                           "traffic": profiled_traffic("k_project_rows", source_digest(TRACE_SOURCES))},
        "k_psf": {"bound": "alu", "achieved": round(psf_ach, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
                  "unit": "TFLOP/s", "frac": round(psf_ach / PEAK_FP32_VECTOR_TFLOPS, 4),
                  "avg_launch_ms": round(psf_avg, 4), "launches_per_step": psf_n / args.steps,
                  "algorithmic_flops_per_launch": psf_flops,
                  "traffic": profiled_traffic("k_psf", source_digest(TRACE_SOURCES))},
    }
    dominant = "k_project_rows" if trace_ms >= psf_ms else "k_psf"
    roof = {k: kernels[dominant][k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")}
    roof["kernel"] = dominant

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
            "mode": "plain",
            "rays": rays,
            "energy_bins": E,
            "hit_rays": cnt["hit_rays"],
            "voxel_segments": cnt["segments"],
        },
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items() if v[1]},
        "hbm_compulsory_GBps": round(hbm, 2),
        "roofline": roof,
        "kernels": kernels,
    }

    forms = [f for f in args.forms.split(",") if f]
    result["forms"] = {}
    if "split_bf16" in forms:
        result["forms"]["split_bf16"] = form_split(pb, cfg, out, args, torch, fc)
    del ws, out
    torch.cuda.empty_cache()
    result["stages"] = {"spectral": spectral_stage(pb, cfg, args, torch, fc)} if args.spectral else {}
    result["next"] = {}
    if args.noise_counts > 0:
        result["next"]["noise_and_projections"] = noise_stage(pb, cfg, args, torch, fc)
    if args.dose:
        result["next"]["dose"] = dose_stage(pb, cfg, args, torch, fc, cnt["hit_rays"])
    if args.fdk:
        result["next"]["fdk"] = fdk_stage(pb, cfg, args, torch, fc)
    if args.rl_iterations > 0:
        result["next"]["optics"] = optics_stage(pb, cfg, args, torch, fc)
    del pb
    torch.cuda.empty_cache()
    if "surrogate" in forms:
        result["forms"]["surrogate"] = form_surrogate(args, torch, fc)

    if args.ceilings:
        add_measured_ceilings(result)
    if args.cpu_angles > 0:
        result["cpu_baseline"] = cpu_baseline(cfg, args.cpu_angles, ray_e / g.n_angles)

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
    return None


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
    result["ceilings"] = ceil
    entries = [result["roofline"], *result["kernels"].values()]
    for group in ("forms", "next", "stages"):
        for v in result.get(group, {}).values():
            for key in ("roofline", "filter"):
                if isinstance(v, dict) and isinstance(v.get(key), dict):
                    entries.append(v[key])
    for e in entries:
        m = measured_ceiling(e, ceil)
        if m:
            e["measured_peak"] = round(m, 2)
            e["frac_measured"] = round(e["achieved"] / m, 4)


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
            "sample": (f"{len(angles)} of {A} angles (evenly spaced), " if len(angles) < A else "all angles, ")
                      + "full detector, all bins, scatter and PSF"}


if __name__ == "__main__":
    main()
