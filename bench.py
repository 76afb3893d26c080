"""Throughput benchmark of the hyperuniform-field hot path on one MI355X.

One step = one call of the whole hot path (white noise, forward FFT, superellipse filter,
inverse FFT, normalisation, sign threshold, continuous and +-1 binned spectra) over one batch:
16 fields on a 2048 x 2048 grid, 128 x 36 bins.  Inputs are synthetic (seeds 1..16, the filter
parameters of the workload), outputs and workspace are preallocated in HBM before timing.

Prints ONE JSON line.  Besides the headline value it carries
  roofline      the dominant kernel's algorithmic bytes per launch / its mean duration
                (HIP events recorded on the launch stream inside the timed region);
  cpu_baseline  the FP64 oracle timed on this host on a bounded sample of the same workload;
  pipeline_roofline_frac  compulsory bytes of the whole pipeline / step time / 8 TB/s;
  plain_form    the same work as one call per field, and the batched speedup over it;
  also          the 3D 256^3 x 4 workload measured the same way; the uneven batch of 512 fields
                (448 2D from 64^2..1024^2, 64 3D from 64^3..128^3) through one replayed graph after
                autotuning, with its plain form; the 512^3 forward plus the adjoint of the
                spectrum-matching loss; the local variance over spherical windows of 8 radii
                (hyperuniformity diagnostic) of the 2D and 3D workloads' fields; and the level cut
                at volume fraction 0.35 with the two-point function S_2 of the cut maps;
  flops         the transform FLOPs of a step (5 N log2 N per transform, and 2.5 N log2 N) and
                the rate they imply;
  parity        the measured error of every output of the 128^2 configuration against the oracle;
  paper_context the paper's two wall times (1024^2, 256^3; hardware not stated) beside one field
                of the same grid here;
  cpu_baseline_all_cores  the oracle's steps with an all-core FFT, with the time of each stage.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the uneven batch and the 512^3 adjoint")
    ap.add_argument("--main-only", action="store_true",
                    help="time only the batched 2D workload (for profiler runs)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="time only the 512^3 forward + adjoint (for profiler runs)")
    ap.add_argument("--c4-only", action="store_true",
                    help="time only the uneven 512-field batch (for profiler runs)")
    ap.add_argument("--workload", default="2d_2048x2048_x16", choices=("2d_2048x2048_x16", "3d_256x256x256_x4"),
                    help="with --main-only: which workload to time")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for scaling PMC byte counters)")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="no GPU: turn rocprofv3 output under DIR into the summaries under profiles/")
    return ap.parse_args()


def algorithmic_bytes(dims, batch):
    """Compulsory HBM bytes per launch of each kernel family and of the whole pipeline.

    Per field, one traversal of the FP32 half spectrum is 8 Nh bytes; the noise is generated in
    registers (never stored); the +-1 map is int8.  2D: 6 traversals + 5N; 3D: 12 traversals + 5N."""
    N = math.prod(dims)
    Nh = N // dims[-1] * (dims[-1] // 2 + 1)
    t = 8 * Nh * batch
    fam = {
        "rows_r2c_noise": t,               # write the half spectrum
        "cols_y_fwd": 2 * t,               # read + write (3D)
        "cols_filter": 2 * t,              # read + write
        "cols_y_inv": 2 * t,
        "rows_c2r_thresh": 2 * t + 5 * N * batch,   # read S, write S(+-1), field f32 and map int8
        "cols_bin": t,                     # read only
    }
    if len(dims) == 2:
        total = 6 * t + 5 * N * batch
    else:
        total = 12 * t + 5 * N * batch
    return fam, total


def adjoint_bytes(dims):
    """Compulsory HBM bytes per launch at one field of the forward (field and continuous spectrum, no
    threshold) and of the adjoint: the gradient pass regenerates the noise spectrum (write), runs the
    y pass (read + write) and reads it once in the axis-0 pass."""
    N = math.prod(dims)
    Nh = N // dims[-1] * (dims[-1] // 2 + 1)
    t = 8 * Nh
    return {"rows_r2c_noise": t, "cols_y_fwd": 2 * t, "cols_filter": 2 * t, "cols_y_inv": 2 * t,
            "rows_c2r": t + 4 * N, "cols_adjoint": t}


# the sources that define the pipeline's kernels and their launch shapes
PIPELINE_SOURCES = ("hu_device.hpp", "hu_common.hpp", "hu_internal.hpp", "hu_host.hpp", "hu_rows.hip", "hu_cols.hip",
                    "hu_filter.hip", "hu_bin.hip", "hu_host.hip", "hu_adjoint.hip", "hu_api.hip", "hu_small.hip",
                    "hu_plane.hip")


def field_bytes_min(dims):
    """Compulsory HBM bytes of one field's whole pipeline: 2D 6 traversals + 5N, 3D 12 + 5N; a 2D
    field whose half spectrum fits in 128 KB (one CU's LDS) could stay on chip: 5N."""
    N = math.prod(dims)
    Nh = N // dims[-1] * (dims[-1] // 2 + 1)
    if len(dims) == 2 and 8 * Nh <= 128 * 1024:
        return 5 * N
    return (6 if len(dims) == 2 else 12) * 8 * Nh + 5 * N


def kernel_source_hash():
    """Hash of the code of the pipeline's kernel sources: line comments and blank lines are left
    out, so an edit of the documentation does not disown counters taken on the same code."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2509_08675_amd", "csrc")
    for f in PIPELINE_SOURCES:
        with open(os.path.join(csrc, f)) as fh:
            for line in fh:
                code = re.sub(r"//.*$", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def pmc_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("workloads", {}).get(workload, {}).get(kernel)


def time_pipeline(hf, torch, cfg, steps, warmup, plain=False):
    dims, seeds, bins = cfg["dims"], cfg["seeds"], cfg["bins"]
    B = len(seeds)
    if plain:
        bufs = [hf.PipelineBuffers(dims, 1, bins) for _ in range(B)]

        def step():
            for i, b in enumerate(bufs):
                hf.pipeline(b, cfg["filt"], [seeds[i]])
    else:
        bufs = hf.PipelineBuffers(dims, B, bins)

        def step():
            hf.pipeline(bufs, cfg["filt"], seeds)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # per-kernel durations: HIP events on the launch stream around every kernel, separate loop
    hf.profile_enable(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    prof = hf.profile_read()
    hf.profile_enable(False)
    check = bufs if not plain else bufs[0]
    hf.check_degenerate(check.stats)
    return el, prof


def autotune_workload(hf, cfg):
    """hu_autotune for a workload's shape class before it is timed (plan search excluded from the
    timing): the plan it keeps and the summed mean kernel time of one pass sequence with the
    default plan and with the tuned one."""
    t0 = time.perf_counter()
    plan, ms = hf.autotune(cfg["dims"], len(cfg["seeds"]), cfg["bins"])
    return dict(plan=[k for k, v in plan.items() if v], default_kernel_ms=round(ms["default_ms"], 4),
                tuned_kernel_ms=round(ms["tuned_ms"], 4), autotune_s=round(time.perf_counter() - t0, 2))


def roofline_obj(cfg, prof, steps, workload):
    fam_bytes, total = algorithmic_bytes(cfg["dims"], len(cfg["seeds"]))
    dom = max(prof.items(), key=lambda kv: kv[1][1])
    name, (launches, ms) = dom
    per_launch_ms = ms / launches
    achieved = fam_bytes.get(name, 0) / (per_launch_ms * 1e-3) / 1e9
    traffic = pmc_traffic(workload, name)
    return dict(bound="hbm", kernel=name, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                algorithmic_bytes_per_launch=fam_bytes.get(name, 0), mean_launch_ms=round(per_launch_ms, 5),
                kernels={k: dict(launches=v[0], mean_ms=round(v[1] / v[0], 5),
                                 gbs=round(fam_bytes.get(k, 0) / (v[1] / v[0] * 1e-3) / 1e9, 1))
                         for k, v in prof.items()}), total


def time_mask_variants(hf, torch, cfg, steps):
    """The whole pipeline on the workload's fields with the mask variants: an antihyperuniform
    filter (alpha = -1) and the offset regularisation (1e-3) on the workload's filter."""
    out = {}
    _, total = algorithmic_bytes(cfg["dims"], len(cfg["seeds"]))
    vox = len(cfg["seeds"]) * math.prod(cfg["dims"])
    for name, change in (("alpha_-1", dict(alpha=-1.0)), ("offset_1e-3", dict(offset=1e-3))):
        c = dict(cfg)
        c["filt"] = dict(cfg["filt"], **change)
        el, _ = time_pipeline(hf, torch, c, steps, 2)
        ms = el / steps * 1e3
        out[name] = dict(filter_change=change, ms_per_step=round(ms, 4), value=round(vox / (ms * 1e-3), 1),
                         pipeline_roofline_frac=round(total / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
    return out


def time_uneven_batch(hf, torch, steps, warmup, plain=True):
    """The uneven batch of 512 fields (448 2D, 64 3D) through hu_pipeline_batch (one replayed
    graph), after autotuning every shape class; and the plain form, one hu_pipeline call per
    field with the default tiles."""
    from paper_2509_08675_amd.workloads import c4_jobs
    jobs = c4_jobs()
    classes = {}
    for j in jobs:
        key = (tuple(j["dims"]), tuple(j["bins"]))
        classes[key] = classes.get(key, 0) + 1
    t0 = time.perf_counter()
    tuning = {}
    for (dims, bins), cnt in classes.items():
        plan, ms = hf.autotune(dims, cnt, bins)
        tuning["x".join(map(str, dims))] = dict(fields=cnt, default_kernel_ms=round(ms["default_ms"], 4),
                                                tuned_kernel_ms=round(ms["tuned_ms"], 4),
                                                plan=[k for k, v in plan.items() if v])
    tune_s = time.perf_counter() - t0
    bb = hf.BatchBuffers(jobs)
    st = hf.pipeline_batch(bb)
    torch.cuda.synchronize()
    if any(st):
        raise RuntimeError("uneven batch: job status %s" % st)
    for _ in range(warmup):
        hf.pipeline_batch(bb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        hf.pipeline_batch(bb)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    for o in bb.out:
        hf.check_degenerate(o["stats"].view(1, 4))
    del bb
    vox = sum(math.prod(j["dims"]) for j in jobs)
    bmin = sum(field_bytes_min(tuple(j["dims"])) for j in jobs)
    if not plain:
        return dict(value=round(vox / (ms * 1e-3), 1), unit="voxels/s", ms_per_step=round(ms, 4), fields=len(jobs),
                    bytes_min=bmin, pipeline_roofline_frac=round(bmin / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    tuning=tuning)
    plain = [hf.PipelineBuffers(j["dims"], 1, j["bins"]) for j in jobs]

    def plain_step():
        for j, b in zip(jobs, plain):
            hf.pipeline(b, j["filt"], [j["seed"]])
    plain_step()
    torch.cuda.synchronize()
    psteps = max(steps // 4, 2)
    t0 = time.perf_counter()
    for _ in range(psteps):
        plain_step()
    torch.cuda.synchronize()
    pms = (time.perf_counter() - t0) / psteps * 1e3
    n2 = sum(1 for j in jobs if len(j["dims"]) == 2)
    return dict(value=round(vox / (ms * 1e-3), 1), unit="voxels/s", ms_per_step=round(ms, 4),
                fields=len(jobs), fields_2d=n2, fields_3d=len(jobs) - n2, voxels=vox, shape_classes=len(classes),
                bytes_min=bmin, pipeline_roofline_frac=round(bmin / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                autotune_s=round(tune_s, 2), tuning=tuning,
                tuning_note="per shape class: summed mean kernel time of one class pass sequence (hu_autotune) "
                            "with the default plan and with the tuned one, and the entries the tuner switched",
                plain_form=dict(desc="one hu_pipeline call per field, default tiles", ms_per_step=round(pms, 4),
                                value=round(vox / (pms * 1e-3), 1), batched_speedup=round(pms / ms, 3)))


def time_adjoint(hf, torch, steps, warmup=1):
    """512^3: forward (field + continuous spectrum) and the adjoint of the spectrum-matching loss."""
    from paper_2509_08675_amd.workloads import C5
    dims, seed, bins = tuple(C5["dims"]), C5["seed"], (C5["nr"], 1)
    filt = C5["filt"]
    N = math.prod(dims)
    Nh = N // dims[-1] * (dims[-1] // 2 + 1)
    field = torch.empty((1,) + dims, dtype=torch.float32, device="cuda")
    wf = hf.alloc_workspace(hf.HU_OP_GEN_FIELD, dims, 1, bins)
    wg = hf.alloc_workspace(hf.HU_OP_LOSS, dims, 1, bins)
    out = hf.gen_field(dims, filt, [seed], cont_bins=bins, work=wf, out=field)
    ts, tc = hf.filter_spectrum(dims, C5["target"], bins)
    cs, cc, stt = out["cont_sum"][0], out["cont_cnt"][0], out["stats"][0]
    loss_t, dL = hf.spectrum_loss_value(bins, cs, cc, ts, tc, 1e-12)      # loss and dL/dP from the library
    loss = float(loss_t.cpu())
    torch.cuda.synchronize()

    def timed(fn, k):
        for _ in range(max(warmup, 1)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k * 1e3
    fwd = timed(lambda: hf.gen_field(dims, filt, [seed], cont_bins=bins, work=wf, out=field), steps)
    bwd = timed(lambda: hf.spectrum_grad(dims, filt, seed, bins, dL, cs, cc, stt, work=wg), steps)
    grad = hf.spectrum_grad(dims, filt, seed, bins, dL, cs, cc, stt, work=wg).cpu().tolist()
    bf, bb = 64 * Nh + 4 * N, 32 * Nh
    return dict(ms_forward=round(fwd, 4), ms_adjoint=round(bwd, 4), ms_total=round(fwd + bwd, 4),
                forward_roofline_frac=round(bf / (fwd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                adjoint_roofline_frac=round(bb / (bwd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                bytes_min_forward=bf, bytes_min_adjoint=bb, loss=loss,
                grad=dict(zip(hf.THETA_NAMES, [float("%.6g" % g) for g in grad])))


def time_window_variance(hf, torch, cfg, steps, radii=(1.0, 2.0, 4.0, 8.0, 16.0, 32.0, 64.0, 128.0)):
    """Local variance over spherical windows of 8 radii for the workload's fields (generated by the
    pipeline beforehand, resident in HBM): one hu_window_variance call per step."""
    dims, seeds, bins = cfg["dims"], cfg["seeds"], cfg["bins"]
    b = hf.PipelineBuffers(dims, len(seeds), bins)
    hf.pipeline(b, cfg["filt"], seeds)
    work = hf.alloc_workspace(hf.HU_OP_WINDOW_VARIANCE, dims, len(seeds))
    fn = lambda: hf.window_variance(b.field, radii, work=work)
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    hf.profile_enable(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    prof = hf.profile_read()
    hf.profile_enable(False)
    N = math.prod(dims)
    Nh = N // dims[-1] * (dims[-1] // 2 + 1)
    B = len(seeds)
    fam = {"rows_r2c_load": 4 * N * B + 8 * Nh * B, "cols_y_fwd": 16 * Nh * B, "cols_wvar": 8 * Nh * B}
    kern = {k: dict(mean_ms=round(v[1] / v[0], 5),
                    gbs=round(fam.get(k, 0) / (v[1] / v[0] * 1e-3) / 1e9, 1)) for k, v in prof.items()}
    modes = Nh * B
    return dict(radii=list(radii), ms_per_call=round(ms, 4), value=round(N * B / (ms * 1e-3), 1), unit="voxels/s",
                kernels=kern, form_factor_evals_per_s=round(modes * len(radii) / (prof["cols_wvar"][1] /
                                                                                   prof["cols_wvar"][0] * 1e-3), 1))


def small_k_after_threshold(hf, torch, cfg, nfit=8):
    """The small-k exponent (Sec. II.A) of the continuous spectrum and of the +-1 map's spectrum of
    the workload's fields (bins pooled over the fields), each with its class of Eqs. (6)-(7): how
    far the threshold refills the low-k hole of the spectrum.  Over a narrow band the continuous
    spectrum's log-slope at the first radial bins exceeds alpha, since the band's Gaussian factor
    adds K (k0 - K) / w^2 to it."""
    dims, bins, seeds = cfg["dims"], cfg["bins"], cfg["seeds"]
    bufs = hf.PipelineBuffers(dims, len(seeds), bins)
    hf.pipeline(bufs, cfg["filt"], seeds)
    torch.cuda.synchronize()
    out = dict(fields=len(seeds), nfit_radial_bins=nfit, filter_alpha=cfg["filt"]["alpha"])
    for name, s, c in (("continuous", bufs.cont_sum, bufs.cont_cnt), ("pm1", bufs.pm1_sum, bufs.pm1_cnt)):
        a = hf.small_k_exponent(s.sum(0), c.sum(0), bins, nfit)
        out[name] = dict(exponent=round(a, 3), hyperuniformity_class=hf.hyperuniformity_class(a, len(dims), tol=0.05))
    return out


def time_two_point(hf, torch, cfg, steps, phi=0.35):
    """Level cut of the workload's fields at volume fraction phi and the two-point function S_2 of
    the resulting maps (fields generated by the pipeline beforehand, resident in HBM)."""
    dims, seeds, bins = cfg["dims"], cfg["seeds"], cfg["bins"]
    b = hf.PipelineBuffers(dims, len(seeds), bins)
    hf.pipeline(b, cfg["filt"], seeds)
    g = torch.empty(b.field.shape, dtype=torch.int8, device="cuda")
    s2 = torch.empty(b.field.shape, dtype=torch.float32, device="cuda")
    work = hf.alloc_workspace(hf.HU_OP_TWO_POINT, dims, len(seeds))

    def fn():
        hf.level_cut(b.field, phi, out=g, counts=False)
        hf.two_point(g, work=work, out=s2)
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    hf.profile_enable(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    prof = hf.profile_read()
    hf.profile_enable(False)
    N = math.prod(dims)
    Nh = N // dims[-1] * (dims[-1] // 2 + 1)
    B = len(seeds)
    t = 8 * Nh * B
    fam = {"threshold": 5 * N * B, "rows_r2c_load": N * B + t, "cols_y_fwd": 2 * t, "cols_square": 2 * t,
           "cols_y_inv": 2 * t, "rows_c2r": t + 4 * N * B}
    kern = {k: dict(mean_ms=round(v[1] / v[0], 5), gbs=round(fam.get(k, 0) / (v[1] / v[0] * 1e-3) / 1e9, 1))
            for k, v in prof.items()}
    total = sum(fam.values()) - (0 if len(dims) == 3 else 4 * t)
    return dict(phi=phi, ms_per_call=round(ms, 4), value=round(N * B / (ms * 1e-3), 1), unit="voxels/s",
                bytes_min=total, roofline_frac=round(total / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), kernels=kern)


def time_small_fields(hf, torch, steps):
    """Small 2D grids through the pass sequence and through the whole-field kernel (plan entry
    whole_field, the half spectrum kept in one workgroup's LDS): the single 128^2 field of the
    parity configuration, and batches of 256 fields of 128^2 and of 64^2.  Compulsory bytes: the
    outputs, 5N per field."""
    from paper_2509_08675_amd.workloads import C1
    out = {}
    for name, dims, B in (("2d_128x128_x1", (128, 128), 1), ("2d_128x128_x256", (128, 128), 256),
                          ("2d_64x64_x256", (64, 64), 256)):
        cfg = dict(C1, name=name, dims=dims, seeds=[1 + i for i in range(B)])
        rec = dict(fields=B)
        for label, whole in (("pass_sequence", 0), ("whole_field", 1)):
            plan = [0] * len(hf.PASS_NAMES)
            plan[hf.PASS_NAMES.index("whole_field")] = whole
            hf.plan_set(dims, B, cfg["bins"], plan)
            el, prof = time_pipeline(hf, torch, cfg, steps, 3)
            ms = el / steps * 1e3
            rec[label] = dict(ms_per_call=round(ms, 4), value=round(B * math.prod(dims) / (ms * 1e-3), 1),
                              kernels={k: round(v[1] / v[0], 5) for k, v in prof.items()})
        hf.plan_set(dims, B, cfg["bins"], [0] * len(hf.PASS_NAMES))
        rec["bytes_min"] = B * field_bytes_min(dims)
        best = min(rec["pass_sequence"]["ms_per_call"], rec["whole_field"]["ms_per_call"])
        rec["roofline_frac_best"] = round(rec["bytes_min"] / (best * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        out[name] = rec
    return out


def flops_obj(cfg, ms):
    """Transform FLOPs of one step: three real transforms per field (the noise's forward, the
    inverse to the field, the +-1 map's forward), counted as 5 N log2 N each (the convention of the
    complex transform) with the real-data figure 2.5 N log2 N beside it."""
    N = math.prod(cfg["dims"])
    B = len(cfg["seeds"])
    f5 = 3 * 5.0 * N * math.log2(N) * B
    f25 = f5 / 2
    return dict(transforms_per_field=3, per_step_5NlogN=f5, per_step_2p5NlogN=f25,
                achieved_tflops_5NlogN=round(f5 / (ms * 1e-3) / 1e12, 2),
                achieved_tflops_2p5NlogN=round(f25 / (ms * 1e-3) / 1e12, 2),
                note="the path is bound by HBM, not by these FLOPs (FP32 vector peak 157.3 TFLOP/s)")


def oracle_stages(cfg, seed, fft):
    """One field through the oracle's steps in the order of the pipeline, timing each; `fft` supplies
    rfftn / irfftn (numpy's, or scipy's on all cores).  Returns {stage: seconds}."""
    import numpy as np
    import oracle
    dims, (nr, na) = tuple(cfg["dims"]), cfg["bins"]
    fp = oracle.FilterParams(**cfg["filt"])
    ax = tuple(range(len(dims)))
    t = {}
    c = time.perf_counter()
    w = oracle.white_noise(dims, seed)
    t["noise"] = time.perf_counter() - c
    c = time.perf_counter()
    W = fft.rfftn(w, axes=ax)
    t["forward_fft"] = time.perf_counter() - c
    c = time.perf_counter()
    F = oracle.amplitude_sym(dims, fp) * W
    t["filter"] = time.perf_counter() - c
    c = time.perf_counter()
    f_raw = fft.irfftn(F, s=dims, axes=ax)
    t["inverse_fft"] = time.perf_counter() - c
    c = time.perf_counter()
    mu = float(f_raw.mean())
    var = float(((f_raw - mu) ** 2).mean())
    f = fp.sigma_f * (f_raw - mu) / np.sqrt(var)
    tm, _, _ = oracle.threshold(f, fp.sigma_f)
    t["normalise_threshold"] = time.perf_counter() - c
    c = time.perf_counter()
    for g in (f, tm.astype(np.float64)):
        G = fft.rfftn(g, axes=ax)
        oracle.bin_power((G.real ** 2 + G.imag ** 2) / g.size, dims, nr, na)
    t["spectra"] = time.perf_counter() - c
    return t


def cpu_baseline_all_cores(cfg, budget_s=12.0):
    """The oracle's steps with scipy.fft on all of this host's cores (workers = the affinity count)
    in place of numpy's single-threaded FFT, on the workload's fields in order until `budget_s`
    seconds have passed, with the time of each stage (the other stages are numpy, one core)."""
    import scipy.fft as sfft
    cores = len(os.sched_getaffinity(0))

    class AllCores:
        @staticmethod
        def rfftn(x, axes):
            return sfft.rfftn(x, axes=axes, workers=cores)

        @staticmethod
        def irfftn(x, s, axes):
            return sfft.irfftn(x, s=s, axes=axes, workers=cores)
    t0 = time.perf_counter()
    n = 0
    stages = {}
    for seed in cfg["seeds"]:
        for k, v in oracle_stages(cfg, seed, AllCores).items():
            stages[k] = stages.get(k, 0.0) + v
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    vox = n * math.prod(cfg["dims"])
    return dict(value=round(vox / el, 1), unit="voxels/s", cores=cores, kind="oracle steps, scipy.fft all cores",
                sample="%d of the %d fields of %s, whole pipeline (field, threshold, both spectra), FP64"
                       % (n, len(cfg["seeds"]), "x".join(map(str, cfg["dims"]))),
                seconds=round(el, 2), stage_seconds_per_field={k: round(v / n, 4) for k, v in stages.items()})


def oracle_stage_breakdown(cfg):
    """Per-stage seconds of the single-core oracle on the workload's first field."""
    import numpy as np

    class OneCore:
        @staticmethod
        def rfftn(x, axes):
            return np.fft.rfftn(x, axes=axes)

        @staticmethod
        def irfftn(x, s, axes):
            return np.fft.irfftn(x, s=s, axes=axes)
    return {k: round(v, 4) for k, v in oracle_stages(cfg, cfg["seeds"][0], OneCore).items()}


def parity_c1(hf, torch):
    """The small parity configuration (128^2, one field, 64 radial bins) on the GPU against the FP64
    oracle: the measured error of every output."""
    import numpy as np
    import oracle
    from paper_2509_08675_amd.workloads import C1
    dims, (nr, na), seed = C1["dims"], C1["bins"], C1["seeds"][0]
    b = hf.PipelineBuffers(dims, 1, (nr, na))
    hf.pipeline(b, C1["filt"], [seed])
    torch.cuda.synchronize()
    fp = oracle.FilterParams(**C1["filt"])
    ref = oracle.pipeline(dims, fp, seed, nr, na)
    cont_ref, _ = oracle.continuous_spectrum_fused(ref["F"], dims, nr, na, fp.sigma_f)
    f = b.field[0].double().cpu().numpy()
    rms = math.sqrt(float(np.mean(ref["f"] ** 2)))
    near = np.abs(ref["f"]) < 1e-5 * rms
    diff = b.pm1[0].cpu().numpy() != ref["t"]
    st = b.stats[0].cpu().numpy()
    cnt = hf.u64_view(b.counts[0])

    def rel(got, r):
        r = np.asarray(r, dtype=np.float64)
        sel = r > 1e-9 * r.max()
        return float(np.max(np.abs(np.asarray(got)[sel] - r[sel]) / r[sel]))
    return dict(workload=C1["name"], field_max_err_over_rms=float(np.max(np.abs(f - ref["f"])) / rms),
                sign_flips=int(diff.sum()), sign_flips_outside_near_zero=int(np.sum(diff & ~near)),
                near_zero_sites=int(near.sum()), mean_err_over_sd=float(abs(st[0] - ref["mu"]) / math.sqrt(ref["var"])),
                var_rel_err=float(abs(st[1] - ref["var"]) / ref["var"]),
                n_pos_err=int(abs(int(cnt[0]) - ref["n_pos"])),
                cont_bins_max_rel_err=rel(b.cont_sum[0].cpu().numpy(), cont_ref),
                pm1_bins_max_rel_err=rel(b.pm1_sum[0].cpu().numpy(), ref["pm1_sum"]),
                bin_counts_exact=bool(np.array_equal(hf.u64_view(b.cont_cnt[0]), ref["cont_cnt"])
                                      and np.array_equal(hf.u64_view(b.pm1_cnt[0]), ref["pm1_cnt"])),
                note="bins compared where the oracle's bin is above 1e-9 of the largest")


def paper_context(hf, torch):
    """The paper's two wall times (hardware, precision and library not stated) beside one field of
    the same grid and parameters through hu_pipeline here."""
    from paper_2509_08675_amd.workloads import paper_preset
    out = {}
    for name, dims, L, alpha, paper_s, where in (
            ("2d_1024sq_alpha20", (1024, 1024), 100.0, 20.0, 0.03, "Sec. III.A"),
            ("3d_256cube_alpha20", (256, 256, 256), 25.0, 20.0, 1.3, "Sec. III.B")):
        filt = paper_preset(dims[0], L, alpha=alpha, p=1.0)
        b = hf.PipelineBuffers(dims, 1, (128, 1))
        for _ in range(3):
            hf.pipeline(b, filt, [1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            hf.pipeline(b, filt, [1])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / 10 * 1e3
        out[name] = dict(paper_seconds=paper_s, paper_source=where, paper_hardware="not stated",
                         here_ms=round(ms, 4), here_outputs="field, sign map, counts, both 128-bin spectra")
        del b
    return out


def cpu_baseline(cfg, budget_s=12.0):
    """The FP64 oracle, as it stands, on the workload's fields in order until `budget_s` seconds
    have passed or all are done (single-threaded numpy; pocketfft runs on one core)."""
    import oracle
    fp = oracle.FilterParams(**cfg["filt"])
    t0 = time.perf_counter()
    nfields = 0
    for s in cfg["seeds"]:
        oracle.pipeline(cfg["dims"], fp, s, *cfg["bins"])
        nfields += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    vox = nfields * math.prod(cfg["dims"])
    return dict(value=round(vox / el, 1), unit="voxels/s", cores=1, kind="oracle",
                sample="%d of the %d fields of %s, whole pipeline (field, threshold, both spectra), FP64"
                       % (nfields, len(cfg["seeds"]), "x".join(map(str, cfg["dims"]))),
                seconds=round(el, 2))


# ---------------------------------------------------------------------------------------------
# rocprofv3 summaries (no GPU): DIR/<workload>/{trace,fetch,write} and DIR/copy_{fetch,write}
# ---------------------------------------------------------------------------------------------
PROFILE_COMMANDS = {
    "trace": "rocprofv3 --kernel-trace --stats -f csv -d DIR/{w}/trace -o trace -- "
             "python3 REPO/bench.py --main-only --workload {w} --steps 20 --warmup 3",
    "fetch": "rocprofv3 --pmc FETCH_SIZE -f csv -d DIR/{w}/fetch -o fetch -- "
             "python3 REPO/bench.py --main-only --workload {w} --steps 3 --warmup 1",
    "write": "rocprofv3 --pmc WRITE_SIZE -f csv -d DIR/{w}/write -o write -- "
             "python3 REPO/bench.py --main-only --workload {w} --steps 3 --warmup 1",
    "copy_fetch": "rocprofv3 --pmc FETCH_SIZE -f csv -d DIR/copy_fetch -o copy_fetch -- "
                  "python3 REPO/bench.py --copy-calibration",
    "copy_write": "rocprofv3 --pmc WRITE_SIZE -f csv -d DIR/copy_write -o copy_write -- "
                  "python3 REPO/bench.py --copy-calibration",
    "adj_trace": "rocprofv3 --kernel-trace --stats -f csv -d DIR/3d_512x512x512_adjoint/trace -o trace -- "
                 "python3 REPO/bench.py --adjoint-only --steps 10 --warmup 2",
    "adj_fetch": "rocprofv3 --pmc FETCH_SIZE -f csv -d DIR/3d_512x512x512_adjoint/fetch -o fetch -- "
                 "python3 REPO/bench.py --adjoint-only --steps 2 --warmup 1",
    "adj_write": "rocprofv3 --pmc WRITE_SIZE -f csv -d DIR/3d_512x512x512_adjoint/write -o write -- "
                 "python3 REPO/bench.py --adjoint-only --steps 2 --warmup 1",
    "sq1": "rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_ACTIVE_INST_VALU "
           "SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_INSTS_VALU_TRANS_F32 -f csv -d DIR/sq1 -o sq1 -- "
           "python3 REPO/bench.py --main-only --steps 2 --warmup 1",
    "c4_trace": "rocprofv3 --kernel-trace --stats -f csv -d DIR/c4_uneven_512_fields/trace -o trace -- "
                "python3 REPO/bench.py --c4-only --steps 10 --warmup 2",
    "sq2": "rocprofv3 --pmc SQ_WAIT_INST_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_ACTIVE_INST_LDS SQ_INSTS_SALU "
           "SQ_WAIT_INST_ANY SQ_INST_CYCLES_VMEM_RD SQ_INSTS_LDS_ATOMIC -f csv -d DIR/sq2 -o sq2 -- "
           "python3 REPO/bench.py --main-only --steps 2 --warmup 1",
}


def kernel_family(name):
    """Pipeline family of a rocprofv3 kernel name (None for other kernels)."""
    import re
    m = re.search(r"hu::(k_\w+)(?:<([^>]*)>)?", name)
    if not m:
        return None
    k, args = m.group(1), [t.strip() for t in (m.group(2) or "").split(",")]
    if k in ("k_finalize", "k_spec_final", "k_grad_coef", "k_grad_final", "k_cols_adjoint"):
        return k[2:]
    if k == "k_rows_r2c":
        return "rows_r2c_noise" if args[1] == "0" else "rows_r2c"
    if k == "k_rows_c2r":
        return "rows_c2r_thresh" if args[1] == "true" else "rows_c2r"
    if k == "k_cols":
        return "cols_y_inv" if args[1] == "true" else "cols_y_fwd"
    if k == "k_plane_inv":
        return "plane_inv_thresh" if args[2] == "true" else "plane_inv"
    if k in ("k_field_lds", "k_plane_fwd"):
        return k[2:]
    return {"k_cols_filter": "cols_filter", "k_cols_bin": "cols_bin", "k_cols_bin_tile": "cols_bin"}.get(k)


def _csv_rows(d, suffix):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit("no *%s under %s" % (suffix, d))
    with open(files[0]) as fh:
        return list(csv.DictReader(fh))


def _per_dispatch(d, counter, family=None, min_value=0.0):
    """{family: median per-dispatch value of counter}; family=None keeps the largest dispatches
    of any kernel (the copy run)."""
    import statistics
    vals = {}
    for r in _csv_rows(d, "_counter_collection.csv"):
        if r["Counter_Name"] != counter:
            continue
        f = kernel_family(r["Kernel_Name"]) if family is None else family
        if f is None:
            continue
        vals.setdefault(f, []).append(float(r["Counter_Value"]))
    if family is not None:
        v = sorted(vals.get(family, []))
        top = [x for x in v if x >= 0.5 * v[-1]] if v else []
        return statistics.median(top) if top else None
    return {f: statistics.median(v) for f, v in vals.items()}


def summarize_profiles(d):
    from paper_2509_08675_amd.workloads import C2, C3
    copy_bytes = 4 << 28
    cf = _per_dispatch(os.path.join(d, "copy_fetch"), "FETCH_SIZE", family="copy")
    cw = _per_dispatch(os.path.join(d, "copy_write"), "WRITE_SIZE", family="copy")
    f_fetch, f_write = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    out = dict(source_hash=kernel_source_hash(), copy_factor=dict(fetch=round(f_fetch, 4), write=round(f_write, 4)),
               workloads={})
    md = ["# Pipeline kernels: rocprofv3 summaries", "",
          "Kernel sources hash (bench.py `kernel_source_hash`): `%s`" % out["source_hash"], "",
          "Commands, each after `cd /tmp && export TMPDIR=/tmp` on one MI355X (`REPO` the repository root, "
          "`DIR` a scratch output folder, `{w}` each workload below); then "
          "`python3 REPO/bench.py --summarize-profiles DIR` writes this file and `pmc_traffic.json`:", ""]
    for k, c in PROFILE_COMMANDS.items():
        md.append("* %s: `%s`" % (k, c))
    md += ["", "## Byte-counter calibration (plain 1 GiB device copy)", "",
           "| counter | KiB per copy dispatch | bytes moved | factor |", "|---|---|---|---|",
           "| FETCH_SIZE | %.0f | %d | %.4f |" % (cf, copy_bytes, f_fetch),
           "| WRITE_SIZE | %.0f | %d | %.4f |" % (cw, copy_bytes, f_write), ""]
    from paper_2509_08675_amd.workloads import C5
    for cfg in (C2, C3, C5):
        w = cfg["name"]
        wd = os.path.join(d, w)
        if not os.path.isdir(wd):
            continue
        if cfg is C5:
            fam_bytes = adjoint_bytes(cfg["dims"])
        else:
            fam_bytes, total = algorithmic_bytes(cfg["dims"], len(cfg["seeds"]))
        md += ["## %s" % w, "", "### Kernel trace (`--kernel-trace --stats`)", "",
               "| kernel | family | calls | mean us | share % |", "|---|---|---|---|---|"]
        for r in _csv_rows(os.path.join(wd, "trace"), "_kernel_stats.csv"):
            if "hu::" not in r["Name"]:
                continue                # the harness's own small torch kernels
            md.append("| `%s` | %s | %s | %.2f | %s |" % (r["Name"].replace("|", "/")[:90], kernel_family(r["Name"]),
                                                        r["Calls"], float(r["AverageNs"]) / 1e3, r["Percentage"]))
        # per-launch durations from the dispatch trace; the last `last` launches of each family are
        # the loop that the bench times with HIP events (the earlier ones are warm-up and the
        # untimed steps)
        last = 10 if cfg is C5 else 20
        per = {}
        for r in _csv_rows(os.path.join(wd, "trace"), "_kernel_trace.csv"):
            f = kernel_family(r["Kernel_Name"])
            if f:
                per.setdefault(f, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
        md += ["", "### Per-launch durations (`--kernel-trace` dispatch records)", "",
               "| family | launches | mean us, all | mean us, last %d (the event-timed loop) |" % last,
               "|---|---|---|---|"]
        for f in sorted(per):
            v = per[f]
            tail = v[-last:]
            md.append("| %s | %d | %.2f | %.2f |" % (f, len(v), sum(v) / len(v), sum(tail) / len(tail)))
        fe = _per_dispatch(os.path.join(wd, "fetch"), "FETCH_SIZE")
        wr = _per_dispatch(os.path.join(wd, "write"), "WRITE_SIZE")
        md += ["", "### HBM traffic per launch (`--pmc FETCH_SIZE`, `--pmc WRITE_SIZE`, calibrated)", "",
               "| family | FETCH KiB | WRITE KiB | traffic bytes | algorithmic bytes | traffic / algorithmic |",
               "|---|---|---|---|---|---|"]
        tr = {}
        for f in sorted(set(fe) | set(wr)):
            b = fe.get(f, 0.0) * 1024 * f_fetch + wr.get(f, 0.0) * 1024 * f_write
            tr[f] = int(round(b))
            alg = fam_bytes.get(f, 0)
            md.append("| %s | %.0f | %.0f | %d | %d | %s |" % (f, fe.get(f, 0.0), wr.get(f, 0.0), tr[f], alg,
                                                               "%.3f" % (b / alg) if alg else "-"))
        out["workloads"][w] = tr
        md.append("")
    sq = {}
    for g in ("sq1", "sq2"):
        if os.path.isdir(os.path.join(d, g)):
            for r in _csv_rows(os.path.join(d, g), "_counter_collection.csv"):
                f = kernel_family(r["Kernel_Name"])
                if f:
                    sq.setdefault(f, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    if sq:
        import statistics
        fam_ms = {}
        for r in _csv_rows(os.path.join(d, C2["name"], "trace"), "_kernel_stats.csv"):
            if kernel_family(r["Name"]):
                fam_ms[kernel_family(r["Name"])] = float(r["AverageNs"]) * 1e-6
        modes = len(C2["seeds"]) * C2["dims"][0] * (C2["dims"][1] // 2 + 1)
        md += ["## Instruction counters, %s (`sq1`, `sq2` passes; whole-chip counts per dispatch)" % C2["name"], "",
               "VALU lane-instructions per half-spectrum mode = SQ_INSTS_VALU x 64 / modes; VALU issue share = "
               "SQ_INSTS_VALU / 256 CUs / (mean duration x 2.4 GHz), i.e. the fraction of cycles in which a CU "
               "issued one wave64 VALU instruction.", "",
               "| family | VALU lane-instr / mode | VALU issue share | LDS instr / mode | LDS bank-conflict cycles / mode "
               "| transcendental lane-instr / mode |", "|---|---|---|---|---|---|"]
        for f in sorted(sq):
            c = {k: statistics.median(v) for k, v in sq[f].items()}
            if f not in fam_ms or "SQ_INSTS_VALU" not in c:
                continue
            share = c["SQ_INSTS_VALU"] / 256.0 / (fam_ms[f] * 1e-3 * 2.4e9)
            md.append("| %s | %.1f | %.2f | %.1f | %.1f | %.1f |" % (
                f, c["SQ_INSTS_VALU"] * 64 / modes, share, c.get("SQ_INSTS_LDS", 0) * 64 / modes,
                c.get("SQ_LDS_BANK_CONFLICT", 0) * 64 / modes, c.get("SQ_INSTS_VALU_TRANS_F32", 0) * 64 / modes))
        md.append("")
    summarize_c4_trace(os.path.join(d, "c4_uneven_512_fields", "trace"))
    with open(os.path.join(ROOT, "profiles", "pmc_traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    with open(os.path.join(ROOT, "profiles", "pipeline_kernels_2048sq_x16_and_256cube_x4.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md))


def summarize_c4_trace(td, replays=10):
    """profiles/batch_kernels_c4_uneven_512.md from the kernel trace of `bench.py --c4-only`: the
    last `replays` graph launches (found as the period of the dispatch sequence), their span on the
    GPU and the summed kernel time per family."""
    if not os.path.isdir(td):
        return
    rows = [r for r in _csv_rows(td, "_kernel_trace.csv") if "hu::" in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    import collections
    names = [r["Kernel_Name"] for r in rows]
    # the classes run on several streams, so the order of the dispatches varies between launches:
    # the period is the smallest K whose last windows of K dispatches hold the same kernels
    period = next((k for k in range(1, len(names) // (replays + 1) + 1)
                   if all(collections.Counter(names[len(names) - (i + 1) * k:len(names) - i * k]) ==
                          collections.Counter(names[len(names) - k:]) for i in range(1, replays))), None)
    if period is None:
        return
    spans, fam = [], {}
    for i in range(replays):
        win = rows[len(rows) - (i + 1) * period:len(rows) - i * period]
        t0 = min(int(r["Start_Timestamp"]) for r in win)
        t1 = max(int(r["End_Timestamp"]) for r in win)
        spans.append((t1 - t0) * 1e-3)
        for r in win:
            f = kernel_family(r["Kernel_Name"]) or r["Kernel_Name"].split("(")[0]
            n, t = fam.get(f, (0, 0.0))
            fam[f] = (n + 1, t + (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    busy = sum(t for _, t in fam.values()) / replays
    md = ["# Uneven batch of 512 fields (448 2D, 64 3D): kernel trace of the replayed graph", "",
          "Command (after `cd /tmp && export TMPDIR=/tmp`; `REPO` the repository root, `DIR` a scratch folder): "
          "`%s`, then `python3 REPO/bench.py --summarize-profiles DIR`." % PROFILE_COMMANDS["c4_trace"], "",
          "The last %d graph launches of the run (%d kernel dispatches each): GPU span of one launch %.1f us "
          "(first dispatch start to last dispatch end), summed kernel time %.1f us per launch (the classes "
          "run on four streams, so kernels overlap and the sum exceeds the span)." % (
              replays, period, sum(spans) / replays, busy), "",
          "| family | dispatches per launch | summed us per launch | mean us per dispatch |", "|---|---|---|---|"]
    for f, (n, t) in sorted(fam.items(), key=lambda kv: -kv[1][1]):
        md.append("| %s | %d | %.1f | %.2f |" % (f, n // replays, t / replays, t / n))

    # the shape class of a dispatch from its template arguments: the row passes take n_x / 2 (2D:
    # tiled layout), the axis-0 and y passes n along that axis (cols_filter names the dimension)
    def shape_class(name):
        import re
        m = re.search(r"hu::k_(\w+)<([^>]*)>", name)
        if not m:
            return None
        k, a = m.group(1), [t.strip() for t in m.group(2).split(",")]
        if k in ("rows_r2c", "rows_c2r"):
            n, d = 2 * int(a[0]), 2 if a[2] == "true" else 3
        elif k == "cols_filter":
            n, d = int(a[0]), int(a[1])
        elif k in ("cols", "cols_bin"):
            n, d = int(a[0]), 3
        elif k == "cols_bin_tile":                 # 2D by default (see the table's caption)
            n, d = int(a[0]), 2
        elif k == "field_lds":                     # <n_x / 2, n0, GEN>: the C4 grids are square
            n, d = int(a[1]), 2
        elif k in ("plane_fwd", "plane_inv"):      # <n_x / 2, n_y, ...>: cubes
            n, d = int(a[1]), 3
        else:
            return None
        return "%dD %d^%d" % (d, n, d)
    cls = {}
    for i in range(replays):
        for r in rows[len(rows) - (i + 1) * period:len(rows) - i * period]:
            c = shape_class(r["Kernel_Name"])
            if c:
                cls[c] = cls.get(c, 0.0) + (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
    md += ["", "Summed kernel time per shape class (the axis passes and the whole-field and plane kernels; "
           "finalize and the final reduction left out).  The one-item-per-workgroup binning kernel's "
           "template arguments do not name the dimension: its dispatches count as 2D, so a 3D class "
           "tuned to it (bin_schedule) shows part of its time under a 2D row of the same length "
           "(here 96 and 128).", "", "| class | summed us per launch |", "|---|---|"]
    for c, t in sorted(cls.items(), key=lambda kv: -kv[1]):
        md.append("| %s | %.1f |" % (c, t / replays))
    with open(os.path.join(ROOT, "profiles", "batch_kernels_c4_uneven_512.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print("\n".join(md))


def copy_calibration(torch):
    n = 1 << 28     # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_bytes_each_way=4 * n, launches=5)), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
        return
    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return
    from paper_2509_08675_amd import hufield as hf
    from paper_2509_08675_amd.workloads import C2, C3
    if args.adjoint_only:
        print(json.dumps(time_adjoint(hf, torch, args.steps, args.warmup)), flush=True)
        return
    if args.c4_only:
        print(json.dumps(time_uneven_batch(hf, torch, args.steps, args.warmup, plain=False)), flush=True)
        return

    cfg = C3 if (args.main_only and args.workload == C3["name"]) else C2
    tuning = autotune_workload(hf, cfg)
    el, prof = time_pipeline(hf, torch, cfg, args.steps, args.warmup)
    ms = el / args.steps * 1e3
    vox = len(cfg["seeds"]) * math.prod(cfg["dims"])
    roof, total = roofline_obj(cfg, prof, args.steps, cfg["name"])
    line = dict(
        metric="field voxels/s (2048^2 2D, 256^3 3D, FP32) + % HBM roofline vs plain form",
        value=round(vox / (ms * 1e-3), 1), unit="voxels/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(ms, 4), higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
        data="synthetic",
        config=dict(workload=cfg["name"], dims=list(cfg["dims"]), batch=len(cfg["seeds"]), bins=list(cfg["bins"]),
                    filter=cfg["filt"], outputs="field f32, +-1 int8, counts, continuous and +-1 spectra"),
        roofline=roof,
        pipeline_roofline_frac=round(total / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        pipeline_bytes_min=total,
        flops=flops_obj(cfg, ms),
        tuning=tuning,
    )
    if args.main_only:
        print(json.dumps(line), flush=True)
        return
    # the same batch with the default plan, for the tuner's gain
    tuned_plan = hf.plan_query(cfg["dims"], len(cfg["seeds"]), cfg["bins"])
    hf.plan_set(cfg["dims"], len(cfg["seeds"]), cfg["bins"], [0] * len(hf.PASS_NAMES))
    del_, _ = time_pipeline(hf, torch, cfg, max(args.steps // 2, 5), 3)
    hf.plan_set(cfg["dims"], len(cfg["seeds"]), cfg["bins"], [tuned_plan[k] for k in hf.PASS_NAMES])
    line["tuning"]["default_plan_ms_per_step"] = round(del_ / max(args.steps // 2, 5) * 1e3, 4)
    pel, _ = time_pipeline(hf, torch, cfg, max(args.steps // 5, 3), 2, plain=True)
    pms = pel / max(args.steps // 5, 3) * 1e3
    line["plain_form"] = dict(desc="one pipeline call per field (16 calls)", ms_per_step=round(pms, 4),
                              value=round(vox / (pms * 1e-3), 1), batched_speedup=round(pms / ms, 3))
    if not args.no_3d:
        tuning3 = autotune_workload(hf, C3)
        el3, prof3 = time_pipeline(hf, torch, C3, max(args.steps // 2, 5), 3)
        ms3 = el3 / max(args.steps // 2, 5) * 1e3
        vox3 = len(C3["seeds"]) * math.prod(C3["dims"])
        roof3, total3 = roofline_obj(C3, prof3, args.steps, C3["name"])
        line["also"] = {C3["name"]: dict(value=round(vox3 / (ms3 * 1e-3), 1), unit="voxels/s",
                                         ms_per_step=round(ms3, 4),
                                         pipeline_roofline_frac=round(total3 / (ms3 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                         roofline=roof3, tuning=tuning3)}
    if not args.no_extra:
        line.setdefault("also", {})
        line["also"]["c4_uneven_512_fields"] = time_uneven_batch(hf, torch, max(args.steps // 5, 5), 2)
        line["also"]["3d_512cube_forward_and_adjoint"] = time_adjoint(hf, torch, max(args.steps // 5, 5))
        line["also"]["window_variance_2048sq_x16_8radii"] = time_window_variance(hf, torch, C2, max(args.steps // 5, 5))
        line["also"]["window_variance_256cube_x4_8radii"] = time_window_variance(hf, torch, C3, max(args.steps // 5, 5))
        line["also"]["level_cut_and_two_point_2048sq_x16"] = time_two_point(hf, torch, C2, max(args.steps // 5, 5))
        line["also"]["level_cut_and_two_point_256cube_x4"] = time_two_point(hf, torch, C3, max(args.steps // 5, 5))
        line["also"]["mask_variants_2048sq_x16"] = time_mask_variants(hf, torch, C2, max(args.steps // 5, 5))
        line["also"]["small_2d_fields"] = time_small_fields(hf, torch, max(args.steps // 5, 5))
        line["also"]["small_k_exponent_after_threshold"] = {c["name"]: small_k_after_threshold(hf, torch, c)
                                                            for c in (C2, C3)}
    line["parity"] = parity_c1(hf, torch)
    line["paper_context"] = paper_context(hf, torch)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg)
        line["cpu_baseline"]["stage_seconds_first_field"] = oracle_stage_breakdown(cfg)
        line["cpu_baseline_all_cores"] = cpu_baseline_all_cores(cfg)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
