"""Benchmark of the MUSER imaging hot path on one MI355X.

A step is one pass of the whole hot path over one batch: dirty image and dirty beam
(prep, weighting, gridding, inverse FFT, correction), batched Hogbom CLEAN with clean-beam
fit and restore, and the adjoint (FFT then degrid) of the residual.  The headline value is
images/s for the 1024^2 MUSER-II-like batch (520 channels, 1770 baselines, 5000 CLEAN
iterations each), with inputs resident in HBM.  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c2|c4|c1]
                  [--no-cpu-baseline] [--no-plain] [--only-steps]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--only-steps", action="store_true", help="timed steps only (for profilers)")
    ap.add_argument("--plain-subset", type=int, default=8)
    ap.add_argument("--team-size", type=int, default=0,
                    help="CLEAN workgroups per image (0: the library's policy)")
    ap.add_argument("--cpu-baseline-full", action="store_true",
                    help="also time the oracle on 16 C2, 4 C3 and 16 C4 instances (1 core, all cores)")
    ap.add_argument("--no-parity", action="store_true", help="skip the instance-0 check against the oracle")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the imaging schedule and the CLEAN team size with the autotuners before timing")
    ap.add_argument("--steer-cycles", type=int, default=40,
                    help="Steer CLEAN stage: iterations per image (0: skip the stage)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the steps, copy this many MiB device-to-device with a plain kernel "
                         "(calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def synth_arcmin():
    from paper_1712_06913_amd import synth
    return synth.ARCMIN


def synth_w_lambda(name):
    """w coordinates of the workload's visibilities, where its generator provides them."""
    from paper_1712_06913_amd import synth
    if name == "c3":
        return synth.c3_w_lambda()
    return None


def make_workload(name):
    from paper_1712_06913_amd import synth
    if name == "c1":
        return synth.c1_snapshot()
    if name == "c2":
        return synth.c2_muser1_batch()
    if name == "c3":
        return synth.c3_muser2()
    return synth.c4_uneven()


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "k_clean_c3_pmc_traffic.txt")
KERNEL_SOURCES = ("paper_1712_06913_amd/csrc/k_clean.hip", "paper_1712_06913_amd/csrc/mi_internal.h")


def kernel_source_hash():
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, team_size):
    """k_clean HBM-side bytes per launch from the committed counter summary, or None when the
    kernel source changed since the counters were taken (or for another workload / team size)."""
    if workload != "c3" or team_size != 0 or not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    try:
        if vals["kernel_source_sha256"] != kernel_source_hash():
            return None
        return float(vals["k_clean_read_bytes"]) + float(vals["k_clean_write_bytes"])
    except (KeyError, ValueError):
        return None


def oracle_image(args):
    """One instance through the FP64 oracle: dirty image and beam, CLEAN, beam fit, restore
    (the oracle's FFT-convolution form of the restore, equal to its direct sum).  Returns
    (stage seconds, dirty, beam, residual, model, clean-beam fit)."""
    from threadpoolctl import threadpool_limits
    from oracle import clean, imager
    v, uv, w, N, cell, mode, niter, gain = args
    with threadpool_limits(1):
        t0 = time.perf_counter()
        dirty = imager.dirty_image(v, uv, w, N, cell, mode)
        beam = imager.dirty_beam(uv, w, N, cell, mode)
        t1 = time.perf_counter()
        R, model, idx, flux = clean.hogbom(dirty, beam, gain=gain, niter=niter)
        abc = clean.fit_clean_beam(beam)
        t2 = time.perf_counter()
        clean.restore_conv(R, model, abc)
        t3 = time.perf_counter()
    return (t1 - t0, t2 - t1, t3 - t2), dirty, beam, R, model, abc


def _oracle_args(wl, i):
    v, uv, w = wl.instance(i)
    return (v, uv, w, int(wl.n_img[i]), float(wl.cell_rad[i]), int(wl.weight_mode[i]), int(wl.niter[i]), wl.gain)


def host_cores():
    """Worker processes for the oracle: the host's cores, at most 16 (one GPU's share of a box)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(wl, n_sample=None):
    """The FP64 oracle (numpy, one thread per process) on a bounded sample of the workload: the
    first instance in one process, then the first `n_sample` instances (default: one per host
    core) over a process pool of the host's cores.  Returns (the baseline record, instance
    0's oracle outputs)."""
    import concurrent.futures as cf
    t0 = time.perf_counter()
    st, dirty, beam, R, model, abc = oracle_image(_oracle_args(wl, 0))
    one = time.perf_counter() - t0
    k = min(host_cores() if n_sample is None else n_sample, wl.n_inst)
    cores = min(host_cores(), k)
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=cores) as ex:
        list(ex.map(oracle_image, [_oracle_args(wl, i) for i in range(k)]))
    many = time.perf_counter() - t0
    N, niter = int(wl.n_img[0]), int(wl.niter[0])
    rec = {"value": k / many, "unit": "images/s", "cores": cores, "kind": "oracle",
           "single_core_images_per_s": 1.0 / one,
           "sample": f"first {k} instances of {wl.name} (N={N}, {niter} iterations each) over {cores} processes, "
                     f"one thread each: {many:.1f} s; instance 0 alone in one process: dirty+beam {st[0]:.1f} s, "
                     f"CLEAN + beam fit {st[1]:.1f} s, restore {st[2]:.1f} s; FP64 numpy"}
    return rec, (dirty, beam, R, model, abc)


def cpu_baseline_full():
    """Oracle timing on the subsets the measurement plan names (C2: 16, C3: 4, C4: 16 instances),
    one process and then all host cores, extrapolated linearly to the full workloads (and
    labelled so).  Several minutes of host time: run with --cpu-baseline-full."""
    import concurrent.futures as cf
    from paper_1712_06913_amd import synth
    out = {}
    for name, wl, k in (("c2", synth.c2_muser1_batch(), 16), ("c3", synth.c3_muser2(), 4), ("c4", synth.c4_uneven(), 16)):
        jobs = [_oracle_args(wl, i) for i in range(k)]
        t0 = time.perf_counter()
        for j, a in enumerate(jobs):
            oracle_image(a)
            log(f"oracle {name}: instance {j} on one core done")
        t1 = time.perf_counter() - t0
        cores = min(host_cores(), k)
        t0 = time.perf_counter()
        with cf.ProcessPoolExecutor(max_workers=cores) as ex:
            for j, _ in enumerate(cf.as_completed([ex.submit(oracle_image, a) for a in jobs])):
                log(f"oracle {name}: {j + 1} of {k} instances over {cores} processes done")
        tn = time.perf_counter() - t0
        out[name] = {"instances_timed": k, "of": wl.n_inst, "one_core_s": t1, "one_core_images_per_s": k / t1,
                     "cores": cores, "all_cores_s": tn, "all_cores_images_per_s": k / tn,
                     "full_workload_one_core_s_extrapolated": t1 * wl.n_inst / k,
                     "full_workload_all_cores_s_extrapolated": tn * wl.n_inst / k}
        log(f"oracle {name}: {k} instances, 1 core {t1:.1f} s, {cores} cores {tn:.1f} s")
    return out


def parity_instance0(ref, dirty, beam, res, b, gain):
    """The GPU's instance 0 against the oracle run the CPU baseline made of it: the maps
    within 1e-4 of the peak, every CLEAN pick accepted by the oracle's replay on the GPU's
    maps, residual (1e-4), model (1e-5) and restored (1e-4) against the replay."""
    from oracle import clean
    o_dirty, o_beam = ref[0], ref[1]
    N = o_dirty.shape[0]
    D = b.split(dirty)[0].cpu().numpy().astype(np.float64)
    B = b.split(beam, beam=True)[0].cpu().numpy().astype(np.float64)
    peak = float(np.max(np.abs(o_dirty)))
    n = int(res["n_comp"][0])
    off = res["comp_off"]
    ok, bad, R, M = clean.replay(D, B, res["comp_idx"][off[0]: off[0] + n].cpu().numpy(),
                                 res["comp_flux"][off[0]: off[0] + n].cpu().numpy(), gain=gain)
    rest = clean.restore_conv(R, M, clean.fit_clean_beam(B))
    e = {"dirty": float(np.max(np.abs(D - o_dirty))) / peak,
         "beam": float(np.max(np.abs(B - o_beam))),
         "residual": float(np.max(np.abs(b.split(res["residual"])[0].cpu().numpy() - R))) / peak,
         "model": float(np.max(np.abs(b.split(res["model"])[0].cpu().numpy() - M))) / peak,
         "restored": float(np.max(np.abs(b.split(res["restored"])[0].cpu().numpy() - rest))) / peak}
    passed = bool(ok and e["dirty"] <= 1e-4 and e["beam"] <= 1e-4 and e["residual"] <= 1e-4 and e["model"] <= 1e-5
                  and e["restored"] <= 1e-4)
    return {"instance": 0, "components": n, "replay_accepts_every_pick": bool(ok), "first_rejected": int(bad),
            "max_err_over_peak": e, "pass": passed}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the imaging instances are independent and the library runs on "
              f"a single MI355X (requested --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)
    log(f"generating workload {args.workload}")
    wl = make_workload(args.workload)
    log(f"workload {wl.name}: {wl.n_inst} instances, {int(wl.vis_offset[-1])} visibilities")
    cpu, oracle0, cpu_full = None, None, None
    if not args.no_cpu_baseline and not args.only_steps:
        # host-only work, done before anything touches the GPU
        log("timing the CPU oracle baseline")
        cpu, oracle0 = cpu_baseline(wl)
        log(f"CPU oracle: {cpu['value']:.4f} images/s on {cpu['cores']} cores")
        if args.cpu_baseline_full:
            cpu_full = cpu_baseline_full()

    import torch
    from paper_1712_06913_amd import _native as nat, api

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    niter = wl.niter.astype(np.int32)
    b = api.Batch.from_workload(wl, dev)
    vis, uv, w = api.workload_tensors(wl, dev)
    n_inst = wl.n_inst
    img_elems = int(b.img_off[-1])
    beam_elems = int(b.beam_off[-1])
    dirty = torch.empty(img_elems, dtype=torch.float32, device=dev)
    beam = torch.empty(beam_elems, dtype=torch.float32, device=dev)
    b0 = torch.empty(2 * n_inst, dtype=torch.float64, device=dev)
    grid_half = torch.empty(int((b.n_img.astype(np.int64) ** 2 // 2).sum() + (2 * b.n_img.astype(np.int64) ** 2).sum()),
                            dtype=torch.complex64, device=dev)
    adj = torch.empty(int(wl.vis_offset[-1]), dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        api.dirty_image(b, vis, uv, w, beam=True, out=dirty, beam_out=beam, b0_out=b0)
        if ev is not None:
            ev[1].record(stream)
        res = api.hogbom_clean(b, dirty, beam, niter, gain=wl.gain, restore=True, team_size=args.team_size)
        if ev is not None:
            ev[2].record(stream)
        api.degrid(b, res["residual"], uv, w, adjoint=True, out=adj)
        if ev is not None:
            ev[3].record(stream)
        return res

    img_tuning = None
    if args.autotune:
        from paper_1712_06913_amd import pipeline
        img_tuning = pipeline.autotune_imaging(b, vis, uv, w)       # left set on the context
        api.dirty_image(b, vis, uv, w, beam=True, out=dirty, beam_out=beam, b0_out=b0)
        torch.cuda.synchronize()
        args.team_size = pipeline.autotune_team_size(b, dirty, beam, niter, wl.gain)
        log(f"autotuned: imaging (grid_chunk, fft_elems) = {img_tuning}, CLEAN team size {args.team_size or 'policy'}")
    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib * (1 << 18), dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)         # one elementwise kernel: reads and writes calib MiB
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calib_copy_mib} MiB done")
    for i in range(args.warmup):
        res = step()
        torch.cuda.synchronize()
        log(f"warmup step {i} done")

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    # HIP events around each Hogbom, gridder and inverse-transform launch
    api.profile_begin(dev.index or 0, kinds=nat.MI_PROF_CLEAN | nat.MI_PROF_GRID | nat.MI_PROF_IFFT | nat.MI_PROF_GRID_FFT)
    t0 = time.perf_counter()
    for k in range(args.steps):
        res = step(evs[k])
    torch.cuda.synchronize()
    prof_ms, prof_kind = api.profile_end_kinds(dev.index or 0)
    kernel_times = [t for t, k in zip(prof_ms, prof_kind) if k == nat.MI_PROF_CLEAN]
    grid_k_ms = sum(t for t, k in zip(prof_ms, prof_kind) if k == nat.MI_PROF_GRID) / args.steps
    ifft_k_ms = sum(t for t, k in zip(prof_ms, prof_kind) if k == nat.MI_PROF_IFFT) / args.steps
    fused_k_ms = sum(t for t, k in zip(prof_ms, prof_kind) if k == nat.MI_PROF_GRID_FFT) / args.steps
    log(f"{args.steps} timed steps done")
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    img_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    clean_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    adj_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    if args.only_steps:
        print(json.dumps({"ms_per_step": ms_step, "imaging_ms": img_ms, "clean_ms": clean_ms, "adjoint_ms": adj_ms}))
        return
    n_comp = res["n_comp"].cpu().numpy()
    status = b.status.cpu().numpy()

    # gridding alone (prep, weights, dirty grid, beam grid): gridded visibilities per second
    _, _, nk = api.grid(b, vis, uv, w, which=2, layout=1, out=grid_half)
    torch.cuda.synchronize()
    kept = int(nk.cpu().numpy().sum())
    ge = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 5
    ge[0].record(stream)
    for _ in range(reps):
        api.grid(b, vis, uv, w, which=2, layout=1, out=grid_half)
    ge[1].record(stream)
    torch.cuda.synchronize()
    grid_ms = ge[0].elapsed_time(ge[1]) / reps

    # sky / disk levels of the dirty maps (histogram + mixture fit; not part of the step)
    levels, mu_a, _ = api.gmm_levels(b, dirty)
    ge[0].record(stream)
    for _ in range(reps):
        api.gmm_levels(b, dirty, levels=levels.view(-1), mu_a=mu_a)
    ge[1].record(stream)
    torch.cuda.synchronize()
    gmm_ms = ge[0].elapsed_time(ge[1]) / reps

    # disk offsets by correlation with the solar disk (not part of the step)
    radius = 16.0 * synth_arcmin() / b.cell_rad
    offs = api.disk_offsets(b, dirty, radius)
    ge[0].record(stream)
    for _ in range(reps):
        api.disk_offsets(b, dirty, radius, out=offs.view(-1))
    ge[1].record(stream)
    torch.cuda.synchronize()
    center_ms = ge[0].elapsed_time(ge[1]) / reps

    # w-projection (not part of the step): dirty images with the w-term corrected, for the
    # workload's own array geometry (w of each visibility), w_max over the kept visibilities
    wproj = None
    w_lambda = synth_w_lambda(args.workload)
    if w_lambda is not None:
        wl_t = torch.from_numpy(w_lambda).to(dev)
        scale = (b.n_img.astype(np.float64) * b.cell_rad)
        w_max = np.zeros(n_inst)
        for i in range(n_inst):
            a0, a1 = int(wl.vis_offset[i]), int(wl.vis_offset[i + 1])
            g = np.abs(np.floor(np.abs(wl.uv[a0:a1].astype(np.float64) * scale[i]) + 0.5))
            keep = np.all(g <= b.n_img[i] // 2 - 4, axis=1) & (wl.w[a0:a1] > 0)
            w_max[i] = float(np.abs(w_lambda[a0:a1][keep].astype(np.float64)).max()) if keep.any() else 0.0
        wimg, _, n_planes = api.dirty_image_w(b, vis, uv, wl_t, w, w_max)     # builds the kernel tables
        torch.cuda.synchronize()
        ge[0].record(stream)
        for _ in range(reps):
            api.dirty_image_w(b, vis, uv, wl_t, w, w_max, out=wimg)
        ge[1].record(stream)
        torch.cuda.synchronize()
        wp_ms = ge[0].elapsed_time(ge[1]) / reps
        r2 = 2.0 * (0.5 * scale) ** 2
        wproj = {"ms": wp_ms, "planes_min": int(n_planes.min()), "planes_max": int(n_planes.max()),
                 "w_max_lambda": float(w_max.max()),
                 "corner_phase_max_rad": float(np.max(np.pi * w_max * r2)),
                 "kept_vis_per_s": kept / (wp_ms * 1e-3)}
        log("w-projection stage done")

    # roofline of the dominant kernel (k_clean): algorithmic bytes = per iteration the
    # beam window (4 N^2 bytes; the residual stays in LDS) plus once per image the dirty
    # map in, residual + restored out (3 x 4 N^2) and the FP64 model out (8 N^2)
    N2 = b.n_img.astype(np.float64) ** 2
    clean_bytes = float(np.sum(4.0 * N2 * n_comp + 20.0 * N2))
    kernel_ms = float(np.mean(kernel_times))
    achieved = clean_bytes / (kernel_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, args.team_size)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "k_clean",
            "kernel_ms": kernel_ms, "kernel_launches_timed": len(kernel_times), "algorithmic_bytes": clean_bytes,
            "traffic_unit": "HBM-side bytes per launch (L2 read and write requests by size)",
            "traffic_over_algorithmic": (traffic / clean_bytes) if traffic else None}

    # gridding and inverse transforms of the step, timed by the same events.  With the fused
    # gridding + first pass (every size here), the dirty image moves per instance: 24 B read
    # per visibility, the FP64 complex half grid (N/2 x N) written once after the v
    # transforms and read once by pass B, the float32 image written; the beam likewise with
    # 16 B per visibility, its FP64 real half grid (N x 2N, as N complex slots) and the
    # (2N)^2 float32 beam.  The survey's information-minimal bytes (visibilities in, FP32
    # half grids in, maps out, no intermediate) are reported beside them.
    Nf = b.n_img.astype(np.float64)
    hd = float(np.sum(Nf / 2 * Nf * 16.0))
    hbr = float(np.sum(Nf * 2 * Nf * 8.0))
    im, bm = float(np.sum(4.0 * Nf ** 2)), float(np.sum(16.0 * Nf ** 2))
    M = float(wl.vis_offset[-1])
    def _roof(alg, ms):
        a = alg / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "ms": ms, "algorithmic_bytes": alg, "achieved": a, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": a / HBM_PEAK_GBS}
    survey_min = 20.0 * M + float(np.sum(Nf * (Nf / 2 + 1) * 8.0)) + float(np.sum(2 * Nf * (Nf + 1) * 4.0)) + im + bm
    if fused_k_ms > 0.0:
        stage_alg = (24.0 * M + 2 * hd + im) + (16.0 * M + 2 * hbr + bm)
        stage_ms = fused_k_ms + ifft_k_ms
        imaging_roof = {
            "imaging_stage": dict(_roof(stage_alg, stage_ms),
                                  kernels="k_grid_fft_a + k_fft_b_c2r (dirty), k_grid_fft_a_real + k_fft_b_c2r_sym (beam)",
                                  fused_grid_and_first_pass_ms=fused_k_ms, second_pass_ms=ifft_k_ms,
                                  survey_minimal_bytes=survey_min,
                                  frac_survey_minimal=survey_min / (stage_ms * 1e-3) / 1e9 / HBM_PEAK_GBS)}
    else:
        grid_alg = hd + 24.0 * M + hbr + 16.0 * M
        fft_alg = 2 * hd + (hd + im) + 2 * hbr + (hbr + bm)
        imaging_roof = {
            "gridding": dict(_roof(grid_alg, grid_k_ms), kernels="k_grid: dirty FP64 complex + beam FP64 real half grids"),
            "inverse_transform": dict(_roof(fft_alg, ifft_k_ms),
                                      kernels="k_fft_a, k_fft_b_c2r (dirty), k_fft_a_real, k_fft_b_c2r_sym (beam)"),
            "imaging_stage": {"ms": grid_k_ms + ifft_k_ms, "survey_minimal_bytes": survey_min,
                              "frac_survey_minimal": survey_min / ((grid_k_ms + ifft_k_ms) * 1e-3) / 1e9 / HBM_PEAK_GBS}}

    sizes = sorted(set(int(x) for x in b.n_img))
    size_label = f"{sizes[0]}^2" if len(sizes) == 1 else f"mixed {sizes[0]}^2-{sizes[-1]}^2"
    # mi_grid alone (gridding_only): the ABI's complex64 half grids written (dirty N/2 x N,
    # beam N x 2N with zero imaginary parts) and 20 B read per visibility, against the
    # survey's information-minimal gridding bytes (FP32 complex dirty and real beam half grids)
    grid_alg = 20.0 * M + float(np.sum(Nf / 2 * Nf * 8.0)) + float(np.sum(Nf * 2 * Nf * 8.0))
    grid_min = 20.0 * M + float(np.sum(Nf * (Nf / 2 + 1) * 8.0)) + float(np.sum(2 * Nf * (Nf + 1) * 4.0))
    imaging_roof["gridding_mi_grid"] = dict(_roof(grid_alg, grid_ms), kernels="k_bin + k_grid (dirty and beam half grids)",
                                            survey_minimal_bytes=grid_min,
                                            frac_survey_minimal=grid_min / (grid_ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
    out = {
        "metric": f"images/s (grid+iFFT+Hogbom CLEAN, {size_label}, batched)",
        "value": n_inst / (ms_step * 1e-3),
        "unit": "images/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (grid/FFT f64)", "data": "synthetic",
        "config": {"workload": wl.name, "n_inst": n_inst, "N": sorted(set(int(x) for x in b.n_img)),
                   "visibilities": int(wl.vis_offset[-1]), "niter_total": int(niter.sum()),
                   "gain": wl.gain, "weighting": "natural" if not wl.weight_mode.any() else "mixed/uniform",
                   "clean_team_size": args.team_size or "library policy",
                   "imaging_tuning": ({"grid_chunk": img_tuning[0], "fft_elems": img_tuning[1], "source": "autotuner"}
                                      if img_tuning else "library default")},
        "stage_ms": {"dirty_image_and_beam": img_ms, "clean_restore": clean_ms, "adjoint": adj_ms,
                     "gridding_only": grid_ms, "gmm_levels": gmm_ms, "disk_offsets": center_ms},
        "gmm_levels_read_GBps": float(np.sum(8.0 * N2)) / (gmm_ms * 1e-3) / 1e9,
        "gridded_vis_per_s": kept / (grid_ms * 1e-3),
        "kept_visibilities": kept,
        "components_total": int(n_comp.sum()),
        "instance_status_nonzero": int(np.count_nonzero(status)),
        "w_projection": wproj,
        "roofline": roof,
        "imaging_roofline": imaging_roof,
    }

    if not args.no_plain:
        # plain path: one instance per call (a lone image gets the library's team for one
        # image of its size: 32 workgroups on one XCD at 1024^2)
        k = min(args.plain_subset, n_inst)
        sub = wl.subset(range(k))
        sb = api.Batch.from_workload(sub, dev)
        sv, suv, sw = api.workload_tensors(sub, dev)
        singles = []
        for i in range(k):
            s1 = sub.subset([i])
            bb = api.Batch.from_workload(s1, dev)
            tv, tuv, tw = api.workload_tensors(s1, dev)
            singles.append((s1, bb, tv, tuv, tw))

        def plain_once():
            for s1, bb, tv, tuv, tw in singles:
                d, bm, _ = api.dirty_image(bb, tv, tuv, tw, beam=True)
                r = api.hogbom_clean(bb, d, bm, s1.niter, gain=s1.gain, restore=True)
                api.degrid(bb, r["residual"], tuv, tw, adjoint=True)

        def batched_once():
            d, bm, _ = api.dirty_image(sb, sv, suv, sw, beam=True)
            r = api.hogbom_clean(sb, d, bm, sub.niter, gain=sub.gain, restore=True)
            api.degrid(sb, r["residual"], suv, sw, adjoint=True)

        plain_once()
        batched_once()
        torch.cuda.synchronize()
        log("plain/batched warmup done")
        t0 = time.perf_counter()
        plain_once()
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        t0 = time.perf_counter()
        batched_once()
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        out["plain"] = {"subset": f"first {k} instances", "plain_images_per_s": k / tp,
                        "batched_images_per_s_same_subset": k / tb, "batched_over_plain_same_subset": tp / tb,
                        "full_batch_over_plain": out["value"] / (k / tp)}

    # the same step captured once into a HIP graph and replayed (one launch sequence per stage)
    from paper_1712_06913_amd import pipeline
    pl = pipeline.ImagingPipeline(wl, dev, team_size=args.team_size)
    pl.capture()
    pl.replay()                              # first replay (graph upload) untimed
    torch.cuda.synchronize()
    gsteps = max(1, min(args.steps, 3))
    t0 = time.perf_counter()
    for _ in range(gsteps):
        pl.replay()
    torch.cuda.synchronize()
    gms = (time.perf_counter() - t0) * 1e3 / gsteps
    out["graph_replay"] = {"steps": gsteps, "ms_per_step": gms, "images_per_s": n_inst / (gms * 1e-3),
                           "components_total": int(pl.res["n_comp"].sum())}
    del pl
    log("graph-replayed steps done")

    # Steer CLEAN (the paper's deconvolver) on the same dirty maps and beams
    if args.steer_cycles > 0:
        nc = np.full(n_inst, args.steer_cycles, np.int32)
        sres = api.steer_clean(b, dirty, beam, nc, gain=wl.gain, restore=True)
        torch.cuda.synchronize()
        ge[0].record(stream)
        sres = api.steer_clean(b, dirty, beam, nc, gain=wl.gain, restore=True, out=sres)
        ge[1].record(stream)
        torch.cuda.synchronize()
        sms = ge[0].elapsed_time(ge[1])
        cyc = sres["n_cycle"].cpu().numpy().astype(np.float64)
        # algorithmic bytes of this design (spectra stored as FP32 complex between the FP64
        # transforms): per iteration the residual read twice and written once, D written and
        # read, the N (N+1) complex row spectra written and read twice each, and the
        # 2N (N+1) complex beam spectrum read; once per call the beam's spectrum, the
        # initial copy and the restore through the clean beam's spectrum
        Nf = b.n_img.astype(np.float64)
        H = Nf * (Nf + 1) * 8.0
        per_it = 20.0 * Nf ** 2 + 6.0 * H
        once = (16.0 * Nf ** 2 + 6.0 * H) + 16.0 * Nf ** 2 + (12.0 * H + 16.0 * Nf ** 2)
        st_bytes = float(np.sum(per_it * cyc + once))
        st_ach = st_bytes / (sms * 1e-3) / 1e9
        out["steer_clean"] = {"ms": sms, "images_per_s": n_inst / (sms * 1e-3), "cycles_cap": args.steer_cycles,
                              "cycles_total": int(cyc.sum()), "ms_per_cycle_batch": sms / max(1, int(cyc.max())),
                              "trim": 0.9, "restore": True, "algorithmic_bytes": st_bytes, "achieved_GBps": st_ach,
                              "frac_of_hbm_peak": st_ach / HBM_PEAK_GBS}
        del sres
        log("Steer CLEAN stage done")

    if oracle0 is not None and not args.no_parity:
        out["parity"] = parity_instance0(oracle0, dirty, beam, res, b, wl.gain)
        log(f"instance-0 parity: {out['parity']}")
    if cpu is not None:
        out["cpu_baseline"] = cpu
    if cpu_full is not None:
        out["cpu_baseline_subsets"] = cpu_full
    print(json.dumps(out), flush=True)
    api.close()


if __name__ == "__main__":
    main()
