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


def cpu_baseline(wl, restore_sample=300):
    """The FP64 oracle on a bounded sample of the workload, single process (numpy, 1 thread):
    one instance's dirty image and beam, its full CLEAN and the beam fit, and the restore of
    the first `restore_sample` model pixels.  The oracle's restore adds one full-image
    Gaussian per model pixel, so its time is scaled by the instance's model-pixel count."""
    from oracle import clean, imager
    i = 0
    v, uv, w = wl.instance(i)
    N, cell, mode, niter = int(wl.n_img[i]), float(wl.cell_rad[i]), int(wl.weight_mode[i]), int(wl.niter[i])
    t0 = time.perf_counter()
    dirty = imager.dirty_image(v, uv, w, N, cell, mode)
    beam = imager.dirty_beam(uv, w, N, cell, mode)
    t1 = time.perf_counter()
    R, model, idx, flux = clean.hogbom(dirty, beam, gain=wl.gain, niter=niter)
    abc = clean.fit_clean_beam(beam)
    t2 = time.perf_counter()
    nz = np.flatnonzero(model)
    k = min(restore_sample, len(nz))
    sub = np.zeros_like(model)
    sub.flat[nz[:k]] = model.flat[nz[:k]]
    clean.restore(R, sub, abc)
    t3 = time.perf_counter()
    scale = len(nz) / max(k, 1)
    per_image = (t2 - t0) + scale * (t3 - t2)
    return {"value": 1.0 / per_image, "unit": "images/s", "cores": 1, "kind": "oracle",
            "sample": f"instance 0 of {wl.name} (N={N}, {len(v)} baselines, {niter} iterations): dirty+beam "
                      f"{t1 - t0:.1f} s, CLEAN + beam fit {t2 - t1:.1f} s, restore of {k} of its {len(nz)} model "
                      f"pixels {t3 - t2:.1f} s scaled x{scale:.2f} -> {per_image:.1f} s per image; FP64 numpy, "
                      f"single process, 1 thread"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the imaging instances are independent and the library runs on "
              f"a single MI355X (requested --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)
    log(f"generating workload {args.workload}")
    wl = make_workload(args.workload)
    log(f"workload {wl.name}: {wl.n_inst} instances, {int(wl.vis_offset[-1])} visibilities")
    cpu = None
    if not args.no_cpu_baseline and not args.only_steps:
        # host-only work, done before anything touches the GPU
        log("timing the CPU oracle baseline")
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            cpu = cpu_baseline(wl)
        log(f"CPU oracle: {cpu['value']:.4f} images/s")

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
    api.profile_begin(dev.index or 0, kinds=nat.MI_PROF_CLEAN | nat.MI_PROF_GRID | nat.MI_PROF_IFFT)
    t0 = time.perf_counter()
    for k in range(args.steps):
        res = step(evs[k])
    torch.cuda.synchronize()
    prof_ms, prof_kind = api.profile_end_kinds(dev.index or 0)
    kernel_times = [t for t, k in zip(prof_ms, prof_kind) if k == nat.MI_PROF_CLEAN]
    grid_k_ms = sum(t for t, k in zip(prof_ms, prof_kind) if k == nat.MI_PROF_GRID) / args.steps
    ifft_k_ms = sum(t for t, k in zip(prof_ms, prof_kind) if k == nat.MI_PROF_IFFT) / args.steps
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

    # gridding and inverse transforms of the step, timed by the same events: algorithmic
    # bytes of this design per step (FP64 complex dirty half grid N/2 x N, FP64 real beam
    # half grid N x 2N, float32 maps; the gridders also read 24 B (dirty) and 16 B (beam)
    # per visibility; the transform's two passes move each half grid in and out of HBM)
    Nf = b.n_img.astype(np.float64)
    hd = float(np.sum(Nf / 2 * Nf * 16.0))
    hbr = float(np.sum(Nf * 2 * Nf * 8.0))
    im, bm = float(np.sum(4.0 * Nf ** 2)), float(np.sum(16.0 * Nf ** 2))
    M = float(wl.vis_offset[-1])
    grid_alg = hd + 24.0 * M + hbr + 16.0 * M
    fft_alg = 2 * hd + (hd + im) + 2 * hbr + (hbr + bm)
    fft_min = (hd + im) + (hbr + bm)
    def _roof(alg, ms):
        a = alg / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "ms": ms, "algorithmic_bytes": alg, "achieved": a, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": a / HBM_PEAK_GBS}
    imaging_roof = {
        "gridding": dict(_roof(grid_alg, grid_k_ms), kernels="k_grid: dirty FP64 complex + beam FP64 real half grids"),
        "inverse_transform": dict(_roof(fft_alg, ifft_k_ms),
                                  kernels="k_fft_a, k_fft_b_c2r (dirty), k_fft_a_real, k_fft_b_c2r_sym (beam)",
                                  information_minimal_bytes=fft_min,
                                  frac_information_minimal=fft_min / (ifft_k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS),
    }

    out = {
        "metric": "images/s (grid+iFFT+Hogbom CLEAN, 1024^2, batched)",
        "value": n_inst / (ms_step * 1e-3),
        "unit": "images/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (grid/FFT f64)", "data": "synthetic",
        "config": {"workload": wl.name, "n_inst": n_inst, "N": sorted(set(int(x) for x in b.n_img)),
                   "visibilities": int(wl.vis_offset[-1]), "niter_total": int(niter.sum()),
                   "gain": wl.gain, "weighting": "natural" if not wl.weight_mode.any() else "mixed/uniform",
                   "clean_team_size": args.team_size or "library policy"},
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
        # plain path: one instance per call, CLEAN spread over the whole GPU for that image
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

    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
