"""Batched imaging step: dirty image + beam -> CLEAN + restore -> adjoint of the residual.

`ImagingPipeline` owns persistent device buffers for one batch descriptor so a step makes
no allocation, and can replay the step from a captured HIP graph (torch.cuda.CUDAGraph).
With threshold="gmm_sky" the step also fits the sky / disk levels of every dirty map
(Sec. 4.1) and CLEAN stops at the sky level mu_a read on the device (Algorithm 1).
`autotune_team_size` picks the CLEAN team size (workgroups per image) for a batch shape by
timing a short proxy run of every candidate; `autotune_imaging` picks the gridder's tiles
per workgroup and the transform's points per workgroup (mi_set_tuning) by timing the dirty
image and beam under each candidate; choices are cached by shape key.  (The oversampling
factor is not a tuning knob: it is part of the method's definition.)
"""
from __future__ import annotations

import time
from typing import Dict, Optional, Tuple

import numpy as np
import torch

from . import api

_TEAM_CACHE: Dict[Tuple, int] = {}


def shape_key(batch: api.Batch, niter) -> Tuple:
    sizes, counts = np.unique(batch.n_img, return_counts=True)
    return (tuple(int(s) for s in sizes), tuple(int(c) for c in counts), int(np.max(niter)) // 500)


def team_candidates(batch: api.Batch):
    n_max, n_min = int(batch.n_img.max()), int(batch.n_img.min())
    g_min = max(1, n_max * n_max // 65536)
    g_cap = min(256, n_min)
    out, g = [0], g_min
    while g <= g_cap:
        out.append(g)
        g *= 2
    return out


def autotune_team_size(batch: api.Batch, dirty, beam, niter, gain=0.1, proxy_iters=200, reps=2) -> int:
    """Fastest CLEAN team size (0 = the library's default policy) for this batch shape."""
    key = shape_key(batch, niter)
    if key in _TEAM_CACHE:
        return _TEAM_CACHE[key]
    proxy = np.minimum(np.asarray(niter, np.int32), proxy_iters)
    best, best_t = 0, float("inf")
    for ts in team_candidates(batch):
        try:
            api.hogbom_clean(batch, dirty, beam, proxy, gain=gain, restore=False, team_size=ts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                api.hogbom_clean(batch, dirty, beam, proxy, gain=gain, restore=False, team_size=ts)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / reps
        except Exception:       # a candidate the device cannot host
            continue
        if t < best_t:
            best, best_t = ts, t
    _TEAM_CACHE[key] = best
    return best


_IMG_CACHE: Dict[Tuple, Tuple[int, int]] = {}


def imaging_shape_key(batch: api.Batch) -> Tuple:
    sizes, counts = np.unique(batch.n_img, return_counts=True)
    per = max(1, int(batch.vis_offset[-1]) // max(1, batch.n_inst))
    return (tuple(int(s) for s in sizes), tuple(int(c) for c in counts), int(np.log2(per)))


def imaging_candidates():
    """(grid_chunk, fft_elems) pairs: tiles per gridder workgroup x transform block size."""
    return [(c, e) for e in (0, 8192) for c in (2, 4, 8, 16, 32)]


def autotune_imaging(batch: api.Batch, vis, uv, w, reps: int = 3) -> Tuple[int, int]:
    """Fastest (grid_chunk, fft_elems) for the dirty image + beam of this batch shape; the
    choice is left set on the batch's context (it applies to every later call there)."""
    key = imaging_shape_key(batch)
    if key in _IMG_CACHE:
        api.set_tuning(batch.ctx, *_IMG_CACHE[key])
        return _IMG_CACHE[key]
    dev = batch.device
    dirty = torch.empty(int(batch.img_off[-1]), dtype=torch.float32, device=dev)
    beam = torch.empty(int(batch.beam_off[-1]), dtype=torch.float32, device=dev)
    b0 = torch.empty(2 * batch.n_inst, dtype=torch.float64, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    best, best_t = (8, 0), float("inf")
    for cand in imaging_candidates():
        api.set_tuning(batch.ctx, *cand)
        api.dirty_image(batch, vis, uv, w, beam=True, out=dirty, beam_out=beam, b0_out=b0)   # plan + warm-up
        ev[0].record()
        for _ in range(reps):
            api.dirty_image(batch, vis, uv, w, beam=True, out=dirty, beam_out=beam, b0_out=b0)
        ev[1].record()
        torch.cuda.synchronize()
        t = ev[0].elapsed_time(ev[1]) / reps
        if t < best_t:
            best, best_t = cand, t
    api.set_tuning(batch.ctx, *best)
    _IMG_CACHE[key] = best
    return best


class ImagingPipeline:
    """One batch descriptor, persistent buffers, eager or graph-replayed steps."""

    def __init__(self, wl, device="cuda:0", team_size: int = 0, restore: bool = True, adjoint: bool = True,
                 threshold=None, positive_only: bool = False):
        self.dev = torch.device(device)
        self.wl = wl
        self.batch = api.Batch.from_workload(wl, self.dev)
        self.vis, self.uv, self.w = api.workload_tensors(wl, self.dev)
        b = self.batch
        self.niter = np.ascontiguousarray(wl.niter, np.int32)
        self.gain = float(wl.gain)
        self.team_size = team_size
        self.restore = restore
        self.adjoint = adjoint
        nimg, nbeam = int(b.img_off[-1]), int(b.beam_off[-1])
        self.dirty = torch.empty(nimg, dtype=torch.float32, device=self.dev)
        self.beam = torch.empty(nbeam, dtype=torch.float32, device=self.dev)
        self.b0 = torch.empty(2 * b.n_inst, dtype=torch.float64, device=self.dev)
        self.adj = torch.empty(int(wl.vis_offset[-1]), dtype=torch.complex64, device=self.dev)
        self.threshold = threshold
        self.positive_only = positive_only
        self.levels = torch.empty(6 * b.n_inst, dtype=torch.float64, device=self.dev)
        self.mu_a = torch.empty(b.n_inst, dtype=torch.float32, device=self.dev)
        self.mu_b = torch.empty(b.n_inst, dtype=torch.float32, device=self.dev)
        self.res = None
        self.graph: Optional[torch.cuda.CUDAGraph] = None

    def step(self):
        b = self.batch
        api.dirty_image(b, self.vis, self.uv, self.w, beam=True, out=self.dirty, beam_out=self.beam, b0_out=self.b0)
        thr = self.threshold
        if isinstance(thr, str):
            if thr != "gmm_sky":
                raise ValueError(f"unknown threshold rule {thr!r}")
            api.gmm_levels(b, self.dirty, levels=self.levels, mu_a=self.mu_a, mu_b=self.mu_b)
            thr = self.mu_a
        self.res = api.hogbom_clean(b, self.dirty, self.beam, self.niter, gain=self.gain, threshold=thr,
                                    positive_only=self.positive_only, restore=self.restore,
                                    team_size=self.team_size, out=self.res)
        if self.adjoint:
            api.degrid(b, self.res["residual"], self.uv, self.w, adjoint=True, out=self.adj)
        return self.res

    def tune(self):
        """Pick the imaging schedule (gridder chunk, transform block) and the CLEAN team size
        with the autotuners; returns (team size, (grid_chunk, fft_elems))."""
        b = self.batch
        self.imaging_tuning = autotune_imaging(b, self.vis, self.uv, self.w)
        api.dirty_image(b, self.vis, self.uv, self.w, beam=True, out=self.dirty, beam_out=self.beam, b0_out=self.b0)
        self.team_size = autotune_team_size(b, self.dirty, self.beam, self.niter, self.gain)
        return self.team_size, self.imaging_tuning

    def capture(self):
        """Warm up (plans, workspaces) and capture one step into a HIP graph."""
        self.step()
        torch.cuda.synchronize()
        s = torch.cuda.Stream(self.dev)
        s.wait_stream(torch.cuda.current_stream(self.dev))
        with torch.cuda.stream(s):
            self.step()
        torch.cuda.current_stream(self.dev).wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()
        return self.res


def improved_clean(wl, radius_px, device="cuda:0", restore: bool = True, team_size: int = 0,
                   deconvolver: str = "hogbom", steer_cycles: int = 200, trim: float = 0.9):
    """Algorithm 1 (improved_clean) over a whole batch, every stage one batched launch:
    dirty map and beam -> sky / disk levels (Sec. 4.1) -> CLEAN to the disk level mu_b ->
    disk offset by correlation with a disk of `radius_px` pixels (Sec. 4.2) -> phase
    correction of the visibilities -> dirty map and beam again -> levels -> CLEAN while the
    peak exceeds the sky level mu_a (Sec. 4.3; positive peaks, loop gain of the workload).
    deconvolver: "hogbom" (the workload's iteration caps) or "steer" (the Steer CLEAN that
    the paper runs in MUSER, at most `steer_cycles` iterations of the given trim).
    Returns (result dict of hogbom_clean or steer_clean, offsets (n, 2) radians, levels
    (n, 6), the corrected visibilities)."""
    if deconvolver not in ("hogbom", "steer"):
        raise ValueError(f"unknown deconvolver {deconvolver!r}")
    dev = torch.device(device)
    b = api.Batch.from_workload(wl, dev)
    vis, uv, w = api.workload_tensors(wl, dev)
    niter = np.ascontiguousarray(wl.niter, np.int32)
    cycles = np.full(b.n_inst, steer_cycles, np.int32)

    def deconvolve(dirty, beam, thr, final):
        if deconvolver == "steer":
            return api.steer_clean(b, dirty, beam, cycles, gain=wl.gain, trim=trim, threshold=thr, positive_only=True,
                                   restore=final and restore, want_model=final)
        return api.hogbom_clean(b, dirty, beam, niter, gain=wl.gain, threshold=thr, positive_only=True,
                                restore=final and restore, want_model=final, want_components=final,
                                team_size=team_size)

    dirty, beam, _ = api.dirty_image(b, vis, uv, w, beam=True)
    _, _, mu_b = api.gmm_levels(b, dirty)
    pre = deconvolve(dirty, beam, mu_b, False)
    offsets = api.disk_offsets(b, pre["residual"], radius_px)
    api.phase_shift(b, vis, uv, offsets)
    dirty, beam, _ = api.dirty_image(b, vis, uv, w, beam=True, out=dirty, beam_out=beam)
    levels, mu_a, _ = api.gmm_levels(b, dirty)
    res = deconvolve(dirty, beam, mu_a, True)
    return res, offsets, levels, vis
