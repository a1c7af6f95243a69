"""Python binding of the C ABI (include/mi.h) over torch device tensors.

Only argument marshalling happens here: every step of the imaging path runs in the HIP
library.  Tensors must live on the context's device; calls are enqueued on torch's
current stream and do not synchronise.
"""
from __future__ import annotations

import atexit
import ctypes
from typing import Dict, List, Optional

import numpy as np
import torch

from . import _native as nat

_ctx_cache: Dict[int, ctypes.c_void_p] = {}
_private: List["Context"] = []


def _create(device: int) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    code = nat.lib().mi_ctx_create(ctypes.byref(ctx), device)
    if code != nat.MI_OK:
        raise nat.MiError(code, "mi_ctx_create failed")
    return ctx


def context(device: int = 0) -> ctypes.c_void_p:
    """Per-device shared library context (created on first use, kept until close())."""
    if device not in _ctx_cache:
        _ctx_cache[device] = _create(device)
    return _ctx_cache[device]


class Context:
    """A private library context (its own plans and workspaces), e.g. for a captured graph
    that must not share the process-wide plan cache.  Destroyed by close() or at exit."""

    def __init__(self, device: int = 0):
        self.device = device
        self.handle = _create(device)
        _private.append(self)

    def close(self):
        if self.handle is not None:
            torch.cuda.synchronize(self.device)
            nat.lib().mi_ctx_destroy(self.handle)
            self.handle = None
        if self in _private:
            _private.remove(self)


def close():
    """Synchronise, destroy every library context and release torch's cached device memory.
    Registered at exit, so the library's device memory is gone before the HIP runtime (and any
    profiler attached to it) shuts down."""
    if not nat.loaded():
        return
    if torch.cuda.is_available() and torch.cuda.is_initialized():
        torch.cuda.synchronize()
    for c in list(_private):
        c.close()
    for dev, ctx in list(_ctx_cache.items()):
        nat.lib().mi_ctx_destroy(ctx)
        del _ctx_cache[dev]
    if torch.cuda.is_available() and torch.cuda.is_initialized():
        torch.cuda.empty_cache()


atexit.register(close)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors passed to the library must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Batch:
    """Host-side batch descriptor (mi_batch) plus a device status array."""

    def __init__(self, vis_offset, n_img, cell_rad, weight_mode, device="cuda:0", ctx: Optional[Context] = None):
        self._own_ctx = ctx
        self.vis_offset = np.ascontiguousarray(vis_offset, dtype=np.int64)
        self.n_img = np.ascontiguousarray(n_img, dtype=np.int32)
        self.cell_rad = np.ascontiguousarray(cell_rad, dtype=np.float64)
        self.weight_mode = np.ascontiguousarray(weight_mode, dtype=np.int8)
        self.device = torch.device(device)
        self.n_inst = len(self.n_img)
        self.status = torch.zeros(self.n_inst, dtype=torch.int32, device=self.device)
        self.img_off = np.concatenate([[0], np.cumsum(self.n_img.astype(np.int64) ** 2)])
        self.beam_off = 4 * self.img_off
        self._c = nat.MiBatch(
            self.n_inst, self.vis_offset.ctypes.data, self.n_img.ctypes.data, self.cell_rad.ctypes.data,
            self.weight_mode.ctypes.data, self.status.data_ptr())

    @classmethod
    def from_workload(cls, wl, device="cuda:0", ctx: Optional[Context] = None) -> "Batch":
        return cls(wl.vis_offset, wl.n_img, wl.cell_rad, wl.weight_mode, device, ctx)

    @property
    def c(self):
        return ctypes.byref(self._c)

    @property
    def ctx(self):
        if self._own_ctx is not None:
            if self._own_ctx.handle is None:
                raise RuntimeError("the batch's library context was closed")
            return self._own_ctx.handle
        return context(self.device.index or 0)

    def split(self, flat: torch.Tensor, beam: bool = False):
        """Views of a packed per-instance image array as a list of (P, P) tensors."""
        off = self.beam_off if beam else self.img_off
        out = []
        for i in range(self.n_inst):
            P = int(self.n_img[i]) * (2 if beam else 1)
            out.append(flat[off[i]: off[i] + P * P].view(P, P))
        return out


def workload_tensors(wl, device="cuda:0"):
    """Device copies (vis complex64, uv float32 [M,2], w float32) of a synthetic workload."""
    dev = torch.device(device)
    vis = torch.from_numpy(np.ascontiguousarray(wl.vis)).to(dev)
    uv = torch.from_numpy(np.ascontiguousarray(wl.uv)).to(dev)
    w = torch.from_numpy(np.ascontiguousarray(wl.w)).to(dev)
    return vis, uv, w


def dirty_image(batch: Batch, vis, uv, w, beam: bool = True, out=None, beam_out=None, b0_out=None):
    """mi_dirty_image: packed float32 dirty images (and beams), plus B0 per instance."""
    dev = batch.device
    out = torch.empty(int(batch.img_off[-1]), dtype=torch.float32, device=dev) if out is None else out
    if beam and beam_out is None:
        beam_out = torch.empty(int(batch.beam_off[-1]), dtype=torch.float32, device=dev)
    b0_out = torch.empty(2 * batch.n_inst, dtype=torch.float64, device=dev) if b0_out is None else b0_out
    nat.check(batch.ctx, nat.lib().mi_dirty_image(batch.ctx, batch.c, _ptr(vis), _ptr(uv), _ptr(w), _ptr(out),
                                                  _ptr(beam_out if beam else None), _ptr(b0_out), _stream(dev)))
    return out, (beam_out if beam else None), b0_out


def dirty_image_w(batch: Batch, vis, uv, w_lambda, w, w_max, phase_tol: float = 0.1, out=None, b0_out=None):
    """mi_dirty_image_w: dirty images with w-projection; returns (images, B0, planes per instance).
    `w_max`: host array, a bound on |w| per instance (wavelengths)."""
    dev = batch.device
    out = torch.empty(int(batch.img_off[-1]), dtype=torch.float32, device=dev) if out is None else out
    b0_out = torch.empty(2 * batch.n_inst, dtype=torch.float64, device=dev) if b0_out is None else b0_out
    wm = np.ascontiguousarray(w_max, dtype=np.float64)
    if wm.shape != (batch.n_inst,):
        raise ValueError("w_max: one value per instance")
    n_planes = np.zeros(batch.n_inst, np.int32)
    prm = nat.MiWprojParams(wm.ctypes.data, float(phase_tol))
    nat.check(batch.ctx, nat.lib().mi_dirty_image_w(batch.ctx, batch.c, _ptr(vis), _ptr(uv), _ptr(w_lambda), _ptr(w),
                                                    ctypes.byref(prm), _ptr(out), _ptr(b0_out), n_planes.ctypes.data,
                                                    _stream(dev)))
    return out, b0_out, n_planes


def dirty_beam(batch: Batch, uv, w, out=None):
    dev = batch.device
    out = torch.empty(int(batch.beam_off[-1]), dtype=torch.float32, device=dev) if out is None else out
    nat.check(batch.ctx, nat.lib().mi_dirty_beam(batch.ctx, batch.c, _ptr(uv), _ptr(w), _ptr(out), _stream(dev)))
    return out


def grid(batch: Batch, vis, uv, w, which: int = 0, layout: int = nat.MI_LAYOUT_FULL, out=None):
    """mi_grid: packed complex64 grids; returns (grid, b0 [n,2] float64, n_kept int32)."""
    dev = batch.device
    n = batch.n_img.astype(np.int64)
    per_full = {0: n * n, 1: 4 * n * n}
    per_half = {0: n * n // 2, 1: 2 * n * n}
    per = per_full if layout == nat.MI_LAYOUT_FULL else per_half
    total = int(per[0].sum() * (which != 1) + per[1].sum() * (which != 0))
    out = torch.empty(total, dtype=torch.complex64, device=dev) if out is None else out
    b0 = torch.empty(2 * batch.n_inst, dtype=torch.float64, device=dev)
    nk = torch.empty(batch.n_inst, dtype=torch.int32, device=dev)
    nat.check(batch.ctx, nat.lib().mi_grid(batch.ctx, batch.c, _ptr(vis), _ptr(uv), _ptr(w), which, layout,
                                           _ptr(out), _ptr(b0), _ptr(nk), _stream(dev)))
    return out, b0, nk


def ifft2(data: torch.Tensor, n, offs, device: int = 0):
    """mi_ifft2 in place on a packed complex64 tensor."""
    n = np.ascontiguousarray(n, dtype=np.int32)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    ctx = context(device)
    nat.check(ctx, nat.lib().mi_ifft2(ctx, _ptr(data), n.ctypes.data, offs.ctypes.data, len(n),
                                      _stream(data.device)))
    return data


def hogbom_clean(batch: Batch, dirty, beam, niter, gain: float = 0.1, threshold=None, positive_only=False,
                 restore: bool = True, want_model: bool = True, want_components: bool = True, team_size: int = 0,
                 out=None, window=None, no_alloc: bool = False):
    """mi_hogbom_clean; returns a dict of device tensors (reused when `out` is a previous result).

    `threshold`: None, a host array (one per instance), or a float32 device tensor (read on
    the device, e.g. the mu_a of gmm_levels).  `window`: None (whole maps) or an
    [n_inst, 4] array of peak-search boxes (x0, y0, x1, y1), half-open.  `no_alloc`: call
    mi_hogbom_clean_noalloc, which works in the library's fixed device scratch array (one
    image size per batch, at most 64 instances, no windows)."""
    dev = batch.device
    niter = np.ascontiguousarray(niter, dtype=np.int32)
    thr_dev = None
    if torch.is_tensor(threshold) and threshold.is_cuda:
        if threshold.dtype != torch.float32 or threshold.numel() != batch.n_inst:
            raise ValueError("device thresholds must be float32, one per instance")
        thr_dev, thr = threshold.contiguous(), None
    else:
        thr = None if threshold is None else np.ascontiguousarray(threshold, dtype=np.float32)
    win = None if window is None else np.ascontiguousarray(window, dtype=np.int32).reshape(batch.n_inst, 4)
    nimg = int(batch.img_off[-1])
    ncomp_total = max(1, int(niter.sum()))
    res = out
    if res is None:
        res = {"residual": torch.empty(nimg, dtype=torch.float32, device=dev)}
        res["model"] = torch.empty(nimg, dtype=torch.float64, device=dev) if want_model else None
        if want_components:
            res["comp_idx"] = torch.full((ncomp_total,), -1, dtype=torch.int32, device=dev)
            res["comp_flux"] = torch.zeros(ncomp_total, dtype=torch.float64, device=dev)
        else:
            res["comp_idx"] = res["comp_flux"] = None
        res["n_comp"] = torch.zeros(batch.n_inst, dtype=torch.int32, device=dev)
        res["restored"] = torch.empty(nimg, dtype=torch.float32, device=dev) if restore else None
        res["cbeam"] = torch.zeros(6 * batch.n_inst, dtype=torch.float64, device=dev) if restore else None
        res["comp_off"] = np.concatenate([[0], np.cumsum(niter.astype(np.int64))])
    prm = nat.MiCleanParams(float(gain), niter.ctypes.data, None if thr is None else thr.ctypes.data,
                            1 if positive_only else 0, int(team_size),
                            None if thr_dev is None else thr_dev.data_ptr(),
                            None if win is None else win.ctypes.data)
    fn = nat.lib().mi_hogbom_clean_noalloc if no_alloc else nat.lib().mi_hogbom_clean
    nat.check(batch.ctx, fn(
        batch.ctx, batch.c, _ptr(dirty), _ptr(beam), ctypes.byref(prm), _ptr(res["residual"]), _ptr(res["model"]),
        _ptr(res["comp_idx"]), _ptr(res["comp_flux"]), _ptr(res["n_comp"]), _ptr(res["restored"]),
        _ptr(res["cbeam"]), _stream(dev)))
    return res


def steer_clean(batch: Batch, dirty, beam, ncycle, gain: float = 0.1, trim: float = 0.9, threshold=None,
                positive_only=False, restore: bool = True, want_model: bool = True, want_log: bool = True,
                want_masks: bool = False, out=None):
    """mi_steer_clean; returns a dict of device tensors (reused when `out` is a previous result):
    residual, model, n_cycle, log ([sum ncycle, 3]: peak, alpha, selected), masks (uint32 bit
    masks per iteration, when asked), restored, cbeam; `log_off` / `mask_off` index them."""
    dev = batch.device
    ncycle = np.ascontiguousarray(ncycle, dtype=np.int32)
    thr_dev = None
    if torch.is_tensor(threshold) and threshold.is_cuda:
        if threshold.dtype != torch.float32 or threshold.numel() != batch.n_inst:
            raise ValueError("device thresholds must be float32, one per instance")
        thr_dev, thr = threshold.contiguous(), None
    else:
        thr = None if threshold is None else np.ascontiguousarray(threshold, dtype=np.float32)
    nimg = int(batch.img_off[-1])
    res = out
    if res is None:
        words = ncycle.astype(np.int64) * batch.n_img.astype(np.int64) ** 2 // 32
        res = {"residual": torch.empty(nimg, dtype=torch.float32, device=dev),
               "model": torch.empty(nimg, dtype=torch.float64, device=dev) if want_model else None,
               "n_cycle": torch.zeros(batch.n_inst, dtype=torch.int32, device=dev),
               "log": torch.zeros(max(1, int(ncycle.sum())) * 3, dtype=torch.float64, device=dev) if want_log else None,
               "masks": torch.zeros(max(1, int(words.sum())), dtype=torch.int32, device=dev) if want_masks else None,
               "restored": torch.empty(nimg, dtype=torch.float32, device=dev) if restore else None,
               "cbeam": torch.zeros(6 * batch.n_inst, dtype=torch.float64, device=dev) if restore else None,
               "log_off": np.concatenate([[0], np.cumsum(ncycle.astype(np.int64))]),
               "mask_off": np.concatenate([[0], np.cumsum(words)])}
    prm = nat.MiSteerParams(float(gain), float(trim), ncycle.ctypes.data, None if thr is None else thr.ctypes.data,
                            None if thr_dev is None else thr_dev.data_ptr(), 1 if positive_only else 0)
    nat.check(batch.ctx, nat.lib().mi_steer_clean(
        batch.ctx, batch.c, _ptr(dirty), _ptr(beam), ctypes.byref(prm), _ptr(res["residual"]), _ptr(res["model"]),
        _ptr(res["n_cycle"]), _ptr(res["log"]), _ptr(res["masks"]), _ptr(res["restored"]), _ptr(res["cbeam"]),
        _stream(dev)))
    return res


def steer_masks(res, batch: Batch, i: int, n: int):
    """Selection masks of instance i's first n iterations as bool [n, N, N] (host)."""
    N = int(batch.n_img[i])
    w = N * N // 32
    words = res["masks"][int(res["mask_off"][i]): int(res["mask_off"][i]) + n * w].cpu().numpy()
    bits = np.unpackbits(words.view(np.uint8), bitorder="little")
    return bits.reshape(n, N, N).astype(bool)


def degrid(batch: Batch, image, uv, w, adjoint: bool = False, out=None):
    """mi_degrid: prediction P(y) (adjoint=False) or A^T y (adjoint=True), complex64 per visibility."""
    dev = batch.device
    m = int(batch.vis_offset[-1])
    out = torch.empty(m, dtype=torch.complex64, device=dev) if out is None else out
    nat.check(batch.ctx, nat.lib().mi_degrid(batch.ctx, batch.c, _ptr(image), _ptr(uv), _ptr(w),
                                             1 if adjoint else 0, _ptr(out), _stream(dev)))
    return out


def predict_transpose(batch: Batch, vis, uv, w, out=None):
    """mi_predict_transpose: P^T v (the transpose of degrid(adjoint=False)), float32 images."""
    dev = batch.device
    out = torch.empty(int(batch.img_off[-1]), dtype=torch.float32, device=dev) if out is None else out
    nat.check(batch.ctx, nat.lib().mi_predict_transpose(batch.ctx, batch.c, _ptr(vis), _ptr(uv), _ptr(w), _ptr(out),
                                                        _stream(dev)))
    return out


def gmm_levels(batch: Batch, images, n_bins: int = 2000, n_iter: int = 500, levels=None, mu_a=None, mu_b=None):
    """mi_gmm_levels: (levels [n_inst, 6] float64, mu_a float32 [n_inst], mu_b float32 [n_inst])."""
    dev = batch.device
    n = batch.n_inst
    levels = torch.empty(6 * n, dtype=torch.float64, device=dev) if levels is None else levels
    mu_a = torch.empty(n, dtype=torch.float32, device=dev) if mu_a is None else mu_a
    mu_b = torch.empty(n, dtype=torch.float32, device=dev) if mu_b is None else mu_b
    nat.check(batch.ctx, nat.lib().mi_gmm_levels(batch.ctx, batch.c, _ptr(images), int(n_bins), int(n_iter),
                                                 _ptr(levels), _ptr(mu_a), _ptr(mu_b), _stream(dev)))
    return levels.view(n, 6), mu_a, mu_b


def disk_offsets(batch: Batch, images, radius_px, out=None):
    """mi_disk_offsets: (n_inst, 2) float64 device tensor of (dl, dm) in radians."""
    dev = batch.device
    r = np.ascontiguousarray(radius_px, dtype=np.float64)
    out = torch.empty(2 * batch.n_inst, dtype=torch.float64, device=dev) if out is None else out
    nat.check(batch.ctx, nat.lib().mi_disk_offsets(batch.ctx, batch.c, _ptr(images), r.ctypes.data_as(ctypes.c_void_p),
                                                   _ptr(out), _stream(dev)))
    return out.view(batch.n_inst, 2)


def phase_shift(batch: Batch, vis, uv, offsets):
    """mi_phase_shift: vis *= exp(+2 pi i (u dl + v dm)) in place; offsets (n_inst, 2) float64 on the device."""
    dev = batch.device
    nat.check(batch.ctx, nat.lib().mi_phase_shift(batch.ctx, batch.c, _ptr(vis), _ptr(uv), _ptr(offsets.contiguous()),
                                                  _stream(dev)))
    return vis


def set_tuning(ctx, grid_chunk: int = 0, fft_elems: int = 0):
    """mi_set_tuning on a context handle (e.g. batch.ctx): gridder tiles per workgroup and
    transform points per workgroup (0 = the library's defaults)."""
    nat.check(ctx, nat.lib().mi_set_tuning(ctx, ctypes.byref(nat.MiTuning(int(grid_chunk), int(fft_elems)))))


def get_tuning(ctx):
    """(grid_chunk, fft_elems) in use on a context handle."""
    t = nat.MiTuning()
    nat.check(ctx, nat.lib().mi_get_tuning(ctx, ctypes.byref(t)))
    return int(t.grid_chunk), int(t.fft_elems)


def profile_begin(device: int = 0, kinds: int = nat.MI_PROF_CLEAN):
    """mi_profile_begin_kinds: record HIP events around every following launch of the kernel
    kinds in the mask (MI_PROF_CLEAN: the Hogbom kernel; MI_PROF_GRID: the FP64 gridders;
    MI_PROF_IFFT: the inverse transform passes)."""
    ctx = context(device)
    nat.check(ctx, nat.lib().mi_profile_begin_kinds(ctx, kinds))


def profile_end_kinds(device: int = 0, cap: int = 4096):
    """mi_profile_end_kinds: (durations in milliseconds, kinds), oldest first."""
    ctx = context(device)
    buf = (ctypes.c_float * cap)()
    kb = (ctypes.c_int32 * cap)()
    n = ctypes.c_int32()
    nat.check(ctx, nat.lib().mi_profile_end_kinds(ctx, buf, kb, cap, ctypes.byref(n)))
    m = min(n.value, cap)
    return [float(buf[i]) for i in range(m)], [int(kb[i]) for i in range(m)]


def profile_end(device: int = 0, cap: int = 1024):
    """mi_profile_end: the recorded kernel durations in milliseconds (oldest first)."""
    return profile_end_kinds(device, cap)[0]
