"""GPU parity of w-projection (Sec. 3.2.2, 6.1) against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import imager, wproj
from paper_1712_06913_amd import synth
from tests.gpu_helpers import log, max_abs, require_gpu

pytestmark = pytest.mark.gpu


def _w_max(wl):
    return np.array([float(np.abs(wl.instance_w(i).astype(np.float64)).max()) for i in range(wl.n_inst)])


def _gpu(wl, w_max, tol=0.1):
    from paper_1712_06913_amd import api
    b = api.Batch.from_workload(wl)
    vis, uv, w = api.workload_tensors(wl)
    wlam = torch.from_numpy(np.ascontiguousarray(wl.w_lambda)).cuda()
    img, b0, n_planes = api.dirty_image_w(b, vis, uv, wlam, w, w_max, phase_tol=tol)
    torch.cuda.synchronize()
    return b, b.split(img), b0.cpu().numpy(), n_planes


def test_wproj_dirty_images_match_oracle():
    log("[wproj] w-projected dirty images vs the oracle (128/256, |w| up to ~6e3)")
    require_gpu()
    wl = synth.wterm_points(seed=11, n=3, sizes=(128, 256, 128), freq_hz=0.4e9)
    w_max = _w_max(wl)
    b, imgs, b0, n_planes = _gpu(wl, w_max)
    for i in range(wl.n_inst):
        v, uv, w_in = wl.instance(i)
        N, cell = int(wl.n_img[i]), float(wl.cell_rad[i])
        ref, (dw, np_ref, sup) = wproj.dirty_image_w(v, uv, wl.instance_w(i), w_in, N, cell, 0, w_max[i])
        got = imgs[i].cpu().numpy()
        err = max_abs(got, ref)
        log(f"  inst {i} N={N}: planes gpu {n_planes[i]} oracle {np_ref}, max support {sup[-1]}, "
            f"max|err| {err:.3e} of peak {np.abs(ref).max():.3e}")
        assert n_planes[i] == np_ref and np_ref > 10
        assert err <= 1e-5 * np.abs(ref).max()


def test_wproj_zero_w_is_one_plane_and_matches_oracle():
    log("[wproj] w = 0: a single plane")
    require_gpu()
    wl = synth.wterm_points(seed=12, n=2, sizes=(64, 128), freq_hz=0.4e9)
    wl.w_lambda = np.zeros_like(wl.w_lambda)
    b, imgs, b0, n_planes = _gpu(wl, np.zeros(wl.n_inst))
    assert list(n_planes) == [1, 1]
    for i in range(wl.n_inst):
        v, uv, w_in = wl.instance(i)
        N, cell = int(wl.n_img[i]), float(wl.cell_rad[i])
        ref, _ = wproj.dirty_image_w(v, uv, wl.instance_w(i), w_in, N, cell, 0, 0.0)
        assert max_abs(imgs[i].cpu().numpy(), ref) <= 1e-5 * np.abs(ref).max()


def test_wproj_is_close_to_the_exact_w_term_image():
    log("[wproj] GPU image vs the exact direct transform with the w-term (method accuracy)")
    require_gpu()
    wl = synth.wterm_points(seed=13, n=1, sizes=(128,), freq_hz=0.4e9)
    # only visibilities whose widened kernels fit inside the grid (edge taps are dropped,
    # which truncates the kernel: a property of the grid size, not of the w-correction)
    g = np.abs(wl.uv.astype(np.float64) * (128 * float(wl.cell_rad[0])))
    wl.w = np.where(np.all(g <= 64 - 12, axis=1), wl.w, 0.0).astype(np.float32)
    w_max = _w_max(wl)
    b, imgs, _, _ = _gpu(wl, w_max, tol=0.02)
    v, uv, w_in = wl.instance(0)
    N, cell = 128, float(wl.cell_rad[0])
    prep = imager.Prep(uv, w_in, N, cell)
    w = imager.weights(prep, 0)
    exact = wproj.exact_dirty(v, uv, wl.instance_w(0), w, prep.keep, N, cell)
    img2d = imager.dirty_image(v, uv, w_in, N, cell, 0)
    # away from the outer eighth of the map, where gridding itself (at any w) departs from
    # the direct transform (aliased sidelobes of bright sources, amplified by the correction)
    inner = (slice(N // 8, N - N // 8), slice(N // 8, N - N // 8))
    ew = np.abs(imgs[0].cpu().numpy() - exact)[inner].max()
    e2 = np.abs(img2d - exact)[inner].max()
    log(f"  max|err| vs exact: w-projection {ew:.3e}, 2-D imaging {e2:.3e}")
    assert ew < 0.05 * e2


def test_wproj_rejects_bad_arguments():
    log("[wproj] argument errors")
    require_gpu()
    from paper_1712_06913_amd import api, _native as nat
    wl = synth.wterm_points(seed=14, n=1, sizes=(64,), freq_hz=0.4e9)
    with pytest.raises(nat.MiError):
        _gpu(wl, np.array([-1.0]))
    with pytest.raises(nat.MiError):
        _gpu(wl, np.array([float("nan")]))


def test_wproj_mixed_sizes_and_uniform_weighting():
    log("[wproj] mixed N (plane groups per (N, cell)) and uniform weighting vs the oracle")
    require_gpu()
    wl = synth.wterm_points(seed=15, n=4, sizes=(64, 128, 256, 128), freq_hz=0.3e9)
    wl.weight_mode = np.array([1, 0, 1, 1], np.int8)
    w_max = _w_max(wl)
    w_max[3] *= 1.5                      # a looser bound: more planes for the same group
    b, imgs, b0, n_planes = _gpu(wl, w_max)
    for i in range(wl.n_inst):
        v, uv, w_in = wl.instance(i)
        N, cell, mode = int(wl.n_img[i]), float(wl.cell_rad[i]), int(wl.weight_mode[i])
        ref, (dw, np_ref, sup) = wproj.dirty_image_w(v, uv, wl.instance_w(i), w_in, N, cell, mode, w_max[i])
        err = max_abs(imgs[i].cpu().numpy(), ref)
        log(f"  inst {i} N={N} mode={mode}: planes {n_planes[i]} / {np_ref}, max|err| {err:.3e}")
        assert n_planes[i] == np_ref
        assert err <= 1e-5 * np.abs(ref).max()


@pytest.mark.parametrize("chan", [0, 130])
def test_wproj_c3_channel_at_1024_with_the_arrays_own_w(chan):
    """A C3 channel at its full size (1024^2) with the MUSER-II-like array's own w coordinates,
    w_max over the kept visibilities as in the benchmark (60+ planes, supports up to 15 cells)."""
    log(f"[wproj] C3 channel {chan} at 1024^2 with the array's w")
    require_gpu()
    wl = synth.c3_muser2(chans=[chan])
    wl.w_lambda = synth.c3_w_lambda(chans=[chan])
    v, uv, w_in = wl.instance(0)
    N, cell = int(wl.n_img[0]), float(wl.cell_rad[0])
    keep = imager.Prep(uv, w_in, N, cell).keep
    w_max = np.array([float(np.abs(wl.w_lambda[keep].astype(np.float64)).max())])
    b, imgs, b0, n_planes = _gpu(wl, w_max)
    ref, (dw, np_ref, sup) = wproj.dirty_image_w(v, uv, wl.instance_w(0), w_in, N, cell, 0, w_max[0])
    err = max_abs(imgs[0].cpu().numpy(), ref)
    log(f"  planes gpu {n_planes[0]} oracle {np_ref}, largest support {max(sup)} cells, "
        f"max|err| {err:.3e} of peak {np.abs(ref).max():.3e}")
    assert n_planes[0] == np_ref and np_ref >= 60
    assert err <= 1e-5 * np.abs(ref).max()
