"""GPU parity of gridding, the inverse FFT, dirty image and dirty beam against the FP64 oracle.

Acceptance (from the imaging requirement): max |GPU - oracle| <= 1e-4 * max |oracle image|.
"""
import numpy as np
import pytest
import torch

from oracle import imager, gcf
from paper_1712_06913_amd import synth
from tests.gpu_helpers import log, max_abs, require_gpu

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _api():
    require_gpu()
    from paper_1712_06913_amd import api
    return api


def _image_parity(wl, check_beam=True):
    api = _api()
    b = api.Batch.from_workload(wl)
    vis, uv, w = api.workload_tensors(wl)
    dirty, beam, b0 = api.dirty_image(b, vis, uv, w, beam=check_beam)
    torch.cuda.synchronize()
    dirty_l = [x.cpu().numpy() for x in b.split(dirty)]
    beam_l = [x.cpu().numpy() for x in b.split(beam, beam=True)] if check_beam else None
    b0 = b0.cpu().numpy().reshape(-1, 2)
    status = b.status.cpu().numpy()
    for i in range(wl.n_inst):
        v, uvi, wi = wl.instance(i)
        N, cell, mode = int(wl.n_img[i]), float(wl.cell_rad[i]), int(wl.weight_mode[i])
        ref, parts = imager.dirty_image(v, uvi, wi, N, cell, mode, return_parts=True)
        if parts["prep"].n_kept == 0:
            assert status[i] & 1 and np.all(dirty_l[i] == 0)
            continue
        assert status[i] == 0
        peak = np.max(np.abs(ref))
        err = max_abs(dirty_l[i], ref)
        log(f"  inst {i} N={N} mode={mode} kept={parts['prep'].n_kept} dirty err/peak={err / peak:.2e}")
        assert err <= TOL * peak
        assert abs(b0[i, 0] - parts["b0"]) <= 1e-6 * parts["b0"]
        if check_beam:
            refb, pb = imager.dirty_beam(uvi, wi, N, cell, mode, return_parts=True)
            errb = max_abs(beam_l[i], refb)
            log(f"           beam err={errb:.2e} centre={beam_l[i][N, N]:.7f}")
            assert errb <= TOL
            assert abs(beam_l[i][N, N] - 1.0) < 1e-5
            assert abs(b0[i, 1] - pb["b0"]) <= 1e-6 * pb["b0"]


@pytest.mark.parametrize("seed", [1, 2])
def test_dirty_image_and_beam_small_batch(seed):
    log(f"[imaging] random batch seed={seed}")
    wl = synth.random_instances(seed, [64, 128, 256, 64, 128], m_range=(1, 300))
    _image_parity(wl)


def test_dirty_image_dense_uv_many_tiles():
    # dense, strongly overlapping samples: many entries per tile, ragged tile fill
    log("[imaging] dense uv")
    wl = synth.random_instances(7, [128, 256], m_range=(2000, 3000), fill=0.95)
    _image_parity(wl)


def test_c1_snapshot_full_size():
    log("[imaging] C1 256^2 780 baselines")
    _image_parity(synth.c1_snapshot())


def test_c3_two_channels_1024():
    log("[imaging] C3 slice: 2 channels at 1024^2")
    _image_parity(synth.c3_muser2(chans=[0, 519]))


def test_largest_image_sizes_2048_and_4096():
    # the largest transforms: a 4096^2 beam (P = 4096, one complex line per block) and an
    # 8192^2 beam (P = 8192, the 8192-element LDS blocks)
    log("[imaging] largest sizes: 2048^2 and 4096^2 (beams 4096^2 and 8192^2)")
    wl = synth.random_instances(31, [2048, 4096], m_range=(150, 200))
    _image_parity(wl)


def test_empty_and_flagged_instances():
    log("[imaging] empty instance")
    wl = synth.random_instances(3, [64, 128], m_range=(20, 20))
    wl.w[: int(wl.vis_offset[1])] = 0.0      # first instance fully flagged
    _image_parity(wl)


def test_kept_band_edges_and_nonfinite_uv():
    log("[imaging] samples at the edge of the kept band, near half-cell ties, NaN / inf / huge uv")
    wl = synth.random_instances(5, [128, 256], m_range=(200, 200))
    for i in range(wl.n_inst):
        a = int(wl.vis_offset[i])
        N, sc = int(wl.n_img[i]), int(wl.n_img[i]) * float(wl.cell_rad[i])
        lim = N // 2 - 4                   # largest kept |cell| (support 7 inside the half grid)
        g = [lim, lim + 0.49, lim + 0.5, -(lim + 0.5), lim - 0.5, -lim - 0.4999, lim + 1, -lim]
        pts = [(x, 3.2) for x in g] + [(2.7, y) for y in g]
        pts += [(np.nan, 1.0), (1.0, np.inf), (-np.inf, 0.0), (1e30, 2.0)]
        for k, (x, y) in enumerate(pts):
            wl.uv[a + k] = (np.float32(x / sc), np.float32(y / sc))
    _image_parity(wl)


@pytest.mark.parametrize("which", [0, 1])
def test_grid_full_layout_matches_oracle(which):
    log(f"[grid] full layout which={which}")
    api = _api()
    wl = synth.random_instances(4, [64, 128], m_range=(50, 200))
    b = api.Batch.from_workload(wl)
    vis, uv, w = api.workload_tensors(wl)
    g, b0, nk = api.grid(b, vis, uv, w, which=which)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    off = 0
    for i in range(wl.n_inst):
        v, uvi, wi = wl.instance(i)
        N = int(wl.n_img[i])
        P = N * (2 if which else 1)
        p = imager.Prep(uvi, wi, N, float(wl.cell_rad[i]))
        ref = imager.grid(p, v, imager.weights(p, int(wl.weight_mode[i])), beam=bool(which))
        got = g[off: off + P * P].reshape(P, P)
        off += P * P
        err = max_abs(got.real, ref.real) + max_abs(got.imag, ref.imag)
        assert err <= 1e-5 * np.max(np.abs(ref))
        assert int(nk.cpu().numpy()[i]) == p.n_kept


def test_ifft2_matches_centred_dft():
    log("[ifft2] batched 64/128/512")
    api = _api()
    rng = np.random.default_rng(9)
    sizes = [64, 128, 512]
    arrs = [(rng.standard_normal((P, P)) + 1j * rng.standard_normal((P, P))) for P in sizes]
    offs = np.concatenate([[0], np.cumsum([P * P for P in sizes])[:-1]])
    flat = torch.from_numpy(np.concatenate([a.ravel() for a in arrs]).astype(np.complex64)).cuda()
    api.ifft2(flat, sizes, offs)
    torch.cuda.synchronize()
    out = flat.cpu().numpy()
    for P, a, o in zip(sizes, arrs, offs):
        ref = imager.ifft2_centred(a.astype(np.complex64).astype(np.complex128))
        got = out[o: o + P * P].reshape(P, P)
        assert np.max(np.abs(got - ref)) <= 2e-6 * np.max(np.abs(ref)) * np.log2(P)


def test_beam_is_exactly_point_symmetric():
    log("[imaging] library beams are bitwise point-symmetric about (N, N)")
    require_gpu()
    from paper_1712_06913_amd import api
    wl = synth.random_instances(31, [64, 256, 512], m_range=(150, 400))
    b = api.Batch.from_workload(wl)
    vis, uv, w = api.workload_tensors(wl)
    beams = b.split(api.dirty_beam(b, uv, w), beam=True)
    for i in range(wl.n_inst):
        N = int(wl.n_img[i])
        B = beams[i].cpu().numpy().view(np.uint32).reshape(2 * N, 2 * N)
        assert np.array_equal(B[1:, 1:], B[:0:-1, :0:-1]), f"instance {i} (N={N})"
