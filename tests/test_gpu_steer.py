"""GPU parity of Steer CLEAN (mi_steer_clean) against the FP64 oracle.

Which pixels pass the trim is decided in floating point, so the GPU's own selections (bit
masks per iteration) are validated by the oracle's replay: every selected pixel at least
trim x peak - eps and every other one below trim x peak + eps, peak within eps of the FP64
peak, alpha within 1e-4 (relative), eps = 1e-5 max|dirty|.  Maps: residual and restored within
1e-4 of the dirty peak, model within 1e-5, against the replay's FP64 maps.  Where the
selection is unique (closed forms) the GPU result is compared directly.
"""
import numpy as np
import pytest
import torch

from oracle import clean, imager, steer
from paper_1712_06913_amd import synth
from tests.gpu_helpers import log, max_abs, require_gpu

pytestmark = pytest.mark.gpu


def _inputs(wl):
    dirty, beams = [], []
    for i in range(wl.n_inst):
        v, uv, w = wl.instance(i)
        N, cell, mode = int(wl.n_img[i]), float(wl.cell_rad[i]), int(wl.weight_mode[i])
        dirty.append(imager.dirty_image(v, uv, w, N, cell, mode).astype(np.float32))
        beams.append(imager.dirty_beam(uv, w, N, cell, mode).astype(np.float32))
    return dirty, beams


def _run(wl, ncycle, inputs, **kw):
    require_gpu()
    from paper_1712_06913_amd import api
    dirty, beams = inputs
    b = api.Batch.from_workload(wl)
    d_t = torch.from_numpy(np.concatenate([x.ravel() for x in dirty])).cuda()
    b_t = torch.from_numpy(np.concatenate([x.ravel() for x in beams])).cuda()
    res = api.steer_clean(b, d_t, b_t, ncycle, want_masks=True, **kw)
    torch.cuda.synchronize()
    return api, b, res


def _check(wl, ncycle, inputs, gain=0.1, trim=0.9, threshold=None, positive_only=False):
    api, b, res = _run(wl, ncycle, inputs, gain=gain, trim=trim, threshold=threshold, positive_only=positive_only)
    dirty, beams = inputs
    nc = res["n_cycle"].cpu().numpy()
    lg = res["log"].cpu().numpy().reshape(-1, 3)
    resid, model, restored = b.split(res["residual"]), b.split(res["model"]), b.split(res["restored"])
    for i in range(wl.n_inst):
        D, B = dirty[i].astype(np.float64), beams[i].astype(np.float64)
        n = int(nc[i])
        L = lg[res["log_off"][i]: res["log_off"][i] + n]
        masks = api.steer_masks(res, b, i, n)
        thr = 0.0 if threshold is None else float(threshold[i])
        ok, bad, R, M = steer.replay(D, B, masks, L[:, 0], L[:, 1], L[:, 2], gain=gain, trim=trim, threshold=thr,
                                     positive_only=positive_only, ncycle=int(ncycle[i]))
        peak = float(np.max(np.abs(D)))
        log(f"  inst {i} N={D.shape[0]} cycles {n}/{int(ncycle[i])} selected {L[:, 2].astype(int).tolist()[:8]}... "
            f"replay ok={ok}")
        assert ok, f"inst {i}: iteration {bad} rejected by the replay"
        assert all(int(m.sum()) == int(c) for m, c in zip(masks, L[:, 2]))
        assert max_abs(resid[i].cpu().numpy(), R) <= 1e-4 * peak
        assert max_abs(model[i].cpu().numpy(), M) <= 1e-5 * peak
        rest = clean.restore_conv(R, M, clean.fit_clean_beam(B))
        assert max_abs(restored[i].cpu().numpy(), rest) <= 1e-4 * peak
    return res


def test_steer_mixed_sizes_match_oracle():
    log("[steer] mixed 64/128/256 batch, trim 0.9 and 0.7")
    wl = synth.random_instances(81, [64, 128, 256], m_range=(150, 300))
    inputs = _inputs(wl)
    _check(wl, np.array([12, 20, 25], np.int32), inputs)
    _check(wl, np.array([10, 10, 10], np.int32), inputs, trim=0.7)


def test_steer_positive_only_and_thresholds():
    log("[steer] positive-only selection; host and device thresholds stop early")
    wl = synth.random_instances(82, [128, 128], m_range=(150, 300))
    inputs = _inputs(wl)
    _check(wl, np.array([15, 15], np.int32), inputs, positive_only=True)
    thr = np.array([0.4 * np.max(np.abs(d)) for d in inputs[0]], np.float32)
    res = _check(wl, np.array([200, 200], np.int32), inputs, threshold=thr)
    assert np.all(res["n_cycle"].cpu().numpy() < 200)
    from paper_1712_06913_amd import api
    b = api.Batch.from_workload(wl)
    d_t = torch.from_numpy(np.concatenate([x.ravel() for x in inputs[0]])).cuda()
    b_t = torch.from_numpy(np.concatenate([x.ravel() for x in inputs[1]])).cuda()
    r2 = api.steer_clean(b, d_t, b_t, np.array([200, 200], np.int32), threshold=torch.from_numpy(thr).cuda())
    torch.cuda.synchronize()
    assert torch.equal(r2["n_cycle"], res["n_cycle"])


def test_steer_c3_channel_at_1024():
    log("[steer] one C3 channel at 1024^2 (limb-brightened disk and sources), 30 iterations, trim 0.9")
    wl = synth.c3_muser2(chans=[5], niter=30)
    _check(wl, np.array([30], np.int32), _inputs(wl))


def test_steer_trim_one_is_a_hogbom_step():
    """trim = 1 selects the peak alone and alpha = gain: the GPU's Steer run equals its Hogbom
    run (FFT convolution against direct subtraction: equal to rounding)."""
    log("[steer] trim 1 against the GPU Hogbom CLEAN")
    wl = synth.random_instances(83, [128], m_range=(200, 200))
    inputs = _inputs(wl)
    api, b, res = _run(wl, np.array([25], np.int32), inputs, trim=1.0)
    lg = res["log"].cpu().numpy().reshape(-1, 3)
    assert np.all(lg[:, 2] == 1) and np.allclose(lg[:, 1], 0.1, rtol=1e-6)
    d_t = torch.from_numpy(inputs[0][0].ravel()).cuda()
    b_t = torch.from_numpy(inputs[1][0].ravel()).cuda()
    hog = api.hogbom_clean(b, d_t, b_t, np.array([25], np.int32))
    torch.cuda.synchronize()
    masks = api.steer_masks(res, b, 0, 25)
    picks = [int(np.flatnonzero(m)[0]) for m in masks]
    assert picks == hog["comp_idx"].cpu().numpy().tolist()
    peak = float(np.max(np.abs(inputs[0][0])))
    assert float((res["residual"] - hog["residual"]).abs().max()) <= 1e-5 * peak
    assert float((res["model"] - hog["model"]).abs().max()) <= 1e-6 * peak


def test_steer_closed_forms():
    log("[steer] lone point: S (1 - (1 - g)^n); flat patch under a delta beam: (1 - g)^n")
    require_gpu()
    from paper_1712_06913_amd import api
    N, S, py, px, g, n = 128, 2.5, 41, 90, 0.1, 20
    yy, xx = np.mgrid[0:2 * N, 0:2 * N]
    B = np.exp(-((xx - N) ** 2 + (yy - N) ** 2) / 0.5).astype(np.float32)
    D = (S * B[N - py: 2 * N - py, N - px: 2 * N - px]).astype(np.float32)
    wl = synth.random_instances(84, [N], m_range=(10, 10))
    b = api.Batch.from_workload(wl)
    res = api.steer_clean(b, torch.from_numpy(D.ravel()).cuda(), torch.from_numpy(B.ravel()).cuda(), [n], gain=g,
                          trim=0.5)
    torch.cuda.synchronize()
    M = res["model"].cpu().numpy().reshape(N, N)
    assert abs(M[py, px] - S * (1 - (1 - g) ** n)) <= 1e-5 * S and np.count_nonzero(M) == 1
    R = res["residual"].cpu().numpy().reshape(N, N)
    assert max_abs(R, S * (1 - g) ** n * B[N - py: 2 * N - py, N - px: 2 * N - px]) <= 1e-5 * S
    # flat source, delta beam: every patch pixel is selected each time and decays geometrically
    B = np.zeros((2 * N, 2 * N), np.float32)
    B[N, N] = 1.0
    D = np.zeros((N, N), np.float32)
    D[30:50, 10:70] = 3.0
    res = api.steer_clean(b, torch.from_numpy(D.ravel()).cuda(), torch.from_numpy(B.ravel()).cuda(), [12], gain=g)
    torch.cuda.synchronize()
    lg = res["log"].cpu().numpy().reshape(-1, 3)
    assert np.all(lg[:, 2] == 20 * 60)
    R = res["residual"].cpu().numpy().reshape(N, N)
    assert max_abs(R, D.astype(np.float64) * (1 - g) ** 12) <= 1e-5 * 3.0


def test_steer_zero_cycles_and_zero_map():
    log("[steer] ncycle 0 keeps the dirty map; an all-zero map stops at once")
    wl = synth.random_instances(85, [64, 64], m_range=(100, 200))
    dirty, beams = _inputs(wl)
    dirty[1] = np.zeros_like(dirty[1])
    api, b, res = _run(wl, np.array([0, 10], np.int32), (dirty, beams))
    assert res["n_cycle"].cpu().numpy().tolist() == [0, 0]
    rs = b.split(res["residual"])
    assert np.array_equal(rs[0].cpu().numpy(), dirty[0]) and not np.any(rs[1].cpu().numpy())
    assert not np.any(res["model"].cpu().numpy())


def test_steer_rejects_bad_arguments():
    log("[steer] argument errors")
    require_gpu()
    from paper_1712_06913_amd import api, _native as nat
    wl = synth.random_instances(86, [64], m_range=(50, 60))
    dirty, beams = _inputs(wl)
    b = api.Batch.from_workload(wl)
    d_t = torch.from_numpy(dirty[0].ravel()).cuda()
    b_t = torch.from_numpy(beams[0].ravel()).cuda()
    for kw in ({"trim": 0.0}, {"trim": 1.5}, {"gain": 0.0}):
        with pytest.raises(nat.MiError):
            api.steer_clean(b, d_t, b_t, [5], **kw)
    with pytest.raises(nat.MiError):
        api.steer_clean(b, d_t, b_t, [-1])


@pytest.mark.parametrize("N", [2048, 4096])
def test_steer_large_images_lone_point_closed_form(N):
    """Sizes whose transforms use the 4096- and 8192-point workgroups: a lone point under a
    Gaussian beam gives model S (1 - (1 - g)^n) at the point and residual S (1 - g)^n x the
    beam window (trim 0.5 selects the point alone)."""
    log(f"[steer] lone point at {N}^2 (transform length {2 * N}), closed form")
    require_gpu()
    from paper_1712_06913_amd import api
    S, g, n = 2.5, 0.1, 6
    py, px = N // 3, (2 * N) // 3 + 5
    ax = np.arange(2 * N, dtype=np.float64) - N
    B = np.exp(-(ax[None, :] ** 2 + ax[:, None] ** 2) / 0.5).astype(np.float32)
    D = (S * B[N - py: 2 * N - py, N - px: 2 * N - px]).astype(np.float32)
    wl = synth.random_instances(87, [N], m_range=(10, 10))
    b = api.Batch.from_workload(wl)
    res = api.steer_clean(b, torch.from_numpy(D.ravel()).cuda(), torch.from_numpy(B.ravel()).cuda(), [n], gain=g,
                          trim=0.5)
    torch.cuda.synchronize()
    assert int(res["n_cycle"][0]) == n
    M = res["model"].cpu().numpy().reshape(N, N)
    assert abs(M[py, px] - S * (1 - (1 - g) ** n)) <= 1e-5 * S and np.count_nonzero(M) == 1
    R = res["residual"].cpu().numpy().reshape(N, N)
    assert max_abs(R, S * (1 - g) ** n * B[N - py: 2 * N - py, N - px: 2 * N - px].astype(np.float64)) <= 1e-5 * S


def test_steer_2048_matches_oracle_replay():
    """A random 2048^2 instance (its 4096-point transforms) against the oracle's replay."""
    log("[steer] random 2048^2 instance, 6 iterations, replay")
    wl = synth.random_instances(88, [2048], m_range=(300, 300))
    _check(wl, np.array([6], np.int32), _inputs(wl))


def test_steer_mixed_64_to_2048_in_one_batch():
    """One batch mixing 64^2 (32 columns per column workgroup), 512^2 and 2048^2 (two per
    workgroup, 4096-point blocks for every size): every instance against the oracle's replay."""
    log("[steer] mixed 64 / 512 / 2048 batch, 5 iterations, replay")
    wl = synth.random_instances(89, [64, 512, 2048], m_range=(200, 300))
    _check(wl, np.array([5, 5, 5], np.int32), _inputs(wl))
