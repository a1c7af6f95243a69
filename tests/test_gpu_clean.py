"""GPU parity of Hogbom CLEAN, the clean-beam fit and restore against the FP64 oracle.

Inputs are oracle-made dirty images and beams rounded to float32 (identical bytes for both
sides).  Components must agree exactly where the picks are tie-free; in general every GPU
pick is validated by the oracle's replay (a pick is correct if it is within 1e-5 of the
peak of the FP64 residual at that step).  Images: max abs <= 1e-4 of the dirty peak.
"""
import numpy as np
import pytest
import torch

from oracle import clean, imager
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


def _run(wl, niter, gain=0.1, threshold=None, positive_only=False, restore=True, team_size=0, inputs=None,
         window=None):
    require_gpu()
    from paper_1712_06913_amd import api
    dirty, beams = inputs if inputs is not None else _inputs(wl)
    b = api.Batch.from_workload(wl)
    d_t = torch.from_numpy(np.concatenate([x.ravel() for x in dirty])).cuda()
    b_t = torch.from_numpy(np.concatenate([x.ravel() for x in beams])).cuda()
    res = api.hogbom_clean(b, d_t, b_t, niter, gain=gain, threshold=threshold, positive_only=positive_only,
                           restore=restore, team_size=team_size, window=window)
    torch.cuda.synchronize()
    return b, dirty, beams, res


def _check(wl, niter, gain=0.1, threshold=None, positive_only=False, exact=False, team_size=0, inputs=None,
           window=None):
    b, dirty, beams, res = _run(wl, niter, gain, threshold, positive_only, team_size=team_size, inputs=inputs,
                                window=window)
    resid = b.split(res["residual"])
    model = b.split(res["model"])
    restored = b.split(res["restored"])
    nc = res["n_comp"].cpu().numpy()
    ci = res["comp_idx"].cpu().numpy()
    cf = res["comp_flux"].cpu().numpy()
    cb = res["cbeam"].cpu().numpy().reshape(-1, 6)
    off = res["comp_off"]
    for i in range(wl.n_inst):
        D = dirty[i].astype(np.float64)
        B = beams[i].astype(np.float64)
        thr = 0.0 if threshold is None else float(threshold[i])
        win = None if window is None else tuple(int(v) for v in window[i])
        R0, M0, idx0, flux0 = clean.hogbom(D, B, gain=gain, niter=int(niter[i]), threshold=thr,
                                           positive_only=positive_only, window=win)
        n = int(nc[i])
        gi, gf = ci[off[i]: off[i] + n], cf[off[i]: off[i] + n]
        peak = np.max(np.abs(D))
        log(f"  inst {i} N={D.shape[0]} n_comp gpu={n} oracle={len(idx0)}")
        if exact:
            assert n == len(idx0)
            assert np.array_equal(gi, idx0)
            assert np.max(np.abs(gf - flux0)) <= 1e-5 * peak
        else:
            ok, bad, Rr, Mr = clean.replay(D, B, gi, gf, gain=gain, threshold=thr, positive_only=positive_only,
                                           window=win)
            assert ok, f"replay rejected pick {bad}"
            if n < int(niter[i]):
                # stopped early: the next peak of the replayed residual is at the threshold
                x0, y0, x1, y1 = win if win is not None else (0, 0, D.shape[0], D.shape[0])
                Rw = Rr[y0:y1, x0:x1]
                nxt = np.max(Rw) if positive_only else np.max(np.abs(Rw))
                assert abs(nxt) <= thr + 1e-5 * peak
            R0, M0 = Rr, Mr
        assert max_abs(resid[i].cpu().numpy(), R0) <= 1e-4 * peak
        assert max_abs(model[i].cpu().numpy(), M0) <= 1e-5 * peak
        a, bb, c, bmaj, bmin, pa = clean.fit_clean_beam(B)
        assert np.allclose(cb[i, :3], [a, bb, c], rtol=1e-4, atol=1e-6)
        assert abs(cb[i, 3] - bmaj) <= 1e-4 * bmaj and abs(cb[i, 4] - bmin) <= 1e-4 * bmin
        rest = clean.restore(R0, M0, (a, bb, c))
        assert max_abs(restored[i].cpu().numpy(), rest) <= 1e-4 * peak


def test_clean_small_batch_mixed_sizes():
    log("[clean] mixed 64/128/256 batch")
    wl = synth.random_instances(21, [64, 128, 256, 64], m_range=(100, 300))
    _check(wl, np.array([50, 120, 200, 0], np.int32))


def test_clean_all_zero_map_yields_no_components():
    log("[clean] an all-zero dirty map next to a normal one: no components, zero maps exactly")
    wl = synth.random_instances(24, [128, 128], m_range=(150, 250))
    dirty, beams = _inputs(wl)
    dirty[1] = np.zeros_like(dirty[1])
    # the zero map's tolerances are all 0 (peak 0): residual, model and restored must be exact zeros
    _check(wl, np.array([60, 60], np.int32), inputs=(dirty, beams))
    _, _, _, res = _run(wl, np.array([60, 60], np.int32), inputs=(dirty, beams))
    assert int(res["n_comp"][1].item()) == 0


def test_clean_threshold_stops_early_and_positive_only():
    log("[clean] threshold / positive-only")
    wl = synth.random_instances(22, [64, 128], m_range=(150, 250))
    dirty, _ = _inputs(wl)
    thr = np.array([0.5 * np.max(np.abs(d)) for d in dirty], np.float32)
    _check(wl, np.array([400, 400], np.int32), threshold=thr)
    _check(wl, np.array([60, 60], np.int32), positive_only=True)


def test_clean_window_restricts_the_peak_search():
    log("[clean] peak-search windows excluding the brightest pixels, 64..1024, replayed by the oracle")
    wl = synth.random_instances(27, [64, 256, 1024, 128], m_range=(150, 300))
    inputs = _inputs(wl)
    win = []
    for d in inputs[0]:
        N = d.shape[0]
        py, px = divmod(int(np.argmax(np.abs(d))), N)
        # a box on the far side of the brightest pixel, so that pixel is never a candidate
        x0, x1 = (px + 3, N) if px < N // 2 else (0, px - 2)
        y0, y1 = (N // 5, N - N // 7)
        win.append((x0, y0, x1, y1))
    win = np.array(win, np.int32)
    niter = np.array([40, 80, 150, 60], np.int32)
    _check(wl, niter, inputs=inputs, window=win)
    _check(wl, niter, inputs=inputs, window=win, positive_only=True)
    # a window covering every map gives exactly the unwindowed components
    full = np.array([(0, 0, d.shape[0], d.shape[0]) for d in inputs[0]], np.int32)
    _, _, _, ra = _run(wl, niter, inputs=inputs, window=full)
    _, _, _, rb = _run(wl, niter, inputs=inputs)
    assert torch.equal(ra["comp_idx"], rb["comp_idx"]) and torch.equal(ra["n_comp"], rb["n_comp"])


def test_clean_window_rejects_bad_boxes():
    log("[clean] bad windows are argument errors")
    require_gpu()
    from paper_1712_06913_amd import api, _native as nat
    wl = synth.random_instances(28, [64], m_range=(50, 60))
    dirty, beams = _inputs(wl)
    b = api.Batch.from_workload(wl)
    d_t = torch.from_numpy(dirty[0].ravel()).cuda()
    b_t = torch.from_numpy(beams[0].ravel()).cuda()
    for w in [(0, 0, 65, 64), (5, 5, 5, 9), (-1, 0, 10, 10), (10, 0, 3, 64)]:
        with pytest.raises(nat.MiError):
            api.hogbom_clean(b, d_t, b_t, np.array([10], np.int32), window=np.array([w], np.int32))


def test_clean_single_point_closed_form_exact():
    log("[clean] single point source closed form")
    require_gpu()
    from paper_1712_06913_amd import api
    wl = synth.random_instances(23, [128], m_range=(200, 200))
    v, uv, w = wl.instance(0)
    N = 128
    B = imager.dirty_beam(uv, w, N, float(wl.cell_rad[0]), 0).astype(np.float32)
    py, px, S = 40, 77, 3.0
    D = (S * B[N - py: 2 * N - py, N - px: 2 * N - px]).astype(np.float32)
    b = api.Batch.from_workload(wl)
    res = api.hogbom_clean(b, torch.from_numpy(D.ravel()).cuda(), torch.from_numpy(B.ravel()).cuda(), [30])
    torch.cuda.synchronize()
    ci = res["comp_idx"].cpu().numpy()
    assert np.all(ci == py * N + px)
    model = res["model"].cpu().numpy()
    assert abs(model[py * N + px] - S * (1 - 0.9 ** 30)) < 1e-5 * S


def test_clean_c1_workload_replay():
    log("[clean] C1 256^2, 500 iterations")
    wl = synth.c1_snapshot()
    _check(wl, wl.niter)


def test_clean_c2_slice_512():
    log("[clean] C2 slice: 2 instances at 512^2, 300 iterations")
    wl = synth.c2_muser1_batch(n_chan=2, n_snap=1)
    _check(wl, np.array([300, 300], np.int32))


def _symmetrized(B):
    """Copy the half with rows < N (and row N, columns < N) onto its point mirror about (N, N)."""
    n2 = B.shape[0]
    N = n2 // 2
    S = B.copy()
    S[N + 1:, 1:] = B[N - 1:0:-1, n2 - 1:0:-1]
    S[N, N + 1:] = B[N, N - 1:0:-1]
    return S


def test_clean_1024_team_sizes_agree_and_replay():
    log("[clean] 1024^2: teams of 16 (64 px/thread, restore staged in two parts) and 32; "
        "mirrored beam reads for an exactly symmetric beam, direct reads otherwise")
    wl = synth.c3_muser2(chans=[7], niter=150)
    dirty, beams = _inputs(wl)
    sym = [_symmetrized(beams[0])]
    asym = [sym[0].copy()]
    asym[0][1, 1] += 1e-3                      # one pixel breaks the symmetry: direct reads
    niter = np.array([150], np.int32)
    for bm in (sym, asym):
        _check(wl, niter, team_size=16, inputs=(dirty, bm))
    outs = []
    for ts in (16, 32):
        _, _, _, res = _run(wl, niter, team_size=ts, inputs=(dirty, sym))
        outs.append({k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in res.items()})
    a, c = outs
    assert np.array_equal(a["n_comp"], c["n_comp"]) and np.array_equal(a["comp_idx"], c["comp_idx"])
    # the same fma sequence per pixel whatever the team shape: bit-identical residuals
    assert np.array_equal(a["residual"], c["residual"])
    assert np.max(np.abs(a["restored"] - c["restored"])) <= 1e-6 * np.max(np.abs(dirty[0]))


def test_profile_hook_times_each_hogbom_launch():
    log("[clean] mi_profile_begin / mi_profile_end record one duration per Hogbom launch")
    require_gpu()
    from paper_1712_06913_amd import api
    wl = synth.random_instances(24, [128, 64], m_range=(100, 200))
    inputs = _inputs(wl)
    api.profile_begin()
    for _ in range(3):
        _run(wl, np.array([40, 40], np.int32), inputs=inputs, restore=False)
    ms = api.profile_end()
    assert len(ms) == 3 and all(t > 0.0 for t in ms), ms
    assert api.profile_end() == []            # recording stopped and cleared


def test_clean_c3_headline_depth_5000_iterations():
    log("[clean] one C3 channel at 1024^2, 5000 iterations: GPU dirty image + beam, GPU CLEAN + restore, "
        "every pick replayed by the oracle")
    require_gpu()
    from paper_1712_06913_amd import api
    wl = synth.c3_muser2(chans=[3])
    b = api.Batch.from_workload(wl)
    vis, uv, w = api.workload_tensors(wl)
    dirty, beam, _ = api.dirty_image(b, vis, uv, w, beam=True)
    res = api.hogbom_clean(b, dirty, beam, wl.niter, gain=wl.gain, restore=True)
    torch.cuda.synchronize()
    v, uvi, wi = wl.instance(0)
    N, cell = int(wl.n_img[0]), float(wl.cell_rad[0])
    D = dirty.cpu().numpy().reshape(N, N).astype(np.float64)
    B = beam.cpu().numpy().reshape(2 * N, 2 * N).astype(np.float64)
    ref = imager.dirty_image(v, uvi, wi, N, cell, 0)
    peak = float(np.max(np.abs(ref)))
    assert max_abs(D, ref) <= 1e-4 * peak
    assert max_abs(B, imager.dirty_beam(uvi, wi, N, cell, 0)) <= 1e-4
    n = int(res["n_comp"][0])
    assert n == 5000 and int(b.status[0]) == 0
    ok, bad, R, M = clean.replay(D, B, res["comp_idx"].cpu().numpy()[:n], res["comp_flux"].cpu().numpy()[:n])
    assert ok, f"replay rejected pick {bad}"
    e_r = max_abs(res["residual"].cpu().numpy().reshape(N, N), R)
    e_m = max_abs(res["model"].cpu().numpy().reshape(N, N), M)
    abc = clean.fit_clean_beam(B)
    rest = clean.restore_conv(R, M, abc)
    e_s = max_abs(res["restored"].cpu().numpy().reshape(N, N), rest)
    log(f"  residual {e_r / peak:.2e}, model {e_m / peak:.2e}, restored {e_s / peak:.2e} of the peak")
    assert e_r <= 1e-4 * peak and e_m <= 1e-5 * peak and e_s <= 1e-4 * peak


def test_clean_c2_slice_full_depth_2000():
    log("[clean] C2 slice at its full depth: 512^2, 2000 iterations")
    wl = synth.c2_muser1_batch(n_chan=1, n_snap=2)
    _check(wl, wl.niter)


def _tie_case(N, coords, vals, extra):
    """A map with |value| ties at `coords` (mixed signs) and distinct smaller values at `extra`."""
    D = np.zeros((N, N), np.float32)
    for (y, x), v in zip(coords, vals):
        D[y, x] = v
    for k, (y, x) in enumerate(extra):
        D[y, x] = 0.5 - 0.01 * k
    return D


@pytest.mark.parametrize("N,team", [(1024, 16), (1024, 32), (256, 0), (256, 4)])
@pytest.mark.parametrize("positive_only", [False, True])
@pytest.mark.parametrize("symmetric", [True, False])
def test_clean_exact_ties_pick_lowest_index(N, team, positive_only, symmetric):
    """Equal |values| of mixed sign spread over lanes, 4-pixel groups, waves and team members:
    with a delta beam and gain 1 each pick removes one pixel, so the pick order is the tie
    rule itself (lowest y N + x first), compared exactly with the oracle."""
    log(f"[clean] exact ties N={N} team={team} positive_only={positive_only} symmetric={symmetric}")
    require_gpu()
    from paper_1712_06913_amd import api
    s = N // 1024 if N >= 1024 else 1
    coords = [(5 * s, 8), (5 * s, 9),            # one 4-pixel group
              (5 * s, 20),                      # another lane of the same wave
              (5 * s, N // 4 + 44),             # another wave, same row
              (N // 16, 0),                     # first pixel of another member (teams of 16)
              (N // 2 + 3, N - 1), (N - 1, 3),   # far members
              (N // 3, N // 2)]
    vals = [1.0, -1.0, 1.0, -1.0, 1.0, -1.0, 1.0, 1.0]
    extra = [(N // 2, N // 2 + 7), (7, 7), (N - 2, N - 9)]
    D = _tie_case(N, coords, vals, extra)
    B = np.zeros((2 * N, 2 * N), np.float32)
    B[N, N] = 1.0
    if not symmetric:
        B[1, 1] = 1e-3                          # reached by no pick here; breaks the point symmetry
    wl = synth.random_instances(29, [N], m_range=(10, 10))
    b = api.Batch.from_workload(wl)
    niter = np.array([20], np.int32)
    res = api.hogbom_clean(b, torch.from_numpy(D.ravel()).cuda(), torch.from_numpy(B.ravel()).cuda(), niter,
                           gain=1.0, positive_only=positive_only, team_size=team)
    torch.cuda.synchronize()
    R0, M0, idx0, flux0 = clean.hogbom(D.astype(np.float64), B.astype(np.float64), gain=1.0, niter=20,
                                       positive_only=positive_only)
    n = int(res["n_comp"][0])
    gi = res["comp_idx"].cpu().numpy()[:n]
    log(f"  gpu picks {gi.tolist()}")
    assert n == len(idx0) and np.array_equal(gi, idx0)
    assert np.array_equal(res["comp_flux"].cpu().numpy()[:n], flux0)
    assert np.array_equal(res["residual"].cpu().numpy().reshape(N, N), R0.astype(np.float32))


@pytest.mark.parametrize("team", [64, 128, 256])
def test_clean_non_local_team_sizes_match_oracle(team):
    """Teams spread over several XCDs (what the autotuner may pick for few images)."""
    log(f"[clean] 1024^2 with teams of {team} workgroups (non-local), replayed by the oracle")
    wl = synth.c3_muser2(chans=[11], niter=120)
    _check(wl, np.array([120], np.int32), team_size=team)


@pytest.mark.parametrize("N,niter", [(2048, 120), (4096, 40)])
def test_clean_large_images(N, niter):
    log(f"[clean] {N}^2 images ({N * N // 65536} workgroups per image), replayed by the oracle")
    require_gpu()
    from paper_1712_06913_amd import api
    wl = synth.random_instances(30, [N], m_range=(600, 600), uniform_frac=0.0)
    b = api.Batch.from_workload(wl)
    vis, uv, w = api.workload_tensors(wl)
    dirty, beam, _ = api.dirty_image(b, vis, uv, w, beam=True)
    res = api.hogbom_clean(b, dirty, beam, np.array([niter], np.int32), restore=True)
    torch.cuda.synchronize()
    assert int(b.status[0]) & 16 == 0
    D = dirty.cpu().numpy().reshape(N, N).astype(np.float64)
    B = beam.cpu().numpy().reshape(2 * N, 2 * N).astype(np.float64)
    del dirty, beam
    n = int(res["n_comp"][0])
    assert n == niter
    ok, bad, R, M = clean.replay(D, B, res["comp_idx"].cpu().numpy()[:n], res["comp_flux"].cpu().numpy()[:n])
    assert ok, f"replay rejected pick {bad}"
    peak = float(np.max(np.abs(D)))
    assert max_abs(res["residual"].cpu().numpy().reshape(N, N), R) <= 1e-4 * peak
    assert max_abs(res["model"].cpu().numpy().reshape(N, N), M) <= 1e-5 * peak
    rest = clean.restore_conv(R, M, clean.fit_clean_beam(B), radius=256)
    assert max_abs(res["restored"].cpu().numpy().reshape(N, N), rest) <= 1e-4 * peak


def test_clean_abort_flags_every_image_of_the_team():
    """Failure path forced from the host: with MI_TEST_CLEAN_STALL set when the context is
    made, one team member never publishes and every team wait gives up after a few polls.
    All images of a team that owns several must come back flagged MI_INST_ABORTED."""
    log("[clean] forced team-wait timeout: every image of the team is flagged")
    require_gpu()
    import os
    from paper_1712_06913_amd import api
    os.environ["MI_TEST_CLEAN_STALL"] = "1"
    try:
        ctx = api.Context(0)
    finally:
        del os.environ["MI_TEST_CLEAN_STALL"]
    try:
        wl = synth.random_instances(33, [256] * 5, m_range=(100, 200))
        dirty, beams = _inputs(wl)
        b = api.Batch.from_workload(wl, ctx=ctx)
        d_t = torch.from_numpy(np.concatenate([x.ravel() for x in dirty])).cuda()
        b_t = torch.from_numpy(np.concatenate([x.ravel() for x in beams])).cuda()
        # one team of 256 workgroups (the whole device at 256^2) owns all five images
        api.hogbom_clean(b, d_t, b_t, np.full(5, 30, np.int32), team_size=256)
        torch.cuda.synchronize()
        st = b.status.cpu().numpy()
        log(f"  status {st.tolist()}")
        assert np.all(st & 16)
    finally:
        ctx.close()
