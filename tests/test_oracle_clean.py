"""Pins of the oracle's Hogbom CLEAN, clean-beam fit and restore (Algorithm 1, Sec. 4.3)."""
import math

import numpy as np
import pytest

from oracle import clean, imager
from paper_1712_06913_amd import synth


def _gauss_beam(N, a, b, c):
    yy, xx = np.mgrid[0:2 * N, 0:2 * N]
    dx, dy = xx - N, yy - N
    return np.exp(-(a * dx * dx + b * dx * dy + c * dy * dy))


def _real_beam(N=32, seed=3):
    wl = synth.random_instances(seed, [N], m_range=(120, 120), uniform_frac=0.0)
    v, uv, w = wl.instance(0)
    return imager.dirty_beam(uv, w, N, float(wl.cell_rad[0]), 0)


@pytest.mark.parametrize("n", [1, 7, 40])
def test_single_point_source_closed_form(n):
    N, g, S = 32, 0.1, 2.0
    beam = _real_beam(N)
    py, px = 11, 19
    dirty = S * beam[N - py: 2 * N - py, N - px: 2 * N - px]
    R, model, idx, flux = clean.hogbom(dirty, beam, gain=g, niter=n)
    assert np.all(idx == py * N + px)
    assert abs(model[py, px] - S * (1 - (1 - g) ** n)) < 1e-12
    assert np.count_nonzero(model) == 1
    assert np.max(np.abs(R - S * (1 - g) ** n * beam[N - py: 2 * N - py, N - px: 2 * N - px])) < 1e-12
    assert np.allclose(flux, g * S * (1 - g) ** np.arange(n), rtol=0, atol=1e-12)


def test_gain_one_removes_point_in_one_step_and_threshold_stops():
    N = 32
    beam = _real_beam(N)
    dirty = -1.5 * beam[N - 5: 2 * N - 5, N - 30: 2 * N - 30]
    R, model, idx, flux = clean.hogbom(dirty, beam, gain=1.0, niter=10, threshold=1e-9)
    assert len(idx) == 1 and idx[0] == 5 * N + 30 and abs(flux[0] + 1.5) < 1e-12
    assert np.max(np.abs(R)) < 1e-12


def test_niter_zero_leaves_dirty():
    N = 16
    beam = _real_beam(N)
    dirty = np.random.default_rng(0).standard_normal((N, N))
    R, model, idx, _ = clean.hogbom(dirty, beam, niter=0)
    assert np.array_equal(R, dirty) and len(idx) == 0 and not model.any()


def test_ties_pick_lowest_linear_index_and_abs_peak():
    N = 16
    beam = np.zeros((2 * N, 2 * N))
    beam[N, N] = 1.0
    dirty = np.zeros((N, N))
    dirty[9, 3] = 4.0
    dirty[2, 14] = -4.0          # same |value|, lower linear index (2*16+14 < 9*16+3)
    _, _, idx, flux = clean.hogbom(dirty, beam, gain=1.0, niter=1)
    assert idx[0] == 2 * N + 14 and flux[0] == -4.0
    _, _, idx, _ = clean.hogbom(dirty, beam, gain=1.0, niter=1, positive_only=True)
    assert idx[0] == 9 * N + 3


def test_clean_identity_on_imaged_sky():
    wl = synth.random_instances(11, [32], m_range=(150, 150))
    v, uv, w = wl.instance(0)
    N, cell = 32, float(wl.cell_rad[0])
    dirty = imager.dirty_image(v, uv, w, N, cell, 1)
    beam = imager.dirty_beam(uv, w, N, cell, 1)
    R, model, idx, flux = clean.hogbom(dirty, beam, gain=0.1, niter=200)
    assert clean.clean_identity(dirty, beam, R, model) < 1e-12 * np.max(np.abs(dirty))
    assert np.max(np.abs(R)) < np.max(np.abs(dirty))
    ok, bad, R2, _ = clean.replay(dirty, beam, idx, flux)
    assert ok and np.max(np.abs(R2 - R)) < 1e-12


def test_replay_rejects_a_wrong_pick():
    wl = synth.random_instances(12, [32], m_range=(150, 150))
    v, uv, w = wl.instance(0)
    N, cell = 32, float(wl.cell_rad[0])
    dirty = imager.dirty_image(v, uv, w, N, cell, 0)
    beam = imager.dirty_beam(uv, w, N, cell, 0)
    _, _, idx, flux = clean.hogbom(dirty, beam, niter=30)
    idx2 = idx.copy()
    idx2[10] = (idx2[10] + 5) % (N * N)
    ok, bad, _, _ = clean.replay(dirty, beam, idx2, flux)
    assert not ok and bad == 10


def test_fit_recovers_exact_gaussian_beam():
    N = 32
    a, b, c = 0.12, 0.05, 0.3
    beam = _gauss_beam(N, a, b, c)
    fa, fb, fc, bmaj, bmin, pa = clean.fit_clean_beam(beam)
    assert abs(fa - a) < 1e-10 and abs(fb - b) < 1e-10 and abs(fc - c) < 1e-10
    # FWHM along principal axes: exp(-lambda r^2) = 1/2
    lmin = 0.5 * (a + c - math.hypot(a - c, b))
    assert abs(bmaj - 2 * math.sqrt(math.log(2) / lmin)) < 1e-9
    assert bmaj >= bmin and 0 <= pa < math.pi


def test_main_lobe_is_connected_region_only():
    N = 16
    beam = _gauss_beam(N, 0.2, 0.0, 0.2)
    beam[N, N + 6] = 0.9                      # isolated bright sidelobe pixel, not connected
    mask = clean.main_lobe(beam)
    assert not mask[N, N + 6] and mask[N, N] and mask[N, N + 1]


def test_restore_without_components_is_residual_and_single_component_is_gaussian():
    N = 16
    R = np.random.default_rng(1).standard_normal((N, N))
    abc = (0.2, 0.0, 0.3)
    assert np.array_equal(clean.restore(R, np.zeros((N, N)), abc), R)
    model = np.zeros((N, N))
    model[4, 9] = 2.0
    out = clean.restore(np.zeros((N, N)), model, abc)
    assert out[4, 9] == 2.0
    assert abs(out[5, 9] - 2.0 * math.exp(-0.3)) < 1e-14 and abs(out[4, 10] - 2.0 * math.exp(-0.2)) < 1e-14


def test_fit_degenerate_lobes_follow_pixel_count_rules():
    N = 16
    # plus-shaped lobe (only axis neighbours above 0.35): b fixed at 0, a and c exact
    beam = _gauss_beam(N, 0.6, 0.0, 0.9)
    (a, b, c, *_), flag = clean.fit_clean_beam(beam, return_flag=True)
    assert clean.main_lobe(beam).sum() == 5
    assert not flag and b == 0.0 and abs(a - 0.6) < 1e-12 and abs(c - 0.9) < 1e-12
    # single-pixel lobe: one-pixel FWHM default, flagged
    beam = _gauss_beam(N, 3.0, 0.0, 3.0)
    (a, b, c, bmaj, bmin, _), flag = clean.fit_clean_beam(beam, return_flag=True)
    assert flag and (a, b, c) == clean.DEGENERATE_ABC and abs(bmaj - 1.0) < 1e-12


def test_replay_positive_only_uses_signed_peak():
    wl = synth.random_instances(13, [32], m_range=(150, 150))
    v, uv, w = wl.instance(0)
    N, cell = 32, float(wl.cell_rad[0])
    dirty = imager.dirty_image(v, uv, w, N, cell, 0)
    beam = imager.dirty_beam(uv, w, N, cell, 0)
    _, _, idx, flux = clean.hogbom(dirty, beam, niter=40, positive_only=True)
    assert clean.replay(dirty, beam, idx, flux, positive_only=True)[0]


def test_window_picks_follow_a_brute_force_search_and_subtract_everywhere():
    # every pick is the lowest-index maximum of |R| over the window's pixels, found here by
    # a plain double loop; the subtraction covers the whole map (checked pixel by pixel)
    N = 16
    beam = _real_beam(N, seed=5)
    rng = np.random.default_rng(31)
    dirty = rng.standard_normal((N, N))
    dirty[1, 1] = 50.0                       # brightest pixel, outside the window
    win = (4, 3, 13, 11)                     # x0, y0, x1, y1
    R, model, idx, flux = clean.hogbom(dirty, beam, gain=0.2, niter=25, window=win)
    assert len(idx) == 25
    Rb = dirty.copy()
    for p, f in zip(idx, flux):
        best, bp = -1.0, -1
        for y in range(win[1], win[3]):
            for x in range(win[0], win[2]):
                if abs(Rb[y, x]) > best:
                    best, bp = abs(Rb[y, x]), y * N + x
        assert p == bp and abs(f - 0.2 * Rb[bp // N, bp % N]) < 1e-12
        py, px = divmod(int(p), N)
        for y in range(N):
            for x in range(N):
                Rb[y, x] -= f * beam[y - py + N, x - px + N]
    assert np.max(np.abs(Rb - R)) < 1e-12
    assert abs(R[1, 1] - dirty[1, 1]) > 0 and model[1, 1] == 0.0   # changed by sidelobes, never picked
    ok, bad, _, _ = clean.replay(dirty, beam, idx, flux, gain=0.2, window=win)
    assert ok
    ok, bad, _, _ = clean.replay(dirty, beam, idx, flux, gain=0.2)      # without the window: the first pick is wrong
    assert not ok and bad == 0


def test_full_window_equals_no_window():
    N = 16
    beam = _real_beam(N, seed=6)
    dirty = np.random.default_rng(32).standard_normal((N, N))
    a = clean.hogbom(dirty, beam, niter=40)
    b = clean.hogbom(dirty, beam, niter=40, window=(0, 0, N, N))
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[0], b[0])


def test_restore_conv_is_the_direct_restore():
    rng = np.random.default_rng(61)
    N = 48
    R = rng.standard_normal((N, N))
    M = np.zeros((N, N))
    M.flat[rng.choice(N * N, 9, replace=False)] = rng.standard_normal(9)
    abc = (0.31, 0.07, 0.22)
    ref = clean.restore(R, M, abc)
    assert np.max(np.abs(clean.restore_conv(R, M, abc) - ref)) < 1e-12
    # a Gaussian this narrow is below 1e-12 of its peak beyond 12 pixels
    assert np.max(np.abs(clean.restore_conv(R, M, abc, radius=12) - ref)) < 1e-10


def test_replay_rejects_picks_below_the_threshold():
    N = 32
    yy, xx = np.mgrid[0:2 * N, 0:2 * N]
    B = np.exp(-((xx - N) ** 2 + (yy - N) ** 2) / 3.0)
    D = 2.0 * B[N - 10: 2 * N - 10, N - 12: 2 * N - 12]
    R, M, idx, flux = clean.hogbom(D, B, gain=0.1, niter=30)
    # the peak falls as 2 (0.9)^k: a threshold between steps 20 and 21 ends a valid run at 21 picks
    thr = 2.0 * 0.9 ** 20.5
    ok, bad, _, _ = clean.replay(D, B, idx[:21], flux[:21], threshold=thr)
    assert ok
    ok, bad, _, _ = clean.replay(D, B, idx, flux, threshold=thr)
    assert not ok and bad == 21
