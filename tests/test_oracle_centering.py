"""Pins of the FP64 disk centering and phase correction (oracle/centering.py)."""
import math

import numpy as np

from oracle import centering, clean, gmm, imager
from paper_1712_06913_amd import synth


def test_fft_correlation_equals_the_direct_sum():
    rng = np.random.default_rng(21)
    N = 12
    img = rng.standard_normal((N, N))
    mod = rng.standard_normal((N, N))
    C = centering.correlate(img, mod)
    ref = np.zeros((N, N))
    for dy in range(N):
        for dx in range(N):
            ref[dy, dx] = sum(img[y, x] * mod[(y - dy) % N, (x - dx) % N] for y in range(N) for x in range(N))
    assert np.max(np.abs(C - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_whole_pixel_shift_is_found_exactly():
    N, r = 128, 20.0
    disk = centering.disk_model(N, r)
    for dx, dy in ((7, -3), (-12, 5), (0, 0), (31, 30)):
        img = np.roll(np.roll(disk, dy, axis=0), dx, axis=1)
        ox, oy = centering.peak_offset(centering.correlate(img, disk))
        assert abs(ox - dx) < 1e-9 and abs(oy - dy) < 1e-9
    # radians follow the cell
    dl, dm = centering.disk_offset(np.roll(disk, 4, axis=1), r, 1e-4)
    assert abs(dl - 4e-4) < 1e-15 and abs(dm) < 1e-15


def test_parabolic_refinement_is_exact_for_a_parabola():
    N = 16
    x = np.arange(N)
    C = np.full((N, N), -1e9)
    C[5, :] = -((x - 6.3) ** 2)           # peak row y = 5, parabola in x with vertex at 6.3
    C[:, 6] = -((np.arange(N) - 5.0) ** 2) - 0.09
    C[5, 6] = -(0.3 ** 2)
    ox, oy = centering.peak_offset(C)
    assert abs(ox - 6.3) < 1e-12 and abs(oy - 5.0) < 1e-12


def test_point_source_phase_correction_closed_form():
    rng = np.random.default_rng(22)
    uv = rng.uniform(-3000, 3000, (200, 2))
    l0, m0, S = 3.1e-4, -1.7e-4, 2.5
    vis = S * np.exp(-2j * math.pi * (uv[:, 0] * l0 + uv[:, 1] * m0))
    out = centering.phase_correct(vis, uv, l0, m0)
    assert np.max(np.abs(out - S)) < 1e-12
    back = centering.phase_correct(out, uv, -l0, -m0)
    assert np.max(np.abs(back - vis)) < 1e-12


def test_displaced_synthetic_sun_is_found_and_centred():
    # end to end on synthetic data (a sanity check, not a precision pin): clean to the disk
    # level, correlate with the disk, correct; the estimate lies within a few pixels of the
    # true displacement and the corrected map is closer to centred
    wl = synth.offset_disk(n=2)
    for i in range(wl.n_inst):
        v, uv, w = wl.instance(i)
        N, cell = int(wl.n_img[i]), float(wl.cell_rad[i])
        d = imager.dirty_image(v, uv, w, N, cell, 0).astype(np.float32)
        bm = imager.dirty_beam(uv, w, N, cell, 0).astype(np.float32)
        mu_b = gmm.levels(d)[3]
        R, _, _, _ = clean.hogbom(d.astype(np.float64), bm.astype(np.float64), niter=3000,
                                  threshold=float(np.float32(mu_b)), positive_only=True)
        rpx = 16.0 * synth.ARCMIN / cell
        dl, dm = centering.disk_offset(R, rpx, cell)
        truth = wl.sky_centre[i]
        err = math.hypot(dl - truth[0], dm - truth[1]) / cell
        assert err < 3.0, f"instance {i}: {err:.2f} px"
        v2 = centering.phase_correct(v, uv, dl, dm)
        d2 = imager.dirty_image(v2, uv, w, N, cell, 0)
        r2 = math.hypot(*centering.disk_offset(d2, rpx, cell)) / cell
        r0 = math.hypot(*centering.disk_offset(d, rpx, cell)) / cell
        assert r2 < 0.5 * r0
