"""Pins of the FP64 w-projection imager (oracle/wproj.py), Sec. 3.2.2 and 6.1."""
import math

import numpy as np

from oracle import gcf, imager, wproj


def _point_source_data(seed, n_vis, N, cell, l0, m0, w_scale):
    rng = np.random.default_rng(seed)
    # uv inside the kept region, w drawn independently (the w-term is what is tested)
    uv = rng.uniform(-0.35, 0.35, (n_vis, 2)) / cell
    wl = rng.uniform(-1.0, 1.0, n_vis) * w_scale
    n0 = math.sqrt(1.0 - l0 * l0 - m0 * m0)
    vis = np.exp(-2j * math.pi * (uv[:, 0] * l0 + uv[:, 1] * m0 + wl * (n0 - 1.0)))
    return (vis.astype(np.complex64), uv.astype(np.float32), wl.astype(np.float32),
            np.ones(n_vis, np.float32))


def test_exact_imager_at_zero_w_is_the_2d_direct_dft():
    N, cell = 32, 4e-4
    vis, uv, wl, w_in = _point_source_data(1, 60, N, cell, 3e-3, -2e-3, 0.0)
    prep = imager.Prep(uv, w_in, N, cell)
    w = imager.weights(prep, 0)
    a = wproj.exact_dirty(vis, uv, np.zeros(len(wl), np.float32), w, prep.keep, N, cell)
    b = imager.dft_image(vis, uv, w, prep.keep, N, cell)
    assert np.max(np.abs(a - b)) < 1e-12


def test_zero_w_kernel_is_the_spheroidal_table_product():
    N, cell = 64, 3e-4
    S = 7
    K = wproj.kernel_table(0.0, S, N, cell, osw=16)
    half = S * 16 // 2
    t = np.arange(-half, half + 1) / 16.0
    c1 = gcf.gcf(t) / gcf.gcf(np.array([0.0]))[0]
    ref = np.outer(c1, c1)
    assert np.max(np.abs(K.imag)) < 1e-12
    # equal up to the truncation of the correction function at the field edge
    assert np.max(np.abs(K.real - ref)) < 2e-3
    assert abs(K.real[half, half] - 1.0) < 2e-3


def test_kernel_symmetries():
    N, cell = 64, 3e-4
    K = wproj.kernel_table(900.0, 11, N, cell, osw=8)
    Km = wproj.kernel_table(-900.0, 11, N, cell, osw=8)
    assert np.max(np.abs(Km - np.conj(K))) < 1e-14
    assert np.max(np.abs(K - K[::-1, ::-1])) < 1e-14          # even in (du, dv)
    assert np.max(np.abs(K - K.T)) < 1e-14                    # the screen is symmetric in l, m


def test_plan_follows_the_phase_rule():
    N, cell = 256, 1.2 * math.pi / 180 / 256
    r2 = wproj.corner_r2(N, cell)
    dw, n, sup = wproj.plan(0.0, N, cell)
    assert n == 1 and sup == [7]
    # the largest rounding error of |w| to its plane moves the corner phase by <= tol / 2
    dw, n, sup = wproj.plan(5000.0, N, cell, tol=0.1)
    assert abs(math.pi * (dw / 2) * r2 - 0.05) < 1e-12
    assert (n - 1) * dw + dw / 2 >= 5000.0
    assert all(s % 2 == 1 for s in sup) and sup == sorted(sup)


def test_w_projection_recovers_the_exact_image_where_2d_imaging_fails():
    # a point source near the field edge, visibilities with a large w-term
    N, cell = 64, 1.2 * math.pi / 180 / 64
    l0 = m0 = 0.3 * N * cell
    r2 = wproj.corner_r2(N, cell)
    w_scale = 4.0 / (math.pi * r2)                 # corner phase up to ~4 rad
    vis, uv, wl, w_in = _point_source_data(2, 120, N, cell, l0, m0, w_scale)
    prep = imager.Prep(uv, w_in, N, cell)
    w = imager.weights(prep, 0)
    exact = wproj.exact_dirty(vis, uv, wl, w, prep.keep, N, cell)
    img2d = imager.dirty_image(vis, uv, w_in, N, cell, 0)
    imgw, (dw, n_planes, sup) = wproj.dirty_image_w(vis, uv, wl, w_in, N, cell, 0, float(np.abs(wl).max()), tol=0.02)
    # compared away from the outermost 4 pixels, where gridding itself (at any w) departs
    # from the direct transform by aliasing amplified by the correction
    inner = (slice(4, N - 4), slice(4, N - 4))
    e2 = np.max(np.abs(img2d - exact)[inner])
    ew = np.max(np.abs(imgw - exact)[inner])
    assert n_planes > 10 and e2 > 0.1
    assert ew < 0.05 * e2 and ew < 1e-2
    # with w = 0 the w-projection imager is the 2-D imager up to the kernel construction
    z = np.zeros_like(wl)
    img0, pl0 = wproj.dirty_image_w(vis, uv, z, w_in, N, cell, 0, 0.0)
    assert pl0[1] == 1 and np.max(np.abs(img0 - img2d)[inner]) < 5e-3
