"""Pins of the synthetic MUSER-shaped workload generator."""
import math

import numpy as np
from scipy import integrate, special

from paper_1712_06913_amd import synth


def _hankel(profile, q, R):
    # V(q) = integral_0^R B(rho) J0(2 pi q rho) 2 pi rho d rho
    val, _ = integrate.quad(lambda r: profile(r) * special.j0(2 * math.pi * q * r) * 2 * math.pi * r,
                            0.0, R, epsabs=1e-14, epsrel=1e-12, limit=400)
    return val


def test_disk_and_limb_visibilities_match_numerical_hankel_transform():
    R = 16 * synth.ARCMIN
    bd = 1.0 / (math.pi * R * R)
    a = 0.55
    for q in (0.0, 10.0, 150.0, 700.0, 2500.0):
        d = synth.disk_vis(np.array([q]), R)[0]
        assert abs(d - _hankel(lambda r: bd, q, R)) < 1e-9
        lv = synth.limb_vis(np.array([q]), R, a, bd)[0]
        assert abs(lv - _hankel(lambda r: bd * a * (r / R) ** 2, q, R)) < 1e-9


def test_gaussian_visibility_matches_2d_quadrature():
    peak, sigma, l0, m0 = 3.0, 2 * synth.ARCMIN, 1.5e-3, -0.7e-3
    u, v = 310.0, -145.0
    val = synth.gauss_vis(np.array([u]), np.array([v]), peak, sigma, l0, m0)[0]
    lim = 8 * sigma
    f = lambda m, l, part: part(peak * math.exp(-((l - l0) ** 2 + (m - m0) ** 2) / (2 * sigma ** 2))
                                * np.exp(-2j * math.pi * (u * l + v * m)))
    re, _ = integrate.dblquad(f, l0 - lim, l0 + lim, m0 - lim, m0 + lim, args=(np.real,), epsabs=1e-14)
    im, _ = integrate.dblquad(f, l0 - lim, l0 + lim, m0 - lim, m0 + lim, args=(np.imag,), epsabs=1e-14)
    assert abs(val - (re + 1j * im)) < 1e-6 * abs(val)


def test_table1_table2_arithmetic():
    # resolution lambda / B_max: 51.5 arcsec at 0.4 GHz and 1.37 arcsec at 15 GHz with 3 km
    res = lambda f: synth.C_LIGHT / f / 3000.0 * 180 / math.pi * 3600
    assert abs(res(0.4e9) - 51.5) < 0.1 and abs(res(15e9) - 1.375) < 0.01
    # image extent = N * pixel (Table 2, column 4), pixel = resolution / 3
    assert abs(256 * 17.2 / 60 - 73.4) < 0.1 and abs(1024 * 5.9 / 60 - 100.7) < 0.1
    # 614,400 images per minute: 2 arrays x 16 channels per 3.125 ms frame
    assert 2 * 16 * 60 / 3.125e-3 == 614400


def test_array_sizes_and_reproducibility():
    assert len(synth.baselines(synth.muser1_array())) == 780
    assert len(synth.baselines(synth.muser2_array())) == 1770
    a, b = synth.c1_snapshot(), synth.c1_snapshot()
    assert np.array_equal(a.vis, b.vis) and np.array_equal(a.uv, b.uv)
    r = np.hypot(*synth.muser2_array().T)
    assert r.max() < 3000 * 1.25 and r.min() > 3.0


def test_workload_shapes():
    c1 = synth.c1_snapshot()
    assert c1.n_inst == 1 and c1.n_img[0] == 256 and c1.niter[0] == 500 and c1.weight_mode[0] == 0
    c4 = synth.c4_uneven(12)
    assert set(c4.n_img) <= {256, 512, 1024}
    counts = np.diff(c4.vis_offset)
    assert counts.min() >= 200 and counts.max() <= 1770
    sub = c4.subset([3, 1])
    assert np.array_equal(sub.instance(0)[0], c4.instance(3)[0])
