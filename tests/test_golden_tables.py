"""The synthetic MUSER generator against the values the paper prints in Tables 1 and 2
(fixtures under tests/golden/, each naming its table)."""
import math
import os

import numpy as np

from paper_1712_06913_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]


def _table1():
    return {r[0]: (float(r[1]), float(r[2])) for r in _rows("table1_muser_arrays.txt")}


def _res_arcsec(freq_hz, baseline_m):
    # diffraction resolution lambda / B of the longest baseline, in arc seconds
    return synth.C_LIGHT / freq_hz / baseline_m * 180.0 / math.pi * 3600.0


def test_arrays_and_channels_follow_table1():
    t = _table1()
    a1, a2 = synth.muser1_array(), synth.muser2_array()
    assert (len(a1), len(a2)) == (int(t["antennas"][0]), int(t["antennas"][1]))
    for arr, k in ((a1, 0), (a2, 1)):
        n = len(arr)
        bl = synth.baselines(arr)
        assert len(bl) == n * (n - 1) // 2
        length = np.hypot(bl[:, 0], bl[:, 1])
        # the shortest baselines a few metres (the log-spiral arms start at the printed minimum
        # radius, so neighbouring antennas there sit closer still)
        assert length.min() < 2.5 * t["baseline_min_m"][k]
    # longest baselines: MUSER-I's arms (1.5 km radius) give Table 1's ~3 km; the MUSER-II-like
    # array follows the workload's arm radius of 3 km, so its longest baselines reach about
    # 5 km (those beyond a channel's grid band are dropped by the imager in any case)
    l1 = np.hypot(*synth.baselines(a1).T)
    l2 = np.hypot(*synth.baselines(a2).T)
    assert 0.75 * t["baseline_max_m"][0] < l1.max() < 1.25 * t["baseline_max_m"][0]
    assert t["baseline_max_m"][1] < l2.max() < 2.0 * 3000.0
    # channel grids: 25 MHz channels inside each array's band, as many as printed
    f2 = np.unique(synth.c2_muser1_batch().freq_hz)
    f3 = np.unique(synth.c3_muser2().freq_hz)
    for f, k in ((f2, 0), (f3, 1)):
        assert len(f) == int(t["channels"][k])
        assert np.allclose(np.diff(f), t["channel_bandwidth_mhz"][k] * 1e6)
        assert f.min() >= t["freq_lo_ghz"][k] * 1e9 and f.max() <= t["freq_hi_ghz"][k] * 1e9


def test_resolution_pixel_and_extent_follow_table2():
    t = _table1()
    bmax = t["baseline_max_m"][0]
    for r in _rows("table2_image_sizes.txt"):
        f_lo, f_hi, res_lo, res_hi, pix_lo, pix_hi, ext_lo, ext_hi = map(float, r[:8])
        n = int(r[8])
        # resolution lambda / B_max at the band edges (3 km); the printed 17.7" at 1.2 GHz
        # is the one value it does not reproduce (17.2"; the printed one matches 2.9 km)
        for f, res in ((f_lo, res_lo), (f_hi, res_hi)):
            if abs(f - 1.2) < 1e-9 and abs(res - 17.7) < 1e-9:
                assert abs(_res_arcsec(f * 1e9, bmax) - 17.2) < 0.05
                continue
            # within the printed rounding and the paper's use of c = 3e8 m/s (0.07 %)
            assert abs(_res_arcsec(f * 1e9, bmax) - res) < 0.05 + 1e-3 * res, (f, res)
        # three pixels per resolution element, the extent N pixels (the table rounds the
        # pixel before multiplying in some rows and after in others)
        for res, pix, ext in ((res_lo, pix_lo, ext_lo), (res_hi, pix_hi, ext_hi)):
            assert abs(res / 3.0 - pix) < 0.06
            err = min(abs(n * (res / 3.0) / 60.0 - ext), abs(n * pix / 60.0 - ext))
            assert err < 0.06, (n, res, pix, ext)
    # the table's extremes equal Table 1's resolution range for each array
    rows = _rows("table2_image_sizes.txt")
    assert float(rows[0][2]) == t["resolution_hi_arcsec"][0] and float(rows[2][3]) == t["resolution_lo_arcsec"][0]
    assert float(rows[3][2]) == t["resolution_hi_arcsec"][1] and float(rows[5][3]) == t["resolution_lo_arcsec"][1]
