"""Pins of the FP64 Steer CLEAN oracle (the Steer-Dewdney-Ito CLEAN named by the paper)."""
import numpy as np
import pytest

from oracle import clean, imager, steer
from paper_1712_06913_amd import synth


def _maps(seed, N, m=250):
    wl = synth.random_instances(seed, [N], m_range=(m, m), uniform_frac=0.0)
    v, uv, w = wl.instance(0)
    cell = float(wl.cell_rad[0])
    return imager.dirty_image(v, uv, w, N, cell, 0), imager.dirty_beam(uv, w, N, cell, 0)


def test_trim_one_is_hogbom():
    D, B = _maps(51, 64)
    R0, M0, idx, flux = clean.hogbom(D, B, gain=0.1, niter=40)
    R1, M1, log = steer.steer(D, B, gain=0.1, trim=1.0, ncycle=40)
    assert len(log) == 40 and all(n == 1 for _, _, n in log)
    assert all(abs(a - 0.1) < 1e-12 for _, a, _ in log)
    assert np.max(np.abs(R1 - R0)) < 1e-11 * np.max(np.abs(D))
    assert np.max(np.abs(M1 - M0)) < 1e-12 * np.max(np.abs(D))
    assert set(np.flatnonzero(M1)) == set(int(p) for p in idx)


@pytest.mark.parametrize("positive_only", [False, True])
def test_lone_point_source_closed_form(positive_only):
    N, S, py, px, g, n = 64, 2.5, 21, 40, 0.1, 25
    yy, xx = np.mgrid[0:2 * N, 0:2 * N]
    B = np.exp(-((xx - N) ** 2 + (yy - N) ** 2) / 0.5)        # second largest value e^-2 < trim
    D = S * B[N - py: 2 * N - py, N - px: 2 * N - px]
    R, M, log = steer.steer(D, B, gain=g, trim=0.5, ncycle=n, positive_only=positive_only)
    assert all(c == 1 for _, _, c in log)
    assert abs(M[py, px] - S * (1 - (1 - g) ** n)) < 1e-12 * S and np.count_nonzero(M) == 1
    assert np.max(np.abs(R - S * (1 - g) ** n * B[N - py: 2 * N - py, N - px: 2 * N - px])) < 1e-12 * S


def test_flat_source_under_delta_beam_decays_geometrically():
    N, g, n = 32, 0.1, 12
    B = np.zeros((2 * N, 2 * N))
    B[N, N] = 1.0
    D = np.zeros((N, N))
    D[8:20, 5:25] = 3.0
    R, M, log = steer.steer(D, B, gain=g, trim=0.9, ncycle=n)
    assert all(c == 12 * 20 for _, _, c in log)
    assert np.max(np.abs(R - D * (1 - g) ** n)) < 1e-12
    assert np.max(np.abs(M - D * (1 - (1 - g) ** n))) < 1e-12


def test_alpha_on_a_two_tap_beam():
    # beam = delta + t at offset (+1 in x): a flat patch gives max|D| = (1 + t) v inside it
    N, g, t = 32, 0.2, 0.5
    B = np.zeros((2 * N, 2 * N))
    B[N, N] = 1.0
    B[N, N + 1] = t
    D = np.zeros((N, N))
    D[10:14, 10:20] = 1.0
    _, _, log = steer.steer(D, B, gain=g, trim=0.9, ncycle=1)
    peak, alpha, cnt = log[0]
    assert peak == 1.0 and cnt == 40
    assert abs(alpha - g / (1 + t)) < 1e-14


@pytest.mark.parametrize("positive_only", [False, True])
def test_clean_identity_and_replay_of_itself(positive_only):
    D, B = _maps(52, 64)
    R, M, log = steer.steer(D, B, gain=0.1, trim=0.8, ncycle=15, positive_only=positive_only)
    assert clean.clean_identity(D, B, R, M) < 1e-12 * np.max(np.abs(D))
    # the replay accepts the oracle's own selections and reproduces its maps
    masks, Rk = [], np.array(D)
    Rk_model = np.zeros_like(D)
    for peak, alpha, cnt in log:
        v = Rk if positive_only else np.abs(Rk)
        sel = v >= 0.8 * peak
        masks.append(sel)
        C = np.where(sel, Rk, 0.0)
        Rk = Rk - alpha * steer.convolve_window(C, B)
        Rk_model += alpha * C
    ok, bad, R2, M2 = steer.replay(D, B, masks, [x[0] for x in log], [x[1] for x in log], [x[2] for x in log],
                                   trim=0.8, positive_only=positive_only, ncycle=15)
    assert ok, bad
    assert np.max(np.abs(R2 - R)) < 1e-12 * np.max(np.abs(D))
    # a selection that drops a pixel well above the trim is rejected
    bad_masks = [m.copy() for m in masks]
    q = np.flatnonzero(bad_masks[2])[0]
    bad_masks[2].flat[q] = False
    ok, bad, _, _ = steer.replay(D, B, bad_masks, [x[0] for x in log], [x[1] for x in log],
                                 [x[2] - (k == 2) for k, x in enumerate(log)], trim=0.8,
                                 positive_only=positive_only, ncycle=15)
    assert not ok and bad == 2


def test_convolve_window_is_the_direct_sum():
    rng = np.random.default_rng(53)
    N = 12
    C = np.zeros((N, N))
    C.flat[rng.choice(N * N, 7, replace=False)] = rng.standard_normal(7)
    B = rng.standard_normal((2 * N, 2 * N))
    ref = np.zeros((N, N))
    for q in np.flatnonzero(C):
        qy, qx = divmod(int(q), N)
        ref += C[qy, qx] * B[N - qy: 2 * N - qy, N - qx: 2 * N - qx]
    assert np.max(np.abs(steer.convolve_window(C, B) - ref)) < 1e-12
