"""FP64 Steer CLEAN (the Steer-Dewdney-Ito CLEAN) -- oracle; test infrastructure.

The paper names the Steer, Dewdney and Ito (1984) CLEAN as MUSER's deconvolver (Sec. 2;
Sec. 4.3; Algorithm 1, `improved_clean`, runs it with the loop gain 0.1 until the peak falls
to the sky level; Table 3 times its iterations), without printing its body.  As published
by Steer, Dewdney and Ito, one iteration takes as components every residual pixel whose
magnitude exceeds a trim fraction of the current peak; the component image, scaled by the
loop gain, is convolved with the dirty beam and subtracted from the residual.  Written out:

    R = dirty, model = 0
    for k < ncycle:
        peak = max |R|                       (max R with positive_only)
        stop if peak <= threshold
        S = { p : |R[p]| >= trim peak }      ({ p : R[p] >= trim peak } with positive_only)
        C = R on S, 0 elsewhere
        D = C (*) beam                        (linear convolution with the 2N beam, cropped:
                                               D[y, x] = sum_q C[q] beam[y - q_y + N, x - q_x + N])
        alpha = gain peak / max |D|
        model += alpha C;  R -= alpha D

Readings where the paper is silent (listed in the design notes): trim 0.9 by default; the
scale alpha makes the largest subtracted value gain x peak, so a selection covering an
extended source does not overshoot (for a lone point, and for trim = 1 without ties, alpha is
exactly the gain and an iteration is a Hogbom step); the convolution is linear like Hogbom's
subtraction; the stop rule is the Hogbom one on the peak.  The convolution is computed with
scipy's FFT convolution (a library primitive).

Replay.  Which pixels pass the trim is decided in floating point, so a GPU run keeps its own
selections; `replay` takes them (a bit mask per iteration) and re-runs the loop in FP64,
accepting iteration k iff the GPU's peak is within eps of the FP64 peak, every selected
pixel is at least trim x peak - eps and every other pixel below trim x peak + eps, the
selection count matches the mask, and the GPU's alpha is within 1e-4 (relative) of the FP64
alpha for that selection; it then continues with the GPU's selection.

Pins (tests/test_oracle_steer.py): trim = 1 gives Hogbom's components and maps; a lone point
source gives model S (1 - (1 - g)^n) and residual S (1 - g)^n x beam window; a flat source
under a delta beam decays as (1 - g)^n; alpha on a two-tap beam is gain / (1 + tap);
R + model (*) beam = dirty.
"""
from __future__ import annotations

import numpy as np
from scipy.signal import fftconvolve


def convolve_window(C, beam):
    """D[y, x] = sum_q C[q] beam[y - q_y + N, x - q_x + N] for the N x N map C."""
    N = C.shape[0]
    full = fftconvolve(np.asarray(C, np.float64), np.asarray(beam, np.float64), mode="full")
    return full[N:2 * N, N:2 * N]


def _peak(R, positive_only):
    return float(np.max(R)) if positive_only else float(np.max(np.abs(R)))


def _select(R, peak, trim, positive_only):
    return (R >= trim * peak) if positive_only else (np.abs(R) >= trim * peak)


def steer(dirty, beam, gain=0.1, trim=0.9, ncycle=10, threshold=0.0, positive_only=False):
    """Returns (residual, model, log) with log = [(peak, alpha, n_selected), ...] per iteration."""
    R = np.array(dirty, np.float64, copy=True)
    N = R.shape[0]
    B = np.asarray(beam, np.float64)
    assert R.shape == (N, N) and B.shape == (2 * N, 2 * N)
    model = np.zeros((N, N))
    log = []
    for _ in range(int(ncycle)):
        peak = _peak(R, positive_only)
        if peak <= threshold:
            break
        sel = _select(R, peak, trim, positive_only)
        C = np.where(sel, R, 0.0)
        D = convolve_window(C, B)
        dmax = float(np.max(np.abs(D)))
        if not dmax > 0.0:
            break
        alpha = gain * peak / dmax
        model += alpha * C
        R -= alpha * D
        log.append((peak, alpha, int(sel.sum())))
    return R, model, log


def replay(dirty, beam, masks, peaks, alphas, counts, gain=0.1, trim=0.9, threshold=0.0, positive_only=False,
           eps=None, ncycle=None):
    """Validate a Steer run made elsewhere from its per-iteration selections.

    masks: bool [K, N, N]; peaks, alphas, counts: the run's per-iteration values.  ncycle:
    when the run stopped before ncycle iterations, its next peak must be at the threshold.
    Returns (ok, first_bad_iteration, residual, model)."""
    R = np.array(dirty, np.float64, copy=True)
    N = R.shape[0]
    B = np.asarray(beam, np.float64)
    if eps is None:
        eps = 1e-5 * float(np.max(np.abs(R)))
    model = np.zeros((N, N))
    for k in range(len(masks)):
        sel = np.asarray(masks[k], bool)
        peak = _peak(R, positive_only)
        v = R if positive_only else np.abs(R)
        if peak <= threshold - eps:
            return False, k, R, model            # the loop should have stopped before k
        if abs(float(peaks[k]) - peak) > eps or int(counts[k]) != int(sel.sum()):
            return False, k, R, model
        if np.any(v[sel] < trim * peak - eps) or np.any(v[~sel] >= trim * peak + eps):
            return False, k, R, model
        C = np.where(sel, R, 0.0)
        D = convolve_window(C, B)
        dmax = float(np.max(np.abs(D)))
        alpha = gain * peak / dmax
        if abs(float(alphas[k]) - alpha) > 1e-4 * alpha:
            return False, k, R, model
        model += alpha * C
        R -= alpha * D
    if ncycle is not None and len(masks) < ncycle:
        if _peak(R, positive_only) > threshold + eps:
            return False, len(masks), R, model
    return True, -1, R, model
