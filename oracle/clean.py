"""FP64 Hogbom CLEAN, clean-beam fit and restore (oracle; test infrastructure).

Algorithm 1 (`improved_clean`) finds the strength and position of the peak of the map,
then repeatedly runs a CLEAN iteration and searches for the peak again while the peak is
above the sky level mu_a; Sec. 4.3 fixes the loop gain at gamma = 0.1 and uses the
threshold to stop.  The paper's production deconvolver is Steer CLEAN; the hot path here
is the classic Hogbom CLEAN (Sec. 2) it builds on:

    R = dirty, model = 0
    for i < niter:
        p = argmax |R| (ties: lowest linear index y N + x)
        stop if |R[p]| <= threshold
        f = gamma R[p];  model[p] += f;  record (p, f)
        R[y, x] -= f beam[y - p_y + N, x - p_x + N]     for all (x, y) in the N x N map

The beam is the 2N x 2N dirty beam (peak at (N, N)), "twice as large as the image" so a
point can be subtracted from any pixel (Sec. 3.2.1).

Window (the paper is silent; reading: the whole map by default): an optional box
(x0, y0, x1, y1), half-open, restricts where the peak is searched; the subtraction still
covers the whole map.  Peaks and ties are taken over the box's pixels in row-major order,
which is the map's linear order restricted to the box.

Clean beam (Algorithm 1's `gpu_cpsf`; the paper does not say how it is made): the main
lobe is the 4-connected region around (N, N) where the beam exceeds 0.35; a Gaussian with
peak 1, exp(-(a dx^2 + b dx dy + c dy^2)), is fitted to ln(beam) over the lobe by linear
least squares.  Restored image = R + model convolved (linear, not circular) with that
Gaussian, cropped to N x N.

Pins (tests/test_oracle_clean.py): a single point source gives model = S (1 - (1-g)^n) and
residual = S (1-g)^n times the beam window; gain 1 stops after one pick; niter 0 leaves R
equal to the dirty map; equal peaks resolve to the lower index; R + model (*) beam window
reproduces the dirty map; an exactly Gaussian beam is fitted exactly.
"""
from __future__ import annotations

import math
from collections import deque

import numpy as np


def _window(beam, N, py, px):
    return beam[N - py: 2 * N - py, N - px: 2 * N - px]


def _box(window, N):
    x0, y0, x1, y1 = (0, 0, N, N) if window is None else (int(v) for v in window)
    assert 0 <= x0 < x1 <= N and 0 <= y0 < y1 <= N, "window must be a non-empty box inside the map"
    return x0, y0, x1, y1


def _peak(R, window, positive_only):
    """(py, px) of the first maximum of R (or |R|) over the window box."""
    x0, y0, x1, y1 = _box(window, R.shape[0])
    sub = R[y0:y1, x0:x1]
    q = int(np.argmax(sub if positive_only else np.abs(sub)))   # first maximum = lowest index
    qy, qx = divmod(q, x1 - x0)
    return y0 + qy, x0 + qx


def hogbom(dirty, beam, gain=0.1, niter=100, threshold=0.0, positive_only=False, window=None):
    """Returns (residual, model, comp_idx, comp_flux)."""
    R = np.array(dirty, dtype=np.float64, copy=True)
    N = R.shape[0]
    B = np.asarray(beam, dtype=np.float64)
    assert R.shape == (N, N) and B.shape == (2 * N, 2 * N)
    model = np.zeros((N, N))
    idx, flux = [], []
    for _ in range(int(niter)):
        py, px = _peak(R, window, positive_only)
        p = py * N + px
        peak = R[py, px]
        if abs(peak) <= threshold:
            break
        f = gain * peak
        model[py, px] += f
        idx.append(p)
        flux.append(f)
        R -= f * _window(B, N, py, px)
    return R, model, np.asarray(idx, np.int64), np.asarray(flux, np.float64)


def replay(dirty, beam, comp_idx, comp_flux, gain=0.1, threshold=0.0, eps=None, n_stop=None,
           positive_only=False, window=None):
    """Validate a component list produced elsewhere (several answers are correct under near-ties).

    Re-runs the loop in FP64 following the given picks: pick i is accepted iff its peak
    value (|R_i[p_i]|, or R_i[p_i] with positive_only) is within eps of the peak value over
    the window (the whole map by default), p_i lies in the window, that peak value is above
    threshold - eps (the loop runs only while the peak exceeds the threshold), and
    |flux_i - gain R_i[p_i]| <= gain eps.  Returns (ok, first_bad_index,
    residual, model).  eps defaults to 1e-5 max|dirty|.
    """
    R = np.array(dirty, dtype=np.float64, copy=True)
    N = R.shape[0]
    B = np.asarray(beam, dtype=np.float64)
    if eps is None:
        eps = 1e-5 * float(np.max(np.abs(R)))
    model = np.zeros((N, N))
    x0, y0, x1, y1 = _box(window, N)
    for i, (p, fl) in enumerate(zip(np.asarray(comp_idx), np.asarray(comp_flux))):
        p = int(p)
        py, px = divmod(p, N)
        sub = R[y0:y1, x0:x1]
        if positive_only:
            m, val = float(np.max(sub)), R[py, px]
        else:
            m, val = float(np.max(np.abs(sub))), abs(R[py, px])
        inside = x0 <= px < x1 and y0 <= py < y1
        if not inside or val < m - eps or m <= threshold - eps or abs(fl - gain * R[py, px]) > gain * eps:
            return False, i, R, model
        f = gain * R[py, px]
        model[py, px] += f
        R -= f * _window(B, N, py, px)
    if n_stop is not None and n_stop < len(comp_idx):
        return False, n_stop, R, model
    return True, -1, R, model


def main_lobe(beam, threshold=0.35):
    """4-connected region around the centre (N, N) where beam > threshold (boolean mask)."""
    P = beam.shape[0]
    c = P // 2
    mask = np.zeros(beam.shape, bool)
    if not beam[c, c] > threshold:
        return mask
    q = deque([(c, c)])
    mask[c, c] = True
    while q:
        y, x = q.popleft()
        for dy, dx in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            yy, xx = y + dy, x + dx
            if 0 <= yy < P and 0 <= xx < P and not mask[yy, xx] and beam[yy, xx] > threshold:
                mask[yy, xx] = True
                q.append((yy, xx))
    return mask


DEGENERATE_ABC = (4.0 * math.log(2.0), 0.0, 4.0 * math.log(2.0))   # FWHM of one pixel


def fit_clean_beam(beam, threshold=0.35, return_flag=False):
    """Least-squares Gaussian fit; returns (a, b, c, bmaj_px, bmin_px, pa_rad).

    bmaj/bmin are FWHM in pixels; pa is the angle of the major axis from +x towards +y.
    Degenerate lobes are decided by pixel counts: if no lobe pixel has dx dy != 0, the
    cross term is fixed at b = 0 and (a, c) are fitted (both axes must hold pixels);
    otherwise, or if the 3 x 3 system is numerically singular, the fit falls back to a
    one-pixel FWHM circular Gaussian and the flag is set.
    """
    B = np.asarray(beam, np.float64)
    P = B.shape[0]
    c0 = P // 2
    mask = main_lobe(B, threshold)
    ys, xs = np.nonzero(mask)
    dx = (xs - c0).astype(np.float64)
    dy = (ys - c0).astype(np.float64)
    rhs = -np.log(B[ys, xs])
    degenerate = False
    if np.any(dx * dy != 0):
        A = np.stack([dx * dx, dx * dy, dy * dy], axis=1)
        ata = A.T @ A
        det = np.linalg.det(ata)
        if abs(det) < 1e-9 * abs(ata[0, 0] * ata[1, 1] * ata[2, 2]):
            degenerate = True
        else:
            a, b, c = np.linalg.solve(ata, A.T @ rhs)
    elif np.any(dx != 0) and np.any(dy != 0):
        A = np.stack([dx * dx, dy * dy], axis=1)
        a, c = np.linalg.solve(A.T @ A, A.T @ rhs)
        b = 0.0
    else:
        degenerate = True
    if degenerate:
        a, b, c = DEGENERATE_ABC
    out = (a, b, c) + gaussian_axes(a, b, c)
    return (out, degenerate) if return_flag else out


def gaussian_axes(a, b, c):
    q = np.array([[a, b / 2.0], [b / 2.0, c]])
    ev, evec = np.linalg.eigh(q)            # ascending: ev[0] smallest -> major axis
    lmin, lmax = ev
    bmaj = 2.0 * math.sqrt(math.log(2.0) / lmin)
    bmin = 2.0 * math.sqrt(math.log(2.0) / lmax)
    vx, vy = evec[:, 0]
    pa = math.atan2(vy, vx)
    if pa < 0:
        pa += math.pi
    if pa >= math.pi:
        pa -= math.pi
    return bmaj, bmin, pa


def restore(residual, model, abc):
    """R + sum over model pixels of model[p] exp(-(a dx^2 + b dx dy + c dy^2)), full extent."""
    a, b, c = abc[:3]
    N = residual.shape[0]
    out = np.array(residual, np.float64, copy=True)
    yy, xx = np.mgrid[0:N, 0:N]
    for p in np.flatnonzero(model):
        py, px = divmod(int(p), N)
        dx = xx - px
        dy = yy - py
        out += model[py, px] * np.exp(-(a * dx * dx + b * dx * dy + c * dy * dy))
    return out


def restore_conv(residual, model, abc, radius=None):
    """The same restore as `restore`, by one FFT convolution of the model with the Gaussian
    sampled at every offset |dx|, |dy| <= radius (default N - 1: every offset between two
    pixels of the map, i.e. the full extent).  scipy's FFT convolution is a library primitive."""
    from scipy.signal import fftconvolve
    a, b, c = abc[:3]
    N = residual.shape[0]
    r = N - 1 if radius is None else min(int(radius), N - 1)
    d = np.arange(-r, r + 1, dtype=np.float64)
    dy, dx = np.meshgrid(d, d, indexing="ij")
    G = np.exp(-(a * dx * dx + b * dx * dy + c * dy * dy))
    full = fftconvolve(np.asarray(model, np.float64), G, mode="full")
    return np.asarray(residual, np.float64) + full[r:r + N, r:r + N]


def clean_identity(dirty, beam, residual, model):
    """max |R + model (*) beam window - dirty| (linear convolution with the 2N beam)."""
    N = dirty.shape[0]
    acc = np.array(residual, np.float64, copy=True)
    for p in np.flatnonzero(model):
        py, px = divmod(int(p), N)
        acc += model[py, px] * _window(np.asarray(beam, np.float64), N, py, px)
    return float(np.max(np.abs(acc - dirty)))
