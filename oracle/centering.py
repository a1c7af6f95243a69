"""FP64 disk centering and phase correction (oracle; test infrastructure).

Sec. 4.2 (disk centering correction), in three steps: the dirty map is first cleaned
until its peak is at or below the disk level mu_b of Sec. 4.1, which removes the active
regions and leaves disk and sky; that map is correlated with a simulated solar disk, and
the position of the correlation peak is the disk's offset from the field centre; the
visibilities' phases are then corrected by that offset (Algorithm 1, pre_clean and the
phase correction in improved_clean).  Readings (the paper gives no formulas):
  * the simulated disk is a uniform disk of the solar radius (in pixels) centred on pixel
    (N/2, N/2);
  * the correlation is circular, C[d] = sum_x map[x] disk[x - d] (indices mod N), computed
    with plain DFTs; its peak (largest value, ties to the lowest linear index) at d gives
    the shift, wrapped to [-N/2, N/2);
  * the peak is refined to a fraction of a pixel by a parabola through the peak and its
    two neighbours, separately in x and in y: delta = (C[-1] - C[+1]) /
    (2 (C[-1] - 2 C[0] + C[+1])), 0 if the denominator is not negative;
  * offsets in radians: (dl, dm) = (dx, dy) * cell; the correction multiplies each
    visibility by exp(+2 pi i (u dl + v dm)), which moves the disk at (dl, dm) to the
    centre (with V = sum I exp(-2 pi i (u l + v m)) and imaging exp(+)).

Pins (tests/test_oracle_centering.py): the FFT correlation equals the direct double sum on
a small map; a disk map shifted by whole pixels is found at exactly that shift; a point
source at (l0, m0) corrected by (l0, m0) has all visibilities equal to its flux; the
synthetic sky displaced by a known offset is found within a few pixels (the limit of a
plain disk template against a dirty, limb-brightened disk) and is much closer to centred
after correction.
"""
from __future__ import annotations

import numpy as np


def disk_model(N: int, radius_px: float):
    """Uniform disk of radius `radius_px` centred on pixel (N/2, N/2), FP64."""
    yy, xx = np.mgrid[0:N, 0:N]
    return (((xx - N // 2) ** 2 + (yy - N // 2) ** 2) <= radius_px * radius_px).astype(np.float64)


def correlate(img, model):
    """Circular correlation C[d] = sum_x img[x] model[x - d], FP64 via DFTs."""
    a = np.fft.fft2(np.asarray(img, np.float64))
    b = np.fft.fft2(np.asarray(model, np.float64))
    return np.real(np.fft.ifft2(a * np.conj(b)))


def _parabola(cm, c0, cp):
    den = cm - 2.0 * c0 + cp
    return (cm - cp) / (2.0 * den) if den < 0.0 else 0.0


def peak_offset(C):
    """(dx, dy) in pixels: wrapped integer peak of C plus the parabolic refinement."""
    N = C.shape[0]
    p = int(np.argmax(C))                      # lowest index among equal maxima
    py, px = divmod(p, N)
    dx = _parabola(C[py, (px - 1) % N], C[py, px], C[py, (px + 1) % N])
    dy = _parabola(C[(py - 1) % N, px], C[py, px], C[(py + 1) % N, px])
    ix = px - N if px >= N // 2 else px
    iy = py - N if py >= N // 2 else py
    return ix + dx, iy + dy


def disk_offset(img, radius_px: float, cell_rad: float):
    """(dl, dm) in radians of the disk in `img` from the field centre."""
    N = img.shape[0]
    dx, dy = peak_offset(correlate(img, disk_model(N, radius_px)))
    return dx * cell_rad, dy * cell_rad


def phase_correct(vis, uv, dl: float, dm: float):
    """vis * exp(+2 pi i (u dl + v dm)) in FP64."""
    uv = np.asarray(uv, np.float64)
    ph = 2.0 * np.pi * (uv[:, 0] * dl + uv[:, 1] * dm)
    return np.asarray(vis, np.complex128) * np.exp(1j * ph)
