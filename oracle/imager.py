"""FP64 gridding imager (oracle; test infrastructure).

Follows the dirty-image step of Algorithm 1 (`dirty_image`: weighting and gridding, then
an inverse FFT that puts the disk at the centre, returning the dirty image and the dirty
beam) with the gridding convolution function of Sec. 3.2.3 and the beam "twice as large
as the image" of Sec. 3.2.1.  Every step is written out plainly; the only library
primitives are numpy's add.at (scatter-add) and ifft2.

Conventions (the paper is silent on them; the readings are listed in the design notes):
  * arrays are row-major [y][x]; pixel (x, y) <-> (l, m) = ((x - N/2) dl, (y - N/2) dl);
  * grid cell (i, j) <-> (u, v) = ((i - P/2) du, (j - P/2) du), du = 1 / (P dl), stored
    G[j][i] (row = v);
  * visibilities follow V = sum I exp(-2 pi i (ul + vm)); imaging uses exp(+2 pi i ...);
  * the beam is computed on a 2N x 2N grid of cell du/2 with the same pixel size dl.

Prep: g = u * (N dl) in FP64; nearest cell c = rhaz(g) with rhaz(x) = sign(x) floor(|x| + 1/2);
oversampling offset o = rhaz((g - c) os).  A visibility is kept iff w_in > 0 and both
|c_u|, |c_v| <= N/2 - 1 - (W - 1)/2; the rule is symmetric, so the Hermitian mirror sample
(-c, -o, conj v) is also on the grid.  The beam grid uses g' = 2 g with the same rounding
and inherits the keep decision.

Weights (Algorithm 1, `wgtGrid_kernel`, mode 1 = uniform, otherwise natural): natural
w = w_in; uniform w = w_in / cnt(cell), cnt = sum of w_in over all samples (mirrors
included) whose nearest N-grid cell is that cell.  The paper scales the gridded cell by
1/cnt after gridding; applied per visibility before the convolution it is the same thing
whenever the kernel is a one-cell pillbox (pinned in the tests), and it is the textbook
form for a wider kernel.

Grid: G[c + d] += w v T[d_u os - o_u] T[d_v os - o_v] for d in [-(W-1)/2, (W-1)/2]^2, plus
the mirror sample.  Transform: I_raw = P^2 fftshift(ifft2(ifftshift(G))), the centred
unnormalised inverse DFT.  Normalisation: B0 = sum_samples w Tsum(o_u) Tsum(o_v) / corr(0)^2
with Tsum(o) = sum_d T[d os - o], i.e. the centre value of the weight grid's transform.
Dirty image = Re I_raw / (corr(x) corr(y) B0_N); dirty beam likewise on the 2N grid with
B0_2N, so that the beam peak at (N, N) is 1.
"""
from __future__ import annotations

import math

import numpy as np

from . import gcf


def rhaz(x):
    """Round half away from zero, written as sign(x) floor(|x| + 1/2) in FP64."""
    x = np.asarray(x, dtype=np.float64)
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


class Prep:
    """Per-visibility cell and oversampling indices on the N grid and on the 2N beam grid."""

    def __init__(self, uv, w_in, N, cell_rad, W=gcf.W_DEFAULT, os=gcf.OS_DEFAULT):
        uv64 = np.asarray(uv, dtype=np.float32).astype(np.float64)
        self.N, self.W, self.os = int(N), int(W), int(os)
        scale = float(N) * float(cell_rad)
        g = uv64 * scale
        cd = rhaz(g)
        lim = self.N // 2 - 1 - (self.W - 1) // 2
        w_in = np.asarray(w_in, dtype=np.float32).astype(np.float64)
        # keep decision in FP64 before any integer conversion (NaN/inf/huge -> dropped)
        with np.errstate(invalid="ignore"):
            self.keep = (w_in > 0) & np.all(np.abs(cd) <= lim, axis=1)
        g = np.where(self.keep[:, None], g, 0.0)
        cd = np.where(self.keep[:, None], cd, 0.0)
        self.c = cd.astype(np.int64)
        self.o = rhaz((g - cd) * os).astype(np.int64)
        g2 = 2.0 * g
        c2 = rhaz(g2)
        self.c2 = c2.astype(np.int64)
        self.o2 = rhaz((g2 - c2) * os).astype(np.int64)
        self.w_in = w_in

    @property
    def n_kept(self) -> int:
        return int(self.keep.sum())


def weights(prep: Prep, mode: int) -> np.ndarray:
    """Per-visibility weights (zero for dropped visibilities)."""
    w = np.where(prep.keep, prep.w_in, 0.0)
    if mode != 1:
        return w
    N = prep.N
    k = prep.keep
    c = prep.c[k]
    key = lambda cc: (cc[:, 1] + N) * (2 * N + 1) + (cc[:, 0] + N)
    keys = np.concatenate([key(c), key(-c)])
    wts = np.concatenate([w[k], w[k]])
    uniq, inv = np.unique(keys, return_inverse=True)
    cnt = np.zeros(len(uniq))
    np.add.at(cnt, inv, wts)
    out = np.zeros_like(w)
    out[k] = w[k] / cnt[inv[: len(c)]]
    return out


def _taps(table, os, W, o):
    """(M, W) kernel weights T[d os - o] for d = -(W-1)/2 .. (W-1)/2."""
    half = (W - 1) // 2
    centre = (len(table) - 1) // 2
    d = np.arange(-half, half + 1)
    return table[centre + d[None, :] * os - o[:, None]]


def grid(prep: Prep, vis, w, beam: bool = False, table=None) -> np.ndarray:
    """Full centred P x P complex grid G[j][i] (P = N, or 2N for the beam with vis = 1)."""
    W, os = prep.W, prep.os
    tab = gcf.kernel_table(W, os) if table is None else np.asarray(table, dtype=np.float64)
    P = 2 * prep.N if beam else prep.N
    c, o = (prep.c2, prep.o2) if beam else (prep.c, prep.o)
    k = prep.keep
    c, o, wk = c[k], o[k], w[k]
    # FP32 inputs are promoted exactly; FP64 inputs (finite-difference checks) keep their precision
    val = np.ones(len(wk), np.complex128) if beam else np.asarray(vis).astype(np.complex128)[k]
    half = (W - 1) // 2
    G = np.zeros((P, P), np.complex128)
    d = np.arange(-half, half + 1)
    for sgn, vv in ((1, val), (-1, np.conj(val))):
        cs, osg = sgn * c, sgn * o
        tu = _taps(tab, os, W, osg[:, 0])          # (M, W)
        tv = _taps(tab, os, W, osg[:, 1])
        contrib = (wk * vv)[:, None, None] * tv[:, :, None] * tu[:, None, :]   # (M, dv, du)
        rows = (cs[:, 1][:, None, None] + d[None, :, None] + P // 2) + 0 * d[None, None, :]
        cols = (cs[:, 0][:, None, None] + d[None, None, :] + P // 2) + 0 * d[None, :, None]
        np.add.at(G, (rows.ravel(), cols.ravel()), contrib.ravel())
    return G


def b0(prep: Prep, w, beam: bool = False, table=None) -> float:
    """Centre value of the transformed weight grid divided by corr(0)^2."""
    W, os = prep.W, prep.os
    tab = gcf.kernel_table(W, os) if table is None else np.asarray(table, dtype=np.float64)
    c0 = float(np.sum(tab)) / os                      # corr(0)
    o = prep.o2 if beam else prep.o
    k = prep.keep
    tsu = _taps(tab, os, W, o[k, 0]).sum(axis=1)
    tsv = _taps(tab, os, W, o[k, 1]).sum(axis=1)
    return float(np.sum(2.0 * w[k] * tsu * tsv) / (c0 * c0))


def ifft2_centred(G) -> np.ndarray:
    """I[y][x] = sum_{j,i} G[j][i] exp(+2 pi i ((i-P/2)(x-P/2) + (j-P/2)(y-P/2)) / P)."""
    P0, P1 = G.shape
    return P0 * P1 * np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(G)))


def dirty_image(vis, uv, w_in, N, cell_rad, mode, W=gcf.W_DEFAULT, os=gcf.OS_DEFAULT, table=None,
                return_parts=False):
    """FP64 dirty image (N x N), and optionally its parts (prep, weights, grid, B0, raw)."""
    prep = Prep(uv, w_in, N, cell_rad, W, os)
    w = weights(prep, mode)
    G = grid(prep, vis, w, beam=False, table=table)
    bn = b0(prep, w, beam=False, table=table)
    raw = ifft2_centred(G)
    corr = gcf.correction(N, W, os, table=table)
    img = raw.real / (np.outer(corr, corr) * bn) if bn > 0 else np.zeros((N, N))
    if return_parts:
        return img, dict(prep=prep, w=w, grid=G, b0=bn, raw=raw, corr=corr)
    return img


def dirty_beam(uv, w_in, N, cell_rad, mode, W=gcf.W_DEFAULT, os=gcf.OS_DEFAULT, table=None,
               return_parts=False):
    """FP64 dirty beam (2N x 2N, peak 1 at (N, N))."""
    prep = Prep(uv, w_in, N, cell_rad, W, os)
    w = weights(prep, mode)
    G = grid(prep, None, w, beam=True, table=table)
    bn = b0(prep, w, beam=True, table=table)
    raw = ifft2_centred(G)
    corr = gcf.correction(2 * N, W, os, table=table)
    img = raw.real / (np.outer(corr, corr) * bn) if bn > 0 else np.zeros((2 * N, 2 * N))
    if return_parts:
        return img, dict(prep=prep, w=w, grid=G, b0=bn, raw=raw, corr=corr)
    return img


def dft_image(vis, uv, w, keep, N, cell_rad):
    """Direct (ungridded) DFT imager over the kept samples and their mirrors:
    I(x, y) = sum_k 2 w_k Re(v_k exp(+2 pi i (u_k l + v_k m))) / sum_k 2 w_k."""
    uv64 = np.asarray(uv, np.float32).astype(np.float64)[keep]
    v = np.asarray(vis, np.complex64).astype(np.complex128)[keep]
    wk = np.asarray(w, np.float64)[keep]
    lm = (np.arange(N) - N // 2) * float(cell_rad)
    eu = np.exp(2j * math.pi * np.outer(uv64[:, 0], lm))     # (M, x)
    ev = np.exp(2j * math.pi * np.outer(uv64[:, 1], lm))     # (M, y)
    img = np.einsum("k,ky,kx->yx", wk * v, ev, eu)
    return 2.0 * img.real / (2.0 * wk.sum())


def image_batch(wl, beam=True):
    """Dirty images (and beams) for every instance of a workload (list of arrays)."""
    dirty, beams, b0s = [], [], []
    for i in range(wl.n_inst):
        v, uv, w = wl.instance(i)
        N, cell, mode = int(wl.n_img[i]), float(wl.cell_rad[i]), int(wl.weight_mode[i])
        img, parts = dirty_image(v, uv, w, N, cell, mode, return_parts=True)
        dirty.append(img)
        b0s.append(parts["b0"])
        if beam:
            beams.append(dirty_beam(uv, w, N, cell, mode))
    return dirty, beams, b0s
