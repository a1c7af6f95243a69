"""FP64 adjoint of the gridding imager: FFT then degrid (oracle; test infrastructure).

The paper has no adjoint; it is the differentiable extension of its imaging operator
(Algorithm 1's `dirty_image`).  The forward operator A maps visibilities (complex, viewed
as a real vector) to the real dirty image; weights and B0 depend on (u, v) and w_in only,
so A is real-linear in the visibilities.

Inner products are real: <a, b>_img = sum a b and <v, u>_vis = Re sum conj(v) u.  Writing
S_k(x) = sum_cell K_k(cell) exp(+2 pi i cell . x'/N), the forward operator is
    dirty(x) = sum_k 2 w_k Re(v_k S_k(x)) / (corr(x) B0)
(the mirror sample folds into the factor 2 because the kernel is real and even), hence
    (A^T y)_k = (2 w_k / B0) P(y)_k,
    P(y)_k   = sum_taps K_k(cell) F[y / (corr_x corr_y)](cell),
where F is the centred unnormalised forward DFT (exp(-...)).  P alone is the degridding
("predict") operator; it approximates the direct prediction sum_x y[x] exp(-2 pi i g . x'/N).

Pins (tests/test_oracle_adjoint.py): <A v, y> = <v, A^T y>; the brute-force transpose of A
built column by column from the forward oracle; P against the direct prediction.
"""
from __future__ import annotations

import numpy as np

from . import gcf
from .imager import Prep, weights, b0, _taps


def fft2_centred(img) -> np.ndarray:
    """F[j][i] = sum_{y,x} img[y][x] exp(-2 pi i ((i-P/2)(x-P/2) + (j-P/2)(y-P/2)) / P)."""
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(img)))


def predict(image, uv, w_in, N, cell_rad, W=gcf.W_DEFAULT, os=gcf.OS_DEFAULT, table=None):
    """P(y)_k for every visibility (zero for visibilities that are not kept)."""
    prep = Prep(uv, w_in, N, cell_rad, W, os)
    tab = gcf.kernel_table(W, os) if table is None else np.asarray(table, np.float64)
    corr = gcf.correction(N, W, os, table=tab)
    F = fft2_centred(np.asarray(image, np.float64) / np.outer(corr, corr))
    k = prep.keep
    c, o = prep.c[k], prep.o[k]
    half = (W - 1) // 2
    d = np.arange(-half, half + 1)
    tu = _taps(tab, os, W, o[:, 0])
    tv = _taps(tab, os, W, o[:, 1])
    rows = c[:, 1][:, None] + d[None, :] + N // 2           # (M, dv)
    cols = c[:, 0][:, None] + d[None, :] + N // 2           # (M, du)
    vals = F[rows[:, :, None], cols[:, None, :]]            # (M, dv, du)
    out = np.zeros(len(prep.keep), np.complex128)
    out[k] = np.einsum("mv,mu,mvu->m", tv, tu, vals)
    return out


def adjoint(image, uv, w_in, N, cell_rad, mode, W=gcf.W_DEFAULT, os=gcf.OS_DEFAULT, table=None):
    """A^T y = (2 w_k / B0_N) P(y)_k."""
    prep = Prep(uv, w_in, N, cell_rad, W, os)
    w = weights(prep, mode)
    bn = b0(prep, w, beam=False, table=table)
    if bn <= 0:
        return np.zeros(len(prep.keep), np.complex128)
    return (2.0 * w / bn) * predict(image, uv, w_in, N, cell_rad, W, os, table)


def dft_predict(image, uv, keep, N, cell_rad):
    """Direct prediction sum_x image[x] exp(-2 pi i (u l + v m)) for the kept visibilities."""
    uv64 = np.asarray(uv, np.float32).astype(np.float64)
    lm = (np.arange(N) - N // 2) * float(cell_rad)
    eu = np.exp(-2j * np.pi * np.outer(uv64[:, 0], lm))
    ev = np.exp(-2j * np.pi * np.outer(uv64[:, 1], lm))
    out = np.einsum("yx,ky,kx->k", np.asarray(image, np.float64), ev, eu)
    return np.where(keep, out, 0.0)
