"""FP64 w-projection imager (oracle; test infrastructure).

Sec. 3.2.2 and 6.1: the imaging relation is a 2-D Fourier transform only while the phase
pi (l^2 + m^2) w stays well below one radian (up to about 0.1 rad is tolerable); otherwise
the w-term is corrected by w-projection before the inverse FFT (Algorithm 1's "W-term
correction"), and it can be skipped when the phase is small enough.  The paper names the
method and the criterion, not the kernels; the readings below are the textbook
construction, with the parameters chosen here:

  * measurement V(u, v, w) = sum I exp(-2 pi i (u l + v m + w (n - 1))), n = sqrt(1 - l^2 - m^2);
    the exact dirty image is I(x, y) = sum_k 2 w_k Re(V_k exp(+2 pi i (u l + v m + w (n - 1))))
    / sum_k 2 w_k over the kept samples (their mirrors (-u, -v, -w, conj V) give the
    conjugate terms);
  * phase tolerance tol (default 0.1 rad): r2 = l^2 + m^2 at the field corner,
    r2 = 2 (N dl / 2)^2; planes w_j = j dw, dw = tol / (pi r2), j = 0 .. n_planes - 1 with
    n_planes = floor(w_max / dw + 1/2) + 1, so rounding |w| to its plane moves the phase at
    the corner by at most tol / 2; one plane (no correction) when pi w_max r2 <= tol / 2;
  * support of plane j (cells, odd): S_j = 2 (3 + ceil(w_j sqrt(r2) N dl)) + 1, i.e. the
    W = 7 prolate spheroidal support widened on each side by the largest uv frequency (in
    cells) of the w-screen over the field;
  * kernel of plane j: K_j(du, dv) = (1/M^2) sum_{a, b} A(a) A(b) exp(+2 pi i w_j (n - 1))
    exp(-2 pi i (du a + dv b) / M) over a, b = -(M/2 - 1) .. M/2 - 1, with M = 64 points
    across the field (l = a (N/M) dl), A(a) = corr(a N / M) the grid-correction function
    of the W = 7 kernel; for w = 0 this is the prolate spheroidal kernel C(du) C(dv) up to
    its truncation at the field edge.  The sample set is symmetric, so K_{-w} = conj(K_w)
    and K_w(-d) = K_w(d);
  * tables: K_j at du, dv = t / OSW (OSW = 16 points per cell), t = -S_j OSW / 2 .. S_j OSW / 2;
    a tap at offset d - f from a sample at fractional cell offset f takes the bilinear
    interpolation of the table;
  * gridding: G[c + d] += w V K_j(d - f) for d in [-(S_j - 1)/2, (S_j - 1)/2]^2, plane j of
    |w| (K conjugated for w < 0), and the mirror sample likewise; taps with |c + d| >= N/2
    in either axis are dropped (so the mirror taps are dropped with them);
  * then the 2-D path's transform, correction by corr(x) corr(y) and normalisation by B0.

Pins (tests/test_oracle_wproj.py): the exact imager at w = 0 equals the 2-D direct DFT;
K_0 matches the prolate spheroidal table product; K_{-w} = conj K_w and K_w is even; the
plane spacing meets the phase rule; a point source's visibilities at large w are imaged by
w-projection 50x closer to the exact image than by the 2-D imager (inside the outermost 4
pixels, where gridding at any w departs from the direct transform), and at w = 0 both agree.
"""
from __future__ import annotations

import math

import numpy as np

from . import gcf, imager

M_FIELD = 64        # points across the field in the kernel construction
OSW = 16            # kernel table points per cell
HALF_PSWF = 3       # half-width of the W = 7 prolate spheroidal support


def exact_dirty(vis, uv, wlam, w, keep, N, cell_rad):
    """Direct dirty image with the w-term, FP64, over the kept samples and their mirrors."""
    u = np.asarray(uv, np.float32).astype(np.float64)[keep]
    ww = np.asarray(wlam, np.float32).astype(np.float64)[keep]
    v = np.asarray(vis, np.complex64).astype(np.complex128)[keep]
    wk = np.asarray(w, np.float64)[keep]
    lm = (np.arange(N) - N // 2) * float(cell_rad)
    L, Mm = np.meshgrid(lm, lm)                       # [y][x]
    nm1 = np.sqrt(1.0 - L * L - Mm * Mm) - 1.0
    img = np.zeros((N, N))
    for k in range(len(wk)):
        ph = 2.0 * math.pi * (u[k, 0] * L + u[k, 1] * Mm + ww[k] * nm1)
        img += 2.0 * wk[k] * np.real(v[k] * np.exp(1j * ph))
    return img / (2.0 * wk.sum())


def corner_r2(N, cell_rad):
    half = 0.5 * N * float(cell_rad)
    return 2.0 * half * half


def plan(w_max, N, cell_rad, tol=0.1):
    """(dw, n_planes, supports) for an instance whose samples have |w| <= w_max."""
    r2 = corner_r2(N, cell_rad)
    dw = tol / (math.pi * r2)
    n_planes = int(math.floor(float(w_max) / dw + 0.5)) + 1
    fov = N * float(cell_rad)
    sup = [2 * (HALF_PSWF + int(math.ceil(j * dw * math.sqrt(r2) * fov))) + 1 for j in range(n_planes)]
    return dw, n_planes, sup


def kernel_table(wj, S, N, cell_rad, osw=OSW, M=M_FIELD):
    """K_j at du, dv = t / osw for t = -S osw/2 .. S osw/2 (complex, [dv][du])."""
    a = np.arange(-(M // 2 - 1), M // 2)              # symmetric point set
    corr = gcf.correction(N)                          # corr(x - N/2), x = 0..N-1
    A = corr[a * (N // M) + N // 2]
    l = a * (N // M) * float(cell_rad)
    Lg, Mg = np.meshgrid(l, l)                        # [b][a]
    screen = np.outer(A, A) * np.exp(2j * math.pi * wj * (np.sqrt(1.0 - Lg * Lg - Mg * Mg) - 1.0))
    half = S * osw // 2
    d = np.arange(-half, half + 1) / osw
    E = np.exp(-2j * math.pi * np.outer(d, a) / M) / M     # (n_d, n_a)
    return E @ screen @ E.T                           # [dv][du]


def _bilinear(tab, half, x, y):
    """Table value at fractional table coordinates (x along du, y along dv), relative to the centre."""
    x0 = np.minimum(np.floor(x), half - 1).astype(np.int64)     # the last interval includes its end
    y0 = np.minimum(np.floor(y), half - 1).astype(np.int64)
    fx, fy = x - x0, y - y0
    i0, j0 = x0 + half, y0 + half
    return ((1 - fy) * ((1 - fx) * tab[j0, i0] + fx * tab[j0, i0 + 1]) +
            fy * ((1 - fx) * tab[j0 + 1, i0] + fx * tab[j0 + 1, i0 + 1]))


def grid_w(prep, uv, cell, vis, wlam, w, w_max, tol=0.1, osw=OSW):
    """Full centred N x N complex grid with w-projection kernels; also returns the plan."""
    N = prep.N
    cell = float(cell)
    dw, n_planes, sup = plan(w_max, N, cell, tol)
    tabs = [kernel_table(j * dw, sup[j], N, cell, osw) for j in range(n_planes)]
    k = prep.keep
    uv64 = np.asarray(uv, np.float32).astype(np.float64)[k]
    g = uv64 * (N * cell)
    cf = imager.rhaz(g)
    f = g - cf
    c = cf.astype(np.int64)
    ww = np.asarray(wlam, np.float32).astype(np.float64)[k]
    val = np.asarray(vis).astype(np.complex128)[k]
    wk = np.asarray(w, np.float64)[k]
    G = np.zeros((N, N), np.complex128)
    for s in range(len(wk)):
        j = min(int(imager.rhaz(abs(ww[s]) / dw)), n_planes - 1)
        S = sup[j]
        H = (S - 1) // 2
        half = S * osw // 2
        d = np.arange(-H, H + 1)
        for sgn, vv, wsign in ((1, val[s], ww[s]), (-1, np.conj(val[s]), -ww[s])):
            cs, fs = sgn * c[s], sgn * f[s]
            X, Y = np.meshgrid((d - fs[0]) * osw, (d - fs[1]) * osw)     # [dv][du]
            kv = _bilinear(tabs[j], half, X, Y)
            if wsign < 0:
                kv = np.conj(kv)
            cu = cs[0] + d
            cv = cs[1] + d
            okx = np.abs(cu) < N // 2
            oky = np.abs(cv) < N // 2
            sub = (wk[s] * vv) * kv
            rows = (cv + N // 2)[oky]
            cols = (cu + N // 2)[okx]
            G[np.ix_(rows, cols)] += sub[np.ix_(oky, okx)]
    return G, (dw, n_planes, sup)


def dirty_image_w(vis, uv, wlam, w_in, N, cell_rad, mode, w_max, tol=0.1):
    """FP64 w-projected dirty image (N x N), normalised like the 2-D path."""
    prep = imager.Prep(uv, w_in, N, cell_rad)
    w = imager.weights(prep, mode)
    G, pl = grid_w(prep, uv, cell_rad, vis, wlam, w, w_max, tol)
    bn = imager.b0(prep, w)
    raw = imager.ifft2_centred(G)
    corr = gcf.correction(N)
    img = raw.real / (np.outer(corr, corr) * bn) if bn > 0 else np.zeros((N, N))
    return img, pl
