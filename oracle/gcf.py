"""Gridding convolution function (GCF) and grid correction, FP64 (oracle; test infrastructure).

Sec. 3.2.3 (gridding convolution function): the visibilities are convolved with a
truncated prolate spheroidal function following Schwab's optimal-gridding analysis.  The
paper names the function family but prints neither its parameters nor coefficients, so
this module computes it from its defining eigen-equation instead of any published rational
approximation:

    psi(nu) is the leading eigenfunction of
        integral_{-1}^{1} (1 - t^2)^alpha cos(c nu t) psi(t) dt = lambda psi(nu)

    C(D) = (1 - (2D/W)^2)^alpha psi(2D/W)      for |D| <= W/2, zero outside,

with support W = 7 cells, alpha = 1 and c = pi W / 2.  The eigen-problem is solved by
Nystrom discretisation on Gauss-Legendre nodes.  The kernel is tabulated at `os` points
per cell (T[t] = C(t/os), t = -os W/2 .. os W/2) and normalised to T[0] = 1.

Grid correction: corr(x') = (1/os) sum_t T[t] cos(2 pi t x' / (os P)) is the discrete-time
Fourier transform of the table evaluated at image offset x' on a P-point grid.

Pins (tests/test_oracle_gcf.py): alpha = 0 against scipy.special.pro_ang1; eigen-equation
residual checked with an independent higher-order quadrature; corr/corr(0) against
psi(2x'/P)/psi(0).
"""
from __future__ import annotations

import functools
import math

import numpy as np

W_DEFAULT = 7
OS_DEFAULT = 128
ALPHA_DEFAULT = 1.0


@functools.lru_cache(maxsize=16)
def _nystrom(alpha: float, c: float, n_nodes: int):
    t, a = np.polynomial.legendre.leggauss(n_nodes)
    d = a * (1.0 - t * t) ** alpha
    k = np.cos(c * np.outer(t, t))
    sq = np.sqrt(d)
    b = sq[:, None] * k * sq[None, :]          # symmetric form of the Nystrom matrix
    evals, evecs = np.linalg.eigh(b)
    lam = evals[-1]
    psi_nodes = evecs[:, -1] / sq
    if psi_nodes[n_nodes // 2] < 0:
        psi_nodes = -psi_nodes
    return t, d, lam, psi_nodes


def pswf(nu, alpha: float = ALPHA_DEFAULT, c: float = math.pi * W_DEFAULT / 2.0, n_nodes: int = 200):
    """Leading eigenfunction psi(nu) of the weighted finite cosine transform (unnormalised)."""
    t, d, lam, psi_nodes = _nystrom(float(alpha), float(c), int(n_nodes))
    nu = np.asarray(nu, dtype=np.float64)
    return (np.cos(c * np.multiply.outer(nu, t)) @ (d * psi_nodes)) / lam


def pswf_eigenvalue(alpha: float = ALPHA_DEFAULT, c: float = math.pi * W_DEFAULT / 2.0, n_nodes: int = 200):
    return _nystrom(float(alpha), float(c), int(n_nodes))[2]


def gcf(delta, W: int = W_DEFAULT, alpha: float = ALPHA_DEFAULT):
    """C(D) for offsets D in cells (unnormalised); zero outside |D| <= W/2."""
    delta = np.asarray(delta, dtype=np.float64)
    eta = 2.0 * delta / W
    out = np.zeros_like(eta)
    inside = np.abs(eta) <= 1.0
    e = eta[inside]
    out[inside] = (1.0 - e * e) ** alpha * pswf(e, alpha, math.pi * W / 2.0)
    return out


@functools.lru_cache(maxsize=16)
def kernel_table(W: int = W_DEFAULT, os: int = OS_DEFAULT, alpha: float = ALPHA_DEFAULT) -> np.ndarray:
    """T[t + os W/2] = C(t/os) / C(0) for t = -os W/2 .. os W/2 (os W/2 must be an integer)."""
    half = os * W // 2
    assert half * 2 == os * W, "os * W must be even"
    t = np.arange(-half, half + 1, dtype=np.float64)
    tab = gcf(t / os, W, alpha)
    tab = tab / tab[half]
    tab.setflags(write=False)
    return tab


def correction(P: int, W: int = W_DEFAULT, os: int = OS_DEFAULT, alpha: float = ALPHA_DEFAULT,
               table: np.ndarray | None = None) -> np.ndarray:
    """corr(x - P/2) for x = 0..P-1 on a P-point grid (DTFT of the tabulated kernel)."""
    tab = kernel_table(W, os, alpha) if table is None else table
    half = (len(tab) - 1) // 2
    t = np.arange(-half, half + 1, dtype=np.float64)
    xp = np.arange(P, dtype=np.float64) - P // 2
    return (np.cos(2.0 * math.pi * np.outer(xp, t) / (os * P)) @ tab) / os
