"""Pins of the oracle adjoint (degrid) of the gridding imager."""
import numpy as np
import pytest

from oracle import adjoint, imager
from paper_1712_06913_amd import synth


def _inst(seed, N, m, uf=0.5):
    wl = synth.random_instances(seed, [N], m_range=(m, m), uniform_frac=uf)
    v, uv, w = wl.instance(0)
    return v, uv, w, N, float(wl.cell_rad[0]), int(wl.weight_mode[0])


@pytest.mark.parametrize("mode", [0, 1])
def test_dot_product_identity(mode):
    v, uv, w, N, cell, _ = _inst(21, 32, 70)
    rng = np.random.default_rng(5)
    y = rng.standard_normal((N, N))
    Av = imager.dirty_image(v, uv, w, N, cell, mode)
    ATy = adjoint.adjoint(y, uv, w, N, cell, mode)
    lhs = np.sum(Av * y)
    rhs = np.real(np.sum(np.conj(v.astype(np.complex128)) * ATy))
    assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1.0)


def test_brute_force_transpose():
    v, uv, w, N, cell, mode = _inst(22, 16, 12, uf=1.0)
    M = len(v)
    cols = []
    for k in range(M):                         # real and imaginary unit vectors
        for unit in (1.0, 1j):
            e = np.zeros(M, np.complex64)
            e[k] = unit
            cols.append(imager.dirty_image(e, uv, w, N, cell, mode).ravel())
    A = np.stack(cols, axis=1)                 # (N^2, 2M) real matrix
    y = np.random.default_rng(6).standard_normal(N * N)
    ATy = A.T @ y
    ours = adjoint.adjoint(y.reshape(N, N), uv, w, N, cell, mode)
    packed = np.stack([ours.real, ours.imag], axis=1).ravel()
    # rounding is amplified by 1/corr (about 1e3 at the map edge), hence 1e-10 not 1e-12
    assert np.max(np.abs(packed - ATy)) < 1e-10 * np.max(np.abs(ATy))


def test_predict_approximates_direct_prediction():
    v, uv, w, N, cell, _ = _inst(23, 64, 80)
    # a smooth, compact image so that aliasing is small
    yy, xx = np.mgrid[0:N, 0:N]
    img = np.exp(-((xx - 30) ** 2 + (yy - 35) ** 2) / 20.0)
    keep = imager.Prep(uv, w, N, cell).keep
    D = adjoint.dft_predict(img, uv, keep, N, cell)
    err7 = np.max(np.abs(adjoint.predict(img, uv, w, N, cell) - D)) / np.max(np.abs(D))
    err9 = np.max(np.abs(adjoint.predict(img, uv, w, N, cell, W=9, os=1024) - D)) / np.max(np.abs(D))
    # gridding approximation: small, and it converges as the kernel support/oversampling grow
    assert err7 < 3e-3
    assert err9 < 0.2 * err7
