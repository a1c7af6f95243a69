"""Pins of the FP64 histogram + Gaussian-mixture levels (oracle/gmm.py)."""
import math
from fractions import Fraction

import numpy as np
from scipy.special import erf

from oracle import gmm


def test_histogram_bins_follow_the_exact_definition():
    rng = np.random.default_rng(11)
    x = rng.standard_normal(3000).astype(np.float32)
    counts, lo, hi = gmm.histogram(x, 2000)
    assert counts.sum() == x.size
    # exact rational bin of every value: floor((x - lo) / (hi - lo) * B), last bin closed
    ref = np.zeros(2000, np.int64)
    flo, fhi = Fraction(lo), Fraction(hi)
    for v in x.astype(np.float64):
        j = int((Fraction(float(v)) - flo) / (fhi - flo) * 2000)
        ref[min(j, 1999)] += 1
    assert np.array_equal(counts, ref)
    # and numpy's histogram on the same range agrees
    np_counts, _ = np.histogram(x.astype(np.float64), bins=2000, range=(lo, hi))
    assert np.array_equal(counts, np_counts)


def test_constant_map_goes_to_one_bin():
    counts, lo, hi = gmm.histogram(np.full((8, 8), 0.25, np.float32), 2000)
    assert counts[0] == 64 and counts.sum() == 64 and lo == hi == 0.25


def test_one_component_fit_is_the_weighted_moments():
    rng = np.random.default_rng(12)
    counts = rng.integers(0, 50, 2000)
    lo, hi = -1.5, 2.5
    ((mu, var, pi),) = gmm.em_fit(counts, lo, hi, K=1, n_iter=1)   # one step: exact moments
    x = lo + (np.arange(2000) + 0.5) * (hi - lo) / 2000
    m = np.average(x, weights=counts)
    v = np.average((x - m) ** 2, weights=counts)
    assert abs(mu - m) <= 1e-12 * abs(m) + 1e-15
    assert abs(var - v) <= 1e-12 * v
    assert pi == 1.0


def _mixture_counts(params, lo, hi, n_bins, total):
    edges = lo + (hi - lo) * np.arange(n_bins + 1) / n_bins
    c = np.zeros(n_bins)
    for mu, sd, pi in params:
        cdf = 0.5 * (1.0 + erf((edges - mu) / (sd * math.sqrt(2.0))))
        c += pi * np.diff(cdf)
    return np.round(c * total).astype(np.int64)


def test_em_log_likelihood_never_decreases():
    counts = _mixture_counts([(0.05, 0.03, 0.7), (0.5, 0.1, 0.3)], -0.2, 1.2, 2000, 1e6)
    trace = []
    gmm.em_fit(counts, -0.2, 1.2, K=2, n_iter=60, trace=trace)
    ll = [gmm.log_likelihood(counts, -0.2, 1.2, t) for t in trace]
    for a, b in zip(ll, ll[1:]):
        assert b >= a - 1e-9 * abs(a)


def test_em_recovers_a_known_two_gaussian_mixture():
    truth = [(0.02, 0.015, 0.83), (0.61, 0.06, 0.17)]       # sky-like and disk-like
    counts = _mixture_counts(truth, -0.1, 1.0, 2000, 1e6)
    (ma, va, pa), (mb, vb, pb) = gmm.em_fit(counts, -0.1, 1.0, K=2)
    for (mu, sd, pi), (m, v, p) in zip(truth, [(ma, va, pa), (mb, vb, pb)]):
        assert abs(m - mu) < 1e-4
        assert abs(math.sqrt(v) - sd) < 1e-2 * sd
        assert abs(p - pi) < 1e-3


def test_levels_of_a_disk_map():
    # uniform disk of brightness 1 on a zero sky, plus small noise: sky ~ 0, disk ~ 1
    N = 256
    yy, xx = np.mgrid[0:N, 0:N]
    disk = ((xx - N / 2) ** 2 + (yy - N / 2) ** 2 <= 40 ** 2).astype(np.float64)
    img = (disk + 0.01 * np.random.default_rng(13).standard_normal((N, N))).astype(np.float32)
    ma, sa, pa, mb, sb, pb = gmm.levels(img)
    assert abs(ma) < 2e-3 and abs(mb - 1.0) < 2e-3
    assert abs(pb - disk.mean()) < 2e-3
