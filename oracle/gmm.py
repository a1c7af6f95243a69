"""FP64 sky and disk levels by a Gaussian mixture fitted to the dirty-image histogram
(oracle; test infrastructure).

Sec. 4.1 (detection of solar disk and sky brightness): the dirty map holds sky background,
solar disk and possibly active regions, whose brightness levels differ; the map's values
are put into 2000 equal ranges and a Gaussian mixture is fitted to that histogram.  The
mean of the faintest component is the sky level mu_a, the CLEAN stop level of Sec. 4.3
and Algorithm 1 (`improved_clean` loops while the peak exceeds mu_a); the next one is the
disk level mu_b, which Sec. 4.2 cleans down to before disk centering.

The paper fixes the 2000 ranges and the use of a Gaussian mixture, and names two curves.
The rest is a reading (listed with the others in the design notes):
  * bins: lo = min, hi = max of the map's finite values (FP64 of the float32 values;
    non-finite pixels are not counted); bin of x is floor((x - lo) / (hi - lo) * B), the
    last bin closed (x = hi goes to B - 1); a constant map puts everything in bin 0;
  * the mixture has K = 2 components, fitted by expectation-maximisation to the bin
    centres x_j = lo + (j + 1/2) h (h = (hi - lo) / B) weighted by their counts n_j;
  * start: means at the histogram's median and 90th percentile (the first bin whose
    cumulative count reaches 1/2 resp. 9/10 of the total), both variances equal to the
    histogram's variance, equal weights;
  * a fixed number of iterations (500); responsibilities in the log domain; a variance
    floor of h^2 (one bin); a component whose responsibility sum is zero keeps its
    previous parameters;
  * components sorted by mean: (a) faintest, (b) the other.

Pins (tests/test_oracle_gmm.py): the histogram equals numpy.histogram on the same edges;
with one component the fit is the closed-form weighted mean and variance; the
log-likelihood never decreases from one iteration to the next; a histogram built from the
exact bin integrals of a known two-Gaussian mixture gives back its parameters.
"""
from __future__ import annotations

import math

import numpy as np

N_BINS = 2000
N_ITER = 500


def histogram(img, n_bins: int = N_BINS):
    """(counts int64[n_bins], lo, hi) of a map, bins as in the module header."""
    x = np.asarray(img, dtype=np.float64).ravel()
    x = x[np.isfinite(x)]                    # non-finite pixels are not counted
    counts = np.zeros(n_bins, dtype=np.int64)
    if x.size == 0:
        return counts, 0.0, 0.0
    lo, hi = float(np.min(x)), float(np.max(x))
    if not hi > lo:
        counts[0] = x.size
        return counts, lo, hi
    idx = np.floor((x - lo) / (hi - lo) * n_bins).astype(np.int64)
    idx = np.minimum(idx, n_bins - 1)
    np.add.at(counts, idx, 1)
    return counts, lo, hi


def _quantile_bin(counts, p):
    """First bin whose cumulative count reaches p of the total (integer arithmetic)."""
    c = np.cumsum(counts)
    total = int(c[-1])
    # cumulative >= p * total, decided without rounding: 10 * c >= (10 p) * total
    num = int(round(p * 10))
    return int(np.argmax(10 * c >= num * total))


def log_likelihood(counts, lo, hi, params):
    """sum_j n_j log sum_k pi_k N(x_j; mu_k, sigma_k^2) over the bin centres."""
    n_bins = len(counts)
    h = (hi - lo) / n_bins
    x = lo + (np.arange(n_bins) + 0.5) * h
    ll = np.zeros(n_bins)
    comp = []
    for mu, var, pi in params:
        comp.append(math.log(pi) - 0.5 * math.log(2.0 * math.pi * var) - (x - mu) ** 2 / (2.0 * var))
    comp = np.array(comp)
    m = np.max(comp, axis=0)
    ll = m + np.log(np.sum(np.exp(comp - m), axis=0))
    return float(np.sum(counts * ll))


def em_fit(counts, lo, hi, K: int = 2, n_iter: int = N_ITER, trace=None):
    """EM fit of a K-component Gaussian mixture to a histogram.

    Returns a list of (mu, var, pi) sorted by mu.  `trace`, if a list, receives the
    parameters after every iteration (for the monotonicity pin)."""
    counts = np.asarray(counts, dtype=np.float64)
    n_bins = len(counts)
    total = float(np.sum(counts))
    if not hi > lo:                          # constant map: one point mass
        return [(lo, 0.0, 1.0)] + [(lo, 0.0, 0.0)] * (K - 1)
    h = (hi - lo) / n_bins
    x = lo + (np.arange(n_bins) + 0.5) * h
    floor_var = h * h
    # start
    mean_all = float(np.sum(counts * x)) / total
    var_all = max(float(np.sum(counts * (x - mean_all) ** 2)) / total, floor_var)
    if K == 1:
        qs = [0.5]
    else:
        qs = [0.5 + 0.4 * k / (K - 1) for k in range(K)]       # K = 2: 0.5 and 0.9
    mu = np.array([x[_quantile_bin(counts, q)] for q in qs])
    var = np.full(K, var_all)
    pi = np.full(K, 1.0 / K)
    for _ in range(n_iter):
        # E step (log domain)
        lg = np.empty((K, n_bins))
        for k in range(K):
            lg[k] = math.log(pi[k]) - 0.5 * math.log(2.0 * math.pi * var[k]) - (x - mu[k]) ** 2 / (2.0 * var[k])
        m = np.max(lg, axis=0)
        e = np.exp(lg - m)
        r = e / np.sum(e, axis=0)
        # M step
        for k in range(K):
            nk = float(np.sum(counts * r[k]))
            if not nk > 0.0:
                continue
            mk = float(np.sum(counts * r[k] * x)) / nk
            vk = float(np.sum(counts * r[k] * (x - mk) ** 2)) / nk
            mu[k] = mk
            var[k] = max(vk, floor_var)
            pi[k] = nk / total
        if trace is not None:
            trace.append([(float(mu[k]), float(var[k]), float(pi[k])) for k in range(K)])
    order = np.argsort(mu, kind="stable")
    return [(float(mu[k]), float(var[k]), float(pi[k])) for k in order]


def levels(img, n_bins: int = N_BINS, n_iter: int = N_ITER):
    """(mu_a, sigma_a, pi_a, mu_b, sigma_b, pi_b): sky level (a) and disk level (b)."""
    counts, lo, hi = histogram(img, n_bins)
    (ma, va, pa), (mb, vb, pb) = em_fit(counts, lo, hi, K=2, n_iter=n_iter)
    return (ma, math.sqrt(va), pa, mb, math.sqrt(vb), pb)
