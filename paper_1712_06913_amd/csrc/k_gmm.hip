// Sky and disk levels of dirty maps: histogram + two-component Gaussian mixture (gfx950).
//
// Sec. 4.1: the dirty map's values are put into 2000 equal ranges and a Gaussian mixture
// is fitted to that histogram; the faintest component's mean is the sky level mu_a (the
// CLEAN stop level of Sec. 4.3 / Algorithm 1) and the next one the disk level mu_b
// (Sec. 4.2).  Choices the paper leaves open: bins span [min, max] of the finite pixel
// values, bin of x = floor((x - lo) / (hi - lo) * B) in FP64 with the last bin closed; two
// components fitted by expectation-maximisation to the bin centres weighted by counts,
// started at the histogram's median and 90th percentile with the histogram's variance and
// equal weights; a fixed iteration count; responsibilities in the log domain; variance
// floor of one bin width squared; a component with zero responsibility keeps its values.
//
// One workgroup per instance: min/max pass, LDS histogram pass, then the EM iterations on
// the B bin counts (FP64, block reductions).  HBM traffic: the map is read twice.
#include <algorithm>

#include "mi_internal.h"

namespace mi {

constexpr int GMM_THREADS = 256;
constexpr int GMM_WAVES = GMM_THREADS / 64;
constexpr int GMM_MAX_BINS = 4096;
constexpr int GMM_BPT = GMM_MAX_BINS / GMM_THREADS;   // bins per thread at most

namespace {

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Sum of NV doubles over the workgroup; every thread gets the totals.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*scratch)[GMM_WAVES]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) scratch[k][wave] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < GMM_WAVES; ++w) t += scratch[k][w];
    v[k] = t;
  }
  __syncthreads();
}

}  // namespace

__global__ void __launch_bounds__(GMM_THREADS)
k_gmm(const InstDesc* __restrict__ inst, const float* __restrict__ images, int n_bins, int n_iter,
      double* __restrict__ levels, float* __restrict__ mu_a_out, float* __restrict__ mu_b_out) {
  __shared__ unsigned hist[GMM_MAX_BINS];
  __shared__ double scratch[4][GMM_WAVES];
  __shared__ float mm[2][GMM_WAVES];
  __shared__ int qbin[2];
  const int i = blockIdx.x;
  const InstDesc d = inst[i];
  const int64_t n = (int64_t)d.N * d.N;
  const float* img = images + d.img_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // pass 1: range of the finite values
  float mn = INFINITY, mx = -INFINITY;
  for (int64_t q = tid; q < n; q += GMM_THREADS) {
    const float v = img[q];
    if (isfinite(v)) {
      mn = fminf(mn, v);
      mx = fmaxf(mx, v);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    mn = fminf(mn, __shfl_xor(mn, o));
    mx = fmaxf(mx, __shfl_xor(mx, o));
  }
  if (lane == 0) { mm[0][wave] = mn; mm[1][wave] = mx; }
  for (int j = tid; j < n_bins; j += GMM_THREADS) hist[j] = 0u;
  __syncthreads();
  mn = mm[0][0];
  mx = mm[1][0];
  for (int w = 1; w < GMM_WAVES; ++w) { mn = fminf(mn, mm[0][w]); mx = fmaxf(mx, mm[1][w]); }
  const bool any = mn <= mx;                          // some finite value
  const double lo = any ? (double)mn : 0.0, hi = any ? (double)mx : 0.0;
  double* L = levels + 6 * (int64_t)i;
  if (!(hi > lo)) {                                   // constant map (or nothing finite: 0)
    if (tid == 0) {
      L[0] = lo; L[1] = 0.0; L[2] = 1.0; L[3] = lo; L[4] = 0.0; L[5] = 0.0;
      if (mu_a_out) mu_a_out[i] = (float)lo;
      if (mu_b_out) mu_b_out[i] = (float)lo;
    }
    return;
  }
  // pass 2: histogram
  const double span = hi - lo, B = (double)n_bins;
  for (int64_t q = tid; q < n; q += GMM_THREADS) {
    const float v = img[q];
    if (!isfinite(v)) continue;
    int j = (int)floor(((double)v - lo) / span * B);
    j = min(j, n_bins - 1);
    atomicAdd(&hist[j], 1u);
  }
  __syncthreads();

  // bin centres and counts owned by this thread
  const double h = span / B;
  double cnt[GMM_BPT], xc[GMM_BPT];
#pragma unroll
  for (int b = 0; b < GMM_BPT; ++b) {
    const int j = tid + b * GMM_THREADS;
    cnt[b] = j < n_bins ? (double)hist[j] : 0.0;
    xc[b] = lo + ((double)j + 0.5) * h;
  }
  // start: median and 90th-percentile bins (integer cumulative counts), histogram moments
  if (tid == 0) {
    int64_t tot = 0;
    for (int j = 0; j < n_bins; ++j) tot += hist[j];
    int64_t c = 0;
    int q5 = -1, q9 = -1;
    for (int j = 0; j < n_bins && q9 < 0; ++j) {
      c += hist[j];
      if (q5 < 0 && 10 * c >= 5 * tot) q5 = j;
      if (q9 < 0 && 10 * c >= 9 * tot) q9 = j;
    }
    qbin[0] = q5;
    qbin[1] = q9;
  }
  double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int b = 0; b < GMM_BPT; ++b) { s[0] += cnt[b]; s[1] += cnt[b] * xc[b]; }
  block_sum<3>(s, scratch);
  const double total = s[0], mean_all = s[1] / total;
  double v1[1] = {0.0};
#pragma unroll
  for (int b = 0; b < GMM_BPT; ++b) v1[0] += cnt[b] * (xc[b] - mean_all) * (xc[b] - mean_all);
  block_sum<1>(v1, scratch);
  const double floor_var = h * h;
  const double var_all = fmax(v1[0] / total, floor_var);
  double mu[2] = {lo + ((double)qbin[0] + 0.5) * h, lo + ((double)qbin[1] + 0.5) * h};
  double var[2] = {var_all, var_all};
  double pi[2] = {0.5, 0.5};
  const double LOG2PI = 1.8378770664093454836;
  for (int t = 0; t < n_iter; ++t) {
    double c0[2];
    for (int k = 0; k < 2; ++k) c0[k] = log(pi[k]) - 0.5 * (LOG2PI + log(var[k]));
    double r0[GMM_BPT], r1[GMM_BPT];
    double a[4] = {0.0, 0.0, 0.0, 0.0};              // n r_0, n r_0 x, n r_1, n r_1 x
#pragma unroll
    for (int b = 0; b < GMM_BPT; ++b) {
      const double d0 = xc[b] - mu[0], d1 = xc[b] - mu[1];
      const double l0 = c0[0] - d0 * d0 / (2.0 * var[0]);
      const double l1 = c0[1] - d1 * d1 / (2.0 * var[1]);
      const double m = fmax(l0, l1);
      const double e0 = exp(l0 - m), e1 = exp(l1 - m);
      const double es = e0 + e1;
      r0[b] = e0 / es;
      r1[b] = e1 / es;
      a[0] += cnt[b] * r0[b];
      a[1] += cnt[b] * r0[b] * xc[b];
      a[2] += cnt[b] * r1[b];
      a[3] += cnt[b] * r1[b] * xc[b];
    }
    block_sum<4>(a, scratch);
    const double nk[2] = {a[0], a[2]};
    const double mk[2] = {nk[0] > 0.0 ? a[1] / nk[0] : mu[0], nk[1] > 0.0 ? a[3] / nk[1] : mu[1]};
    double v[2] = {0.0, 0.0};
#pragma unroll
    for (int b = 0; b < GMM_BPT; ++b) {
      const double d0 = xc[b] - mk[0], d1 = xc[b] - mk[1];
      v[0] += cnt[b] * r0[b] * d0 * d0;
      v[1] += cnt[b] * r1[b] * d1 * d1;
    }
    block_sum<2>(v, scratch);
    for (int k = 0; k < 2; ++k) {
      if (!(nk[k] > 0.0)) continue;
      mu[k] = mk[k];
      var[k] = fmax(v[k] / nk[k], floor_var);
      pi[k] = nk[k] / total;
    }
  }
  if (tid == 0) {
    const int lo_k = mu[1] < mu[0] ? 1 : 0, hi_k = 1 - lo_k;
    L[0] = mu[lo_k]; L[1] = sqrt(var[lo_k]); L[2] = pi[lo_k];
    L[3] = mu[hi_k]; L[4] = sqrt(var[hi_k]); L[5] = pi[hi_k];
    if (mu_a_out) mu_a_out[i] = (float)mu[lo_k];
    if (mu_b_out) mu_b_out[i] = (float)mu[hi_k];
  }
}

hipError_t launch_gmm(const InstDesc* inst, int n_inst, const float* images, int n_bins, int n_iter,
                      double* levels, float* mu_a, float* mu_b, hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gmm, dim3(n_inst), dim3(GMM_THREADS), 0, st, inst, images, n_bins, n_iter, levels, mu_a,
                     mu_b);
  return hipGetLastError();
}

}  // namespace mi
