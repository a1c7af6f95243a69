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
// the B bin counts (FP64, workgroup sums).  HBM traffic: the map is read twice.
#include <algorithm>

#include "mi_internal.h"

namespace mi {

constexpr int GMM_THREADS = 256;
constexpr int GMM_WAVES = GMM_THREADS / 64;
constexpr int GMM_MAX_BINS = 4096;
constexpr int GMM_UNROLL = 8;        // map loads in flight per thread

namespace {

// A double moved between lanes by a DPP pattern (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over the wave, the same in every lane: within each row of 16 lanes by DPP (lane
// i ^ 1, i ^ 2, then the mirrored lane of the half row and of the row), then the four row
// sums read from lanes 0, 16, 32, 48.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xb1>(v);     // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4e>(v);     // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141>(v);    // row_half_mirror
  v += dpp_f64<0x140>(v);    // row_mirror
  const int lo = __double2loint(v), hi = __double2hiint(v);
  double t = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    t += __hiloint2double(__builtin_amdgcn_readlane(hi, 16 * r), __builtin_amdgcn_readlane(lo, 16 * r));
  return t;
}

// Sum of NV doubles over the workgroup with one barrier: wave sums go to one of two
// scratch buffers (alternating between calls, so a buffer is rewritten only after a later
// barrier has passed); every thread then adds the wave sums in wave order.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*scratch)[6][GMM_WAVES], int& parity) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) scratch[parity][k][wave] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < GMM_WAVES; ++w) t += scratch[parity][k][w];
    v[k] = t;
  }
  parity ^= 1;
}

// 1 / x and 1 / sqrt(x) for positive x: the hardware estimates refined by Newton steps to
// within an ulp or two (the EM's sums carry far more rounding than that); a responsibility
// sum too small for the estimate's range takes the IEEE division
__device__ __forceinline__ double rcp_f64(double x) {
  if (x < 1e-290) return 1.0 / x;
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double rsqrt_f64(double x) {
  double r = __builtin_amdgcn_rsq(x);
  // r <- r (3 - x r^2) / 2, three times from the estimate
  for (int k = 0; k < 3; ++k) r = r * fma(-0.5 * x * r, r, 1.5);
  return r;
}

// 2^(j/64), j = 0..63, correctly rounded
__constant__ double kExp2Tab64[64] = {
    0x1.0000000000000p+0, 0x1.02c9a3e778061p+0, 0x1.059b0d3158574p+0, 0x1.0874518759bc8p+0,
    0x1.0b5586cf9890fp+0, 0x1.0e3ec32d3d1a2p+0, 0x1.11301d0125b51p+0, 0x1.1429aaea92de0p+0,
    0x1.172b83c7d517bp+0, 0x1.1a35beb6fcb75p+0, 0x1.1d4873168b9aap+0, 0x1.2063b88628cd6p+0,
    0x1.2387a6e756238p+0, 0x1.26b4565e27cddp+0, 0x1.29e9df51fdee1p+0, 0x1.2d285a6e4030bp+0,
    0x1.306fe0a31b715p+0, 0x1.33c08b26416ffp+0, 0x1.371a7373aa9cbp+0, 0x1.3a7db34e59ff7p+0,
    0x1.3dea64c123422p+0, 0x1.4160a21f72e2ap+0, 0x1.44e086061892dp+0, 0x1.486a2b5c13cd0p+0,
    0x1.4bfdad5362a27p+0, 0x1.4f9b2769d2ca7p+0, 0x1.5342b569d4f82p+0, 0x1.56f4736b527dap+0,
    0x1.5ab07dd485429p+0, 0x1.5e76f15ad2148p+0, 0x1.6247eb03a5585p+0, 0x1.6623882552225p+0,
    0x1.6a09e667f3bcdp+0, 0x1.6dfb23c651a2fp+0, 0x1.71f75e8ec5f74p+0, 0x1.75feb564267c9p+0,
    0x1.7a11473eb0187p+0, 0x1.7e2f336cf4e62p+0, 0x1.82589994cce13p+0, 0x1.868d99b4492edp+0,
    0x1.8ace5422aa0dbp+0, 0x1.8f1ae99157736p+0, 0x1.93737b0cdc5e5p+0, 0x1.97d829fde4e50p+0,
    0x1.9c49182a3f090p+0, 0x1.a0c667b5de565p+0, 0x1.a5503b23e255dp+0, 0x1.a9e6b5579fdbfp+0,
    0x1.ae89f995ad3adp+0, 0x1.b33a2b84f15fbp+0, 0x1.b7f76f2fb5e47p+0, 0x1.bcc1e904bc1d2p+0,
    0x1.c199bdd85529cp+0, 0x1.c67f12e57d14bp+0, 0x1.cb720dcef9069p+0, 0x1.d072d4a07897cp+0,
    0x1.d5818dcfba487p+0, 0x1.da9e603db3285p+0, 0x1.dfc97337b9b5fp+0, 0x1.e502ee78b3ff6p+0,
    0x1.ea4afa2a490dap+0, 0x1.efa1bee615a27p+0, 0x1.f50765b6e4540p+0, 0x1.fa7c1819e90d8p+0};

// exp(t) for the E step (t <= 0, finite) by Tang's table-driven method (ACM TOMS 15, 1989):
// t = (64 m + j) ln2 / 64 + r with |r| <= ln2 / 128, exp(t) = 2^m 2^(j/64) exp(r), exp(r) - 1
// from its Taylor polynomial to degree 5 (truncation below 4e-17 at |r| <= ln2 / 128), the
// reduction with ln2 / 64 split in two parts.  Within a few ulp of exp(t), ten FP64
// operations and one LDS read instead of the library's longer sequence; very negative t
// gives 0 through ldexp.
__device__ __forceinline__ double exp_tang(double t, const double* __restrict__ tab64) {
  const double INV = 0x1.71547652b82fep+6;            // 64 / ln2
  const double L_HI = 0x1.62e42fefa39efp-7, L_LO = 0x1.abc9e3b39803fp-62;   // ln2 / 64
  const double k = rint(t * INV);
  const int n = (int)k;
  const double r = fma(-k, L_LO, fma(-k, L_HI, t));
  double c = fma(r, 1.0 / 120.0, 1.0 / 24.0);
  c = fma(r, c, 1.0 / 6.0);
  c = fma(r, c, 0.5);
  const double p = fma(r * r, c, r);                  // exp(r) - 1
  const double tj = tab64[n & 63];
  return ldexp(fma(tj, p, tj), n >> 6);
}

}  // namespace

// One workgroup of 256 threads per map, BPT bins per thread (8 for up to 2048 bins, so
// that three workgroups share a compute unit and all maps of a 520-map batch are resident
// at once).  Each wave owns 64 BPT consecutive bins (bin of lane l, slot b: wave 64 BPT +
// 64 b + l).  A wave whose bins are all empty (the bright tail of a dirty map's histogram)
// skips the E step; the others run it without branches, so that a thread's BPT
// exponentials overlap (an empty bin adds exact zeros: its count multiplies every term).
// The E step needs one exponential per bin (the larger of the two log terms gives
// exp(0) = 1 exactly), and an iteration's sums take one workgroup reduction, i.e. one
// barrier.
template <int GMM_BPT>
__global__ void __launch_bounds__(GMM_THREADS)
k_gmm(const InstDesc* __restrict__ inst, const float* __restrict__ images, int n_bins, int n_iter,
      double* __restrict__ levels, float* __restrict__ mu_a_out, float* __restrict__ mu_b_out) {
  __shared__ unsigned hist[GMM_MAX_BINS];
  __shared__ double scratch[2][6][GMM_WAVES];
  __shared__ float mm[2][GMM_WAVES];
  __shared__ int qbin[2];
  __shared__ double tab64[64];
  if (threadIdx.x < 64) tab64[threadIdx.x] = kExp2Tab64[threadIdx.x];   // read after the histogram barriers
  const int i = blockIdx.x;
  const InstDesc d = inst[i];
  const int64_t n = (int64_t)d.N * d.N;
  const float* img = images + d.img_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int parity = 0;

  // pass 1: range of the finite values (16-byte loads; N^2 is a multiple of 4), GMM_UNROLL
  // loads in flight per thread (one map per workgroup leaves few waves to hide latency);
  // a position past the map loads element 0 and is ignored where the values are used
  float mn = INFINITY, mx = -INFINITY;
  const float4* img4 = reinterpret_cast<const float4*>(img);
  const int64_t n4 = n / 4;
  for (int64_t q0 = tid; q0 < n4; q0 += GMM_UNROLL * GMM_THREADS) {
    float4 v4[GMM_UNROLL];
#pragma unroll
    for (int u = 0; u < GMM_UNROLL; ++u) {
      const int64_t q = q0 + u * GMM_THREADS;
      v4[u] = img4[q < n4 ? q : 0];
    }
#pragma unroll
    for (int u = 0; u < GMM_UNROLL; ++u) {
      const bool in = q0 + u * GMM_THREADS < n4;
      const float v[4] = {v4[u].x, v4[u].y, v4[u].z, v4[u].w};
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (in && isfinite(v[j])) {
          mn = fminf(mn, v[j]);
          mx = fmaxf(mx, v[j]);
        }
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
  for (int64_t q0 = tid; q0 < n4; q0 += GMM_UNROLL * GMM_THREADS) {
    float4 v4[GMM_UNROLL];
#pragma unroll
    for (int u = 0; u < GMM_UNROLL; ++u) {
      const int64_t q = q0 + u * GMM_THREADS;
      v4[u] = img4[q < n4 ? q : 0];
    }
#pragma unroll
    for (int u = 0; u < GMM_UNROLL; ++u) {
      const bool in = q0 + u * GMM_THREADS < n4;
      const float v[4] = {v4[u].x, v4[u].y, v4[u].z, v4[u].w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (!in || !isfinite(v[j])) continue;
        int b = (int)floor(((double)v[j] - lo) / span * B);
        b = min(b, n_bins - 1);
        atomicAdd(&hist[b], 1u);
      }
    }
  }
  __syncthreads();

  // bin centres and counts owned by this thread (bins past n_bins count zero)
  const double h = span / B;
  double cnt[GMM_BPT], xc[GMM_BPT];
  bool mine = false;
#pragma unroll
  for (int b = 0; b < GMM_BPT; ++b) {
    const int j = wave * 64 * GMM_BPT + b * 64 + lane;
    cnt[b] = j < n_bins ? (double)hist[j] : 0.0;
    xc[b] = lo + ((double)j + 0.5) * h;
    mine |= cnt[b] > 0.0;
  }
  const bool wave_busy = __any(mine);                 // uniform over the wave
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
  double s[2] = {0.0, 0.0};
#pragma unroll
  for (int b = 0; b < GMM_BPT; ++b) { s[0] += cnt[b]; s[1] += cnt[b] * xc[b]; }
  block_sum<2>(s, scratch, parity);
  const double total = s[0], mean_all = s[1] / total;
  double v1[1] = {0.0};
#pragma unroll
  for (int b = 0; b < GMM_BPT; ++b) v1[0] += cnt[b] * (xc[b] - mean_all) * (xc[b] - mean_all);
  block_sum<1>(v1, scratch, parity);
  const double floor_var = h * h;
  const double var_all = fmax(v1[0] / total, floor_var);
  double mu[2] = {lo + ((double)qbin[0] + 0.5) * h, lo + ((double)qbin[1] + 0.5) * h};
  double var[2] = {var_all, var_all};
  double pi[2] = {0.5, 0.5};
  const double LOG2PI = 1.8378770664093454836;
  // The M step's sums in one workgroup reduction: per component n r, n r x', n r x'^2 with
  // x' = x - xm (xm = the range's centre, so |x'| <= span / 2), and the variance about the
  // new mean as sum n r x'^2 / nk - m'^2 (equal to sum n r (x - mk)^2 / nk; the shift keeps
  // the cancellation small: a relative error of about 1e-16 (span / 2)^2 / var)
  const double xm = lo + 0.5 * span;
  double xs[GMM_BPT];
#pragma unroll
  for (int b = 0; b < GMM_BPT; ++b) xs[b] = xc[b] - xm;
  const double inv_total = 1.0 / total;
  for (int t = 0; t < n_iter; ++t) {
    // log(pi / sqrt(2 pi var)) and 1 / (2 var): one logarithm and one reciprocal square
    // root per component (each iteration's serial part is short)
    double c0[2], iv[2];
    for (int k = 0; k < 2; ++k) {
      const double rs = rsqrt_f64(var[k]);
      c0[k] = log(pi[k] * rs) - 0.5 * LOG2PI;
      iv[k] = 0.5 * rs * rs;
    }
    double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (wave_busy) {
#pragma unroll
      for (int b = 0; b < GMM_BPT; ++b) {
        const double d0 = xc[b] - mu[0], d1 = xc[b] - mu[1];
        const double l0 = c0[0] - d0 * d0 * iv[0];
        const double l1 = c0[1] - d1 * d1 * iv[1];
        const double e = exp_tang(fmin(l0, l1) - fmax(l0, l1), tab64);   // the other term is exp(0) = 1
        // 1 / (1 + e) from the hardware reciprocal and two Newton steps (1 + e is in [1, 2])
        const double den = 1.0 + e;
        double inv = __builtin_amdgcn_rcp(den);
        inv = fma(inv, fma(-den, inv, 1.0), inv);
        inv = fma(inv, fma(-den, inv, 1.0), inv);
        const double w0 = cnt[b] * (l0 >= l1 ? inv : e * inv);
        const double w1 = cnt[b] * (l0 >= l1 ? e * inv : inv);
        a[0] += w0;
        a[1] += w0 * xs[b];
        a[2] += w0 * xs[b] * xs[b];
        a[3] += w1;
        a[4] += w1 * xs[b];
        a[5] += w1 * xs[b] * xs[b];
      }
    }
    block_sum<6>(a, scratch, parity);
    for (int k = 0; k < 2; ++k) {
      const double nk = a[3 * k];
      if (!(nk > 0.0)) continue;            // no responsibility: the component keeps its values
      const double inv_nk = rcp_f64(nk);
      const double m = a[3 * k + 1] * inv_nk;
      mu[k] = xm + m;
      var[k] = fmax(a[3 * k + 2] * inv_nk - m * m, floor_var);
      pi[k] = nk * inv_total;
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
  if (n_bins <= 8 * GMM_THREADS)
    hipLaunchKernelGGL(k_gmm<8>, dim3(n_inst), dim3(GMM_THREADS), 0, st, inst, images, n_bins, n_iter, levels, mu_a,
                       mu_b);
  else
    hipLaunchKernelGGL(k_gmm<GMM_MAX_BINS / GMM_THREADS>, dim3(n_inst), dim3(GMM_THREADS), 0, st, inst, images, n_bins,
                       n_iter, levels, mu_a, mu_b);
  return hipGetLastError();
}

}  // namespace mi
