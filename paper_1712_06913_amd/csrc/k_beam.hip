// Beam-side kernels of the CLEAN stage (gfx950): the clean-beam fit and the check of the
// beam's point symmetry before CLEAN.
#include <algorithm>

#include "mi_internal.h"

namespace mi {

constexpr int FIT_THREADS = 1024;
constexpr int FIT_WAVES = FIT_THREADS / 64;
constexpr int FIT_HALF = 63;                 // fit box half-width (pixels)
constexpr int FIT_BOX = 2 * FIT_HALF + 1;
constexpr int RESTORE_RMAX = 64;             // restore radius cap (pixels)

// The beam of Hermitian-completed visibilities is point-symmetric about (N, N):
// B[N + a][N + b] = B[N - a][N - b] (the library's own beams are stored exactly so).
// k_beam_symcheck flags instances whose beam is not exactly symmetric over the rows and
// columns 1..2N-1 that CLEAN windows read: per instance, the mirror pixels (r, c) with
// r > N, or r = N and c > N, and 1 <= c <= 2N-1.
__global__ void __launch_bounds__(256)
k_beam_symcheck(const InstDesc* __restrict__ inst, const float* __restrict__ beam, int* __restrict__ asym) {
  const InstDesc d = inst[blockIdx.y];
  const int N = d.N, twoN = 2 * N;
  const unsigned* B = reinterpret_cast<const unsigned*>(beam + d.beam_off);
  const int64_t npair = (int64_t)N * twoN;
  bool bad = false;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < npair; q += (int64_t)gridDim.x * 256) {
    const int r = N + (int)(q / twoN), c = (int)(q % twoN);
    if (c == 0 || (r == N && c <= N)) continue;
    bad |= B[(int64_t)r * twoN + c] != B[(int64_t)(twoN - r) * twoN + (twoN - c)];
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&asym[blockIdx.y], 1);
}

// Clean-beam fit: one workgroup per instance.
__global__ void __launch_bounds__(FIT_THREADS)
k_beamfit(const InstDesc* __restrict__ inst, const float* __restrict__ beam, double* __restrict__ cbeam,
          int* __restrict__ rrad, int* __restrict__ status) {
  __shared__ unsigned char lab[FIT_BOX * FIT_BOX];
  __shared__ int changed;
  __shared__ double red[8][FIT_WAVES];
  __shared__ int cnt[3][FIT_WAVES];
  const int i = blockIdx.x;
  const InstDesc d = inst[i];
  const int N = d.N, twoN = 2 * N;
  const int hb = min(N - 1, FIT_HALF), side = 2 * hb + 1;
  const float* B = beam + d.beam_off;
  const float thr = 0.35f;
  auto bval = [&](int q) -> float {
    const int dy = q / side - hb, dx = q % side - hb;
    return B[(int64_t)(N + dy) * twoN + (N + dx)];
  };
  for (int q = threadIdx.x; q < side * side; q += FIT_THREADS) lab[q] = 0;
  __syncthreads();
  if (threadIdx.x == 0) lab[hb * side + hb] = bval(hb * side + hb) > thr ? 1 : 0;
  __syncthreads();
  for (;;) {
    if (threadIdx.x == 0) changed = 0;
    __syncthreads();
    for (int q = threadIdx.x; q < side * side; q += FIT_THREADS) {
      if (lab[q]) continue;
      const int r = q / side, c = q % side;
      const bool nb = (r > 0 && lab[q - side]) || (r < side - 1 && lab[q + side]) ||
                      (c > 0 && lab[q - 1]) || (c < side - 1 && lab[q + 1]);
      if (nb && bval(q) > thr) { lab[q] = 1; changed = 1; }
    }
    __syncthreads();
    const int ch = changed;
    __syncthreads();
    if (!ch) break;
  }
  // least squares: minimise sum (a dx^2 + b dx dy + c dy^2 + ln beam)^2 over the lobe.
  // Degenerate lobes are decided by integer pixel counts: no pixel with dx dy != 0 -> b = 0
  // and a 2-term fit (needs pixels on both axes); otherwise a one-pixel-FWHM default.
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int clipped = 0, n_xy = 0, n_x = 0, n_y = 0;
  for (int q = threadIdx.x; q < side * side; q += FIT_THREADS) {
    if (!lab[q]) continue;
    const int r = q / side, c = q % side;
    if (r == 0 || c == 0 || r == side - 1 || c == side - 1) clipped = 1;
    const int ix = c - hb, iy = r - hb;
    n_xy += (ix != 0 && iy != 0);
    n_x += (ix != 0);
    n_y += (iy != 0);
    const double dx = ix, dy = iy;
    const double t = -log((double)bval(q));
    const double x2 = dx * dx, xy = dx * dy, y2 = dy * dy;
    s[0] += x2 * x2; s[1] += x2 * xy; s[2] += x2 * y2; s[3] += xy * y2; s[4] += y2 * y2;
    s[5] += x2 * t;  s[6] += xy * t;  s[7] += y2 * t;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    double v = s[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[k][wave] = v;
  }
  for (int o = 32; o > 0; o >>= 1) {
    n_xy += __shfl_xor(n_xy, o);
    n_x += __shfl_xor(n_x, o);
    n_y += __shfl_xor(n_y, o);
  }
  if (lane == 0) { cnt[0][wave] = n_xy; cnt[1][wave] = n_x; cnt[2][wave] = n_y; }
  if (clipped && status) atomicOr(&status[i], 2);
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[8];
    int nxy = 0, nx = 0, ny = 0;
    for (int k = 0; k < 8; ++k) {
      t[k] = 0.0;
      for (int w = 0; w < FIT_WAVES; ++w) t[k] += red[k][w];
    }
    for (int w = 0; w < FIT_WAVES; ++w) { nxy += cnt[0][w]; nx += cnt[1][w]; ny += cnt[2][w]; }
    // normal matrix [[x4, x3y, x2y2], [x3y, x2y2, xy3], [x2y2, xy3, y4]]
    const double m00 = t[0], m01 = t[1], m02 = t[2], m11 = t[2], m12 = t[3], m22 = t[4];
    const double r0 = t[5], r1 = t[6], r2 = t[7];
    const double ln2 = 0.69314718055994530942;
    double a = 4.0 * ln2, b = 0.0, c = 4.0 * ln2;
    bool degenerate = true;
    if (nxy > 0) {
      const double det = m00 * (m11 * m22 - m12 * m12) - m01 * (m01 * m22 - m12 * m02) + m02 * (m01 * m12 - m11 * m02);
      if (fabs(det) >= 1e-9 * fabs(m00 * m11 * m22)) {
        a = (r0 * (m11 * m22 - m12 * m12) - m01 * (r1 * m22 - m12 * r2) + m02 * (r1 * m12 - m11 * r2)) / det;
        b = (m00 * (r1 * m22 - m12 * r2) - r0 * (m01 * m22 - m12 * m02) + m02 * (m01 * r2 - r1 * m02)) / det;
        c = (m00 * (m11 * r2 - r1 * m12) - m01 * (m01 * r2 - r1 * m02) + r0 * (m01 * m12 - m11 * m02)) / det;
        degenerate = false;
      }
    } else if (nx > 0 && ny > 0) {
      // b = 0: [[x4, x2y2], [x2y2, y4]] (a, c) = (x2 t, y2 t)
      const double det2 = m00 * m22 - m02 * m02;
      a = (r0 * m22 - m02 * r2) / det2;
      c = (m00 * r2 - m02 * r0) / det2;
      degenerate = false;
    }
    if (degenerate && status) atomicOr(&status[i], 2);
    const double mean = 0.5 * (a + c), dev = sqrt(0.25 * (a - c) * (a - c) + 0.25 * b * b);
    const double lmin = mean - dev, lmax = mean + dev;
    double pa = 0.5 * atan2(-b, c - a);
    if (pa < 0) pa += 3.14159265358979323846;
    if (pa >= 3.14159265358979323846) pa -= 3.14159265358979323846;
    double* cb = cbeam + 6 * i;
    cb[0] = a; cb[1] = b; cb[2] = c;
    cb[3] = lmin > 0 ? 2.0 * sqrt(ln2 / lmin) : 0.0;
    cb[4] = lmax > 0 ? 2.0 * sqrt(ln2 / lmax) : 0.0;
    cb[5] = pa;
    int rr = RESTORE_RMAX;
    if (lmin > 0) {
      const double rneed = ceil(sqrt(27.631021115928547 / lmin));   // exp(-27.63) = 1e-12
      if (rneed <= RESTORE_RMAX) rr = (int)rneed;
      else if (status) atomicOr(&status[i], 4);
    } else if (status) {
      atomicOr(&status[i], 4);
    }
    rrad[i] = rr;
  }
}

// Clean-beam fit: one workgroup per instance.
hipError_t launch_beamfit(const InstDesc* inst, int n_inst, const float* beam, double* cbeam, int* rrad,
                          int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_beamfit, dim3(n_inst), dim3(FIT_THREADS), 0, st, inst, beam, cbeam, rrad, status);
  return hipGetLastError();
}

static int sym_blocks(int max_N) { return std::max(1, std::min(256, max_N * max_N / 4096)); }

hipError_t launch_beam_symcheck(const InstDesc* inst, int n_inst, int max_N, const float* beam, int* asym,
                                hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_beam_symcheck, dim3(sym_blocks(max_N), n_inst), dim3(256), 0, st, inst, beam, asym);
  return hipGetLastError();
}

}  // namespace mi
