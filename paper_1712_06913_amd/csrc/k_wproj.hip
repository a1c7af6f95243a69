// w-projection gridding (gfx950): Sec. 3.2.2 and 6.1.  When the phase pi (l^2 + m^2) w
// over the field is not small, each visibility is gridded with a kernel that also carries
// the w-term: the field's Fourier transform of corr(l) corr(m) exp(+2 pi i w (n - 1)),
// n = sqrt(1 - l^2 - m^2), for the w-plane nearest to |w| (conjugated for w < 0).  The
// transform, grid correction and normalisation that follow are those of the 2-D path.
//
// Tables (built once per plan): plane p of support S_p cells is sampled at WP_OS points per
// cell, K_p(t / WP_OS, s / WP_OS) for t, s = -S_p WP_OS / 2 .. S_p WP_OS / 2, row-major
// [dv][du].  The field is sampled at WP_M - 1 symmetric points a = -(WP_M/2 - 1) ..
// WP_M/2 - 1 (pixel a N / WP_M), so the tables are exactly even and K_{-w} = conj(K_w).
// The 2-D DFT is separable: K = E screen E^T with E[t][a] = exp(-2 pi i t a / (WP_OS WP_M)) / WP_M.
//
// Gridding: one wavefront per visibility; its lanes take the S x S taps of the sample and
// of its Hermitian mirror, interpolate the table bilinearly at (d - f) WP_OS, and add into
// the FP64 half grid with hardware FP64 atomics.  Taps outside the half plane u <= 0 or
// with |cell| >= N/2 are dropped (the mirror of a dropped tap is dropped too).
#include <algorithm>

#include "mi_wproj.h"

namespace mi {

namespace {

constexpr int WP_NA = WP_M - 1;          // field points per axis

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

}  // namespace

// screen_p[b][a] = corr(a) corr(b) exp(+2 pi i w_p (n(a, b) - 1)) for every plane p.
__global__ void __launch_bounds__(256)
k_wscreen(const WPlane* __restrict__ planes, int n_planes, Tables T, double2* __restrict__ screen) {
  const int p = blockIdx.y;
  if (p >= n_planes) return;
  const WPlane pl = planes[p];
  const double* ic = T.inv_corr + (pl.N - 64);
  const int step = pl.N / WP_M;
  for (int q = threadIdx.x + blockIdx.x * blockDim.x; q < WP_NA * WP_NA; q += gridDim.x * blockDim.x) {
    const int ia = q % WP_NA, ib = q / WP_NA;
    const int a = ia - (WP_M / 2 - 1), b = ib - (WP_M / 2 - 1);
    const double l = (double)(a * step) * pl.cell, m = (double)(b * step) * pl.cell;
    const double amp = (1.0 / ic[a * step + pl.N / 2]) * (1.0 / ic[b * step + pl.N / 2]);
    const double ph = 2.0 * pl.w * (sqrt(1.0 - l * l - m * m) - 1.0);   // in units of pi
    double s, c;
    sincospi(ph, &s, &c);
    screen[(int64_t)p * WP_NA * WP_NA + q] = make_double2(amp * c, amp * s);
  }
}

// E[t + half_max][a] = exp(-2 pi i t a / (WP_OS WP_M)) / WP_M for t = -half_max .. half_max.
__global__ void __launch_bounds__(256) k_wdft(int half_max, double2* __restrict__ E) {
  constexpr int PER = WP_OS * WP_M;
  const int n = (2 * half_max + 1) * WP_NA;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const int t = q / WP_NA - half_max, a = q % WP_NA - (WP_M / 2 - 1);
    const int r = ((t * a) % PER + PER) % PER;       // exact integer reduction of the phase
    double s, c;
    sincospi(-2.0 * (double)r / PER, &s, &c);
    E[q] = make_double2(c / WP_M, s / WP_M);
  }
}

// K_p[dv][du] for one (plane, dv row) per workgroup: row1[a] = sum_b E[dv][b] screen[b][a],
// then K[dv][du] = sum_a row1[a] E[du][a].
__global__ void __launch_bounds__(256)
k_wkernel(const WPlane* __restrict__ planes, const int2* __restrict__ rows, const double2* __restrict__ screen,
          const double2* __restrict__ E, int half_max, double2* __restrict__ tabs) {
  __shared__ double2 row1[WP_NA];
  const int2 pr = rows[blockIdx.x];                  // (plane, dv index)
  const WPlane pl = planes[pr.x];
  const int nd = pl.S * WP_OS + 1, half = pl.S * WP_OS / 2;
  const double2* e_dv = E + (int64_t)(pr.y - half + half_max) * WP_NA;
  const double2* scr = screen + (int64_t)pr.x * WP_NA * WP_NA;
  for (int a = threadIdx.x; a < WP_NA; a += blockDim.x) {
    double2 acc = make_double2(0.0, 0.0);
    for (int b = 0; b < WP_NA; ++b) {
      const double2 t = cmul(e_dv[b], scr[b * WP_NA + a]);
      acc.x += t.x;
      acc.y += t.y;
    }
    row1[a] = acc;
  }
  __syncthreads();
  double2* out = tabs + pl.off + (int64_t)pr.y * nd;
  for (int iu = threadIdx.x; iu < nd; iu += blockDim.x) {
    const double2* e_du = E + (int64_t)(iu - half + half_max) * WP_NA;
    double2 acc = make_double2(0.0, 0.0);
    for (int a = 0; a < WP_NA; ++a) {
      const double2 t = cmul(row1[a], e_du[a]);
      acc.x += t.x;
      acc.y += t.y;
    }
    out[iu] = acc;
  }
}

// One wavefront per visibility of instance blockIdx.y (grid-stride over its visibilities).
__global__ void __launch_bounds__(256)
k_grid_w(const InstDesc* __restrict__ inst, const float2* __restrict__ vis, const float2* __restrict__ uv,
         const float* __restrict__ wl, const float* __restrict__ w_in, const float* __restrict__ wts,
         const WInst* __restrict__ winst, const WPlane* __restrict__ planes, const double2* __restrict__ tabs,
         double2* __restrict__ grid) {
  const InstDesc d = inst[blockIdx.y];
  const WInst wi = winst[blockIdx.y];
  const int N = d.N, h = N / 2;
  const int lane = threadIdx.x & 63;
  const int nwave = gridDim.x * (blockDim.x >> 6);
  double2* G = grid + d.gd_off;
  for (int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); k < d.n_vis; k += nwave) {
    const int64_t vi = d.vis_off + k;
    const float2 q = uv[vi];
    const Sample sm = prep_sample(q.x, q.y, w_in[vi], d.scale, N);
    if (!sm.keep) continue;                          // uniform per wave
    const double gu = (double)q.x * d.scale, gv = (double)q.y * d.scale;
    const double fu = gu - (double)sm.cu, fv = gv - (double)sm.cv;
    const double wt = (double)wts[vi];
    const float2 v = vis[vi];
    const double wr = wt * (double)v.x, wim = wt * (double)v.y;
    const double ww = (double)wl[vi];
    int j = (int)floor(fabs(ww) / wi.dw + 0.5);
    j = min(j, wi.n_planes - 1);
    const WPlane pl = planes[wi.plane0 + j];
    const int S = pl.S, H = (S - 1) / 2, nd = S * WP_OS + 1, half = S * WP_OS / 2;
    const double2* tab = tabs + pl.off;
    for (int t = lane; t < 2 * S * S; t += 64) {
      const int m = t >= S * S;                       // 0: the sample, 1: its mirror
      const int tt = t - m * S * S;
      const int du = tt % S - H, dv = tt / S - H;
      const int cu = (m ? -sm.cu : sm.cu) + du, cv = (m ? -sm.cv : sm.cv) + dv;
      if (cu > 0 || cu <= -h || cv >= h || cv <= -h) continue;
      const double x = ((double)du - (m ? -fu : fu)) * WP_OS, y = ((double)dv - (m ? -fv : fv)) * WP_OS;
      const int x0 = min((int)floor(x), half - 1), y0 = min((int)floor(y), half - 1);
      const double ax = x - x0, ay = y - y0;
      const double2* t0 = tab + (int64_t)(y0 + half) * nd + (x0 + half);
      const double2 k00 = t0[0], k01 = t0[1], k10 = t0[nd], k11 = t0[nd + 1];
      double kr = (1 - ay) * ((1 - ax) * k00.x + ax * k01.x) + ay * ((1 - ax) * k10.x + ax * k11.x);
      double ki = (1 - ay) * ((1 - ax) * k00.y + ax * k01.y) + ay * ((1 - ax) * k10.y + ax * k11.y);
      if ((m ? -ww : ww) < 0.0) ki = -ki;             // K_{-w} = conj(K_w)
      const double vr = wr, vim = m ? -wim : wim;
      double gr = vr * kr - vim * ki, gi = vr * ki + vim * kr;
      const int kp = cu + h - 1, jj = cv + h;
      if (((kp + 1) + jj) & 1) { gr = -gr; gi = -gi; }
      double* cell = reinterpret_cast<double*>(G + (int64_t)kp * N + jj);
      unsafeAtomicAdd(cell, gr);
      unsafeAtomicAdd(cell + 1, gi);
    }
  }
}

hipError_t launch_wtables(const WPlane* planes, int n_planes, const int2* rows, int n_rows, int half_max,
                          const Tables& T, double2* screen, double2* E, double2* tabs, hipStream_t st) {
  if (n_planes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_wdft, dim3(64), dim3(256), 0, st, half_max, E);
  hipLaunchKernelGGL(k_wscreen, dim3(4, n_planes), dim3(256), 0, st, planes, n_planes, T, screen);
  hipLaunchKernelGGL(k_wkernel, dim3(n_rows), dim3(256), 0, st, planes, rows, screen, E, half_max, tabs);
  return hipGetLastError();
}

hipError_t launch_grid_w(const InstDesc* inst, int n_inst, int max_nvis, const float2* vis, const float2* uv,
                         const float* wl, const float* w_in, const float* wts, const WInst* winst,
                         const WPlane* planes, const double2* tabs, double2* grid, hipStream_t st) {
  if (n_inst <= 0 || max_nvis <= 0) return hipSuccess;
  const int bx = std::min(64, (max_nvis + 3) / 4);
  hipLaunchKernelGGL(k_grid_w, dim3(bx, n_inst), dim3(256), 0, st, inst, vis, uv, wl, w_in, wts, winst, planes,
                     tabs, grid);
  return hipGetLastError();
}

}  // namespace mi
