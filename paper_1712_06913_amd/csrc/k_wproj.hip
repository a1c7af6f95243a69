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
// Gridding, in the tiled form of the 2-D gridder: k_bin_w sorts each (sample, tile) pair of
// the dirty half grid's 16 x 64 tiles into per-tile lists (a sample's support is that of
// its plane, up to 5 x 2 tiles), then k_grid_wt accumulates each tile's samples in LDS
// (FP64), taps interpolated bilinearly from the plane's table at (d - f) WP_OS, and writes
// the tile once, zeros included: no global atomics and no separate clearing pass.  Taps
// outside the half plane u <= 0 or with |cell| >= N/2 are dropped (the mirror of a dropped
// tap is dropped too).
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

// Exclusive prefix sum of a[0..n) in LDS by the first wavefront (the caller synchronises).
__device__ void wave0_exclusive_scan(int* a, int n) {
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  const int per = (n + 63) / 64;
  const int lo = min(n, lane * per), hi = min(n, lo + per);
  int s = 0;
  for (int q = lo; q < hi; ++q) s += a[q];
  int incl = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  int run = incl - s;
  for (int q = lo; q < hi; ++q) {
    const int t = a[q];
    a[q] = run;
    run += t;
  }
}

// Plane of a visibility: nearest to |w| (halves away from zero, the cell rounding), at most
// the instance's last; a non-finite w compares false and takes the last plane too, so no
// NaN or infinity reaches the integer conversion.
__device__ __forceinline__ int plane_of(const WInst& wi, double w) {
  const double p = rhaz(fabs(w) / wi.dw);
  return p < (double)(wi.n_planes - 1) ? (int)p : wi.n_planes - 1;
}

// Tile lists of the dirty half grid for w-projection: one workgroup per instance, counting
// sort of (sample, tile) entries (k << 1 | mirror) into ent[vis_off * WP_ENT ...].
__global__ void __launch_bounds__(1024)
k_bin_w(const InstDesc* __restrict__ inst, const float2* __restrict__ uv, const float* __restrict__ w_in,
        const float* __restrict__ wl, const WInst* __restrict__ winst, const WPlane* __restrict__ planes,
        int* __restrict__ ent, int* __restrict__ tstart, int* __restrict__ tcount) {
  extern __shared__ int cnt[];
  const int i = blockIdx.x;
  const InstDesc d = inst[i];
  const WInst wi = winst[i];
  const int N = d.N, h = N / 2, ntj = N / TJ, nt = (h / TK) * ntj;
  int* E = ent + d.vis_off * WP_ENT;
  for (int t = threadIdx.x; t < nt; t += blockDim.x) cnt[t] = 0;
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    for (int k = threadIdx.x; k < d.n_vis; k += blockDim.x) {
      const int64_t vi = d.vis_off + k;
      const float2 q = uv[vi];
      const Sample sm = prep_sample(q.x, q.y, w_in[vi], d.scale, N);
      if (!sm.keep) continue;
      const int H = (planes[wi.plane0 + plane_of(wi, (double)wl[vi])].S - 1) / 2;
      for (int m = 0; m < 2; ++m) {
        const int cu = m ? -sm.cu : sm.cu, cv = m ? -sm.cv : sm.cv;
        const int kp_lo = max(0, cu - H + h - 1), kp_hi = min(h - 1, cu + H + h - 1);
        const int j_lo = max(1, cv - H + h), j_hi = min(N - 1, cv + H + h);
        if (kp_lo > kp_hi || j_lo > j_hi) continue;
        for (int tk = kp_lo / TK; tk <= kp_hi / TK; ++tk)
          for (int tj = j_lo / TJ; tj <= j_hi / TJ; ++tj) {
            const int slot = atomicAdd(&cnt[tk * ntj + tj], 1);
            if (pass) E[slot] = (k << 1) | m;
          }
      }
    }
    __syncthreads();
    if (pass == 0) {
      for (int t = threadIdx.x; t < nt; t += blockDim.x) tcount[d.tile_base_d + t] = cnt[t];
      __syncthreads();
      wave0_exclusive_scan(cnt, nt);
      __syncthreads();
      for (int t = threadIdx.x; t < nt; t += blockDim.x) tstart[d.tile_base_d + t] = (int)(d.vis_off * WP_ENT) + cnt[t];
      __syncthreads();
    }
  }
}

constexpr int WG_THREADS = 256;
constexpr int WG_CHUNK = 8;      // tiles per workgroup
constexpr int WG_EB = 256;       // samples staged at a time
// LDS accumulator row stride: one cell of padding moves the rows that the lanes of one
// sample add into (same column, consecutive rows) onto different banks.
constexpr int WG_RS = TJ + 1;

// Grid cells are written once and read only by the next kernel: nontemporal 16-byte stores.
typedef double wt_double2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void put_wcell(double2* p, double x, double y) {
  const wt_double2 v = {x, y};
  __builtin_nontemporal_store(v, reinterpret_cast<wt_double2*>(p));
}

// Tiled w-projection gridder: WG_CHUNK consecutive tiles of the dirty half grids per
// workgroup; (sample, tap row) items over the threads, FP64 LDS accumulation, one flush.
__global__ void __launch_bounds__(WG_THREADS)
k_grid_wt(const InstDesc* __restrict__ inst, const int* __restrict__ tile_inst, int n_tiles,
          const float2* __restrict__ vis, const float2* __restrict__ uv, const float* __restrict__ wl,
          const float* __restrict__ w_in, const float* __restrict__ wts, const int* __restrict__ ent,
          const int* __restrict__ tstart, const int* __restrict__ tcount, const WInst* __restrict__ winst,
          const WPlane* __restrict__ planes, const double2* __restrict__ tabs, double2* __restrict__ grid) {
  __shared__ double2 acc[TK * WG_RS];
  __shared__ int m_inst[WG_CHUNK], m_start[WG_CHUNK], m_cnt[WG_CHUNK];
  __shared__ int s_kp[WG_EB], s_j[WG_EB], s_pl[WG_EB];
  __shared__ double s_fu[WG_EB], s_fv[WG_EB], s_wr[WG_EB], s_wi[WG_EB];
  const int tid = threadIdx.x;
  const int g0 = blockIdx.x * WG_CHUNK;
  if (g0 >= n_tiles) return;
  const int gn = min(WG_CHUNK, n_tiles - g0);
  for (int t = tid; t < gn; t += WG_THREADS) {
    m_inst[t] = tile_inst[g0 + t];
    m_start[t] = tstart[g0 + t];
    m_cnt[t] = tcount[g0 + t];
  }
  __syncthreads();
  for (int tt = 0; tt < gn; ++tt) {
    const int g = g0 + tt;
    const int i = __builtin_amdgcn_readfirstlane(m_inst[tt]);
    const InstDesc d = inst[i];
    const WInst wi = winst[i];
    const int N = d.N, h = N / 2, ntj = N / TJ;
    const int t = g - d.tile_base_d;
    const int k0 = (t / ntj) * TK, j0 = (t % ntj) * TJ;
    double2* out = grid + d.gd_off + (int64_t)k0 * N + j0;
    const int n = __builtin_amdgcn_readfirstlane(m_cnt[tt]);
    if (n == 0) {                                    // empty tile: plain zero fill
      for (int q = tid; q < TK * TJ; q += WG_THREADS) put_wcell(out + (int64_t)(q / TJ) * N + (q % TJ), 0.0, 0.0);
      continue;
    }
    const int Smax = planes[wi.plane0 + wi.n_planes - 1].S, Hmax = (Smax - 1) / 2;
    for (int q = tid; q < TK * WG_RS; q += WG_THREADS) acc[q] = make_double2(0.0, 0.0);
    const int st = m_start[tt];
    for (int e0 = 0; e0 < n; e0 += WG_EB) {
      const int ne = min(WG_EB, n - e0);
      __syncthreads();                               // acc zeroed / previous batch consumed
      if (tid < ne) {
        const int en = ent[st + e0 + tid];
        const int k = en >> 1;
        const bool mirror = en & 1;
        const int64_t vi = d.vis_off + k;
        const float2 q = uv[vi];
        const Sample sm = prep_sample(q.x, q.y, w_in[vi], d.scale, N);
        const double fu = (double)q.x * d.scale - (double)sm.cu, fv = (double)q.y * d.scale - (double)sm.cv;
        const double wt = (double)wts[vi];
        const float2 v = vis[vi];
        const double ww = (double)wl[vi];
        const int pl = wi.plane0 + plane_of(wi, ww);
        const bool cj = (mirror ? -ww : ww) < 0.0;   // K_{-w} = conj(K_w)
        s_kp[tid] = (mirror ? -sm.cu : sm.cu) + h - 1;
        s_j[tid] = (mirror ? -sm.cv : sm.cv) + h;
        s_pl[tid] = cj ? ~pl : pl;
        s_fu[tid] = mirror ? -fu : fu;
        s_fv[tid] = mirror ? -fv : fv;
        s_wr[tid] = wt * (double)v.x;
        s_wi[tid] = wt * (double)(mirror ? -v.y : v.y);
      }
      __syncthreads();
      for (int it = tid; it < ne * Smax; it += WG_THREADS) {
        const int e = it / Smax, du = it - e * Smax - Hmax;
        const int plx = s_pl[e];
        const bool cj = plx < 0;
        const WPlane pl = planes[cj ? ~plx : plx];
        const int H = (pl.S - 1) / 2;
        if (du < -H || du > H) continue;
        const int kp = s_kp[e] + du;
        if (kp < k0 || kp >= k0 + TK || kp < 0 || kp > h - 1) continue;
        const int nd = pl.S * WP_OS + 1, half = pl.S * WP_OS / 2;
        const double x = ((double)du - s_fu[e]) * WP_OS;
        const int x0 = min((int)floor(x), half - 1);
        const double ax = x - x0;
        const double2* trow = tabs + pl.off + (x0 + half);
        const int jb = s_j[e];
        const double fv = s_fv[e], wr = s_wr[e], wim = s_wi[e];
        for (int dv = -H; dv <= H; ++dv) {
          const int j = jb + dv;
          if (j < j0 || j >= j0 + TJ || j < 1 || j > N - 1) continue;
          const double y = ((double)dv - fv) * WP_OS;
          const int y0 = min((int)floor(y), half - 1);
          const double ay = y - y0;
          const double2* t0 = trow + (int64_t)(y0 + half) * nd;
          const double2 k00 = t0[0], k01 = t0[1], k10 = t0[nd], k11 = t0[nd + 1];
          const double kr = (1 - ay) * ((1 - ax) * k00.x + ax * k01.x) + ay * ((1 - ax) * k10.x + ax * k11.x);
          double ki = (1 - ay) * ((1 - ax) * k00.y + ax * k01.y) + ay * ((1 - ax) * k10.y + ax * k11.y);
          if (cj) ki = -ki;
          double* a = reinterpret_cast<double*>(&acc[(kp - k0) * WG_RS + (j - j0)]);
          atomicAdd(a, wr * kr - wim * ki);
          atomicAdd(a + 1, wr * ki + wim * kr);
        }
      }
    }
    __syncthreads();
    for (int q = tid; q < TK * TJ; q += WG_THREADS) {
      const int l = q / TJ, jj = q % TJ;
      double2 val = acc[l * WG_RS + jj];
      if (((k0 + l + 1) + (j0 + jj)) & 1) { val.x = -val.x; val.y = -val.y; }
      put_wcell(out + (int64_t)l * N + jj, val.x, val.y);
    }
    __syncthreads();
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

hipError_t launch_bin_w(const InstDesc* inst, int n_inst, size_t lds_bytes, const float2* uv, const float* w_in,
                       const float* wl, const WInst* winst, const WPlane* planes, int* ent, int* tstart, int* tcount,
                       hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bin_w, dim3(n_inst), dim3(1024), lds_bytes, st, inst, uv, w_in, wl, winst, planes, ent, tstart,
                     tcount);
  return hipGetLastError();
}

hipError_t launch_grid_wt(const InstDesc* inst, const int* tile_inst, int n_tiles, const float2* vis, const float2* uv,
                          const float* wl, const float* w_in, const float* wts, const int* ent, const int* tstart,
                          const int* tcount, const WInst* winst, const WPlane* planes, const double2* tabs,
                          double2* grid, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  const int blocks = (n_tiles + WG_CHUNK - 1) / WG_CHUNK;
  hipLaunchKernelGGL(k_grid_wt, dim3(blocks), dim3(WG_THREADS), 0, st, inst, tile_inst, n_tiles, vis, uv, wl, w_in,
                     wts, ent, tstart, tcount, winst, planes, tabs, grid);
  return hipGetLastError();
}

}  // namespace mi
