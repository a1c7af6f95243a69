// Prep, weighting, tile binning and LDS-tiled convolutional gridding (gfx950).
//
// Sec. 3.2.3: visibilities are convolved with the prolate spheroidal gridding function and
// resampled onto the uniform UV grid, with natural or uniform weighting (Algorithm 1,
// wgtGrid_kernel: mode 1 = uniform, otherwise natural).  The paper's kernel scales gridded
// cells by 1/cnt over the half plane; here the same weights are applied per visibility
// (w_in / cnt of its nearest cell, mirrors included), which is what the cell scaling does
// for a one-cell kernel and the usual definition for a wider one.
//
// Data flow per batch:
//   k_bin   one workgroup per instance: keep/cell decisions, uniform counts (sparse
//           scratch grid, touched cells only), per-visibility weights, B0 sums, and a
//           counting sort of (sample, tile) entries for the dirty and the beam half grids.
//   k_grid  a chunk of consecutive tiles of TK lines x TJ cells of a half grid per
//           workgroup: accumulate each tile's samples into LDS (no global atomics), then one
//           coalesced flush of nontemporal 16-byte stores that writes every cell of the
//           tile (zeros included), so no separate memset pass.
#include <type_traits>

#include "mi_internal.h"

namespace mi {

namespace {

constexpr int BIN_THREADS = 1024;

__device__ __forceinline__ int wave_sum_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Exclusive scan of a[0..n) in LDS, in place; returns the total.  All threads call it.
__device__ int block_exclusive_scan(int* a, int n, int* wave_tot) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int per = (n + nthr - 1) / nthr;
  const int lo = min(n, tid * per), hi = min(n, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += a[i];
  // inclusive wave scan of the per-thread sums
  const int lane = tid & 63, wave = tid >> 6;
  int incl = s;
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wave_tot[wave] = incl;
  __syncthreads();
  const int nw = nthr >> 6;
  if (tid == 0) {
    int acc = 0;
    for (int w = 0; w < nw; ++w) { int t = wave_tot[w]; wave_tot[w] = acc; acc += t; }
    wave_tot[nw] = acc;
  }
  __syncthreads();
  int run = wave_tot[wave] + incl - s;
  for (int i = lo; i < hi; ++i) { int t = a[i]; a[i] = run; run += t; }
  int total = wave_tot[nw];
  __syncthreads();
  return total;
}

// Tiles of the half grid (lines k' = 0..P/2-1 for u-cells c_u = k'+1-P/2 <= 0) touched by
// a sample centred on cell (cu, cv).  Returns false when no tap lies in the half plane.
__device__ __forceinline__ bool tile_range(int cu, int cv, int P, int& tk0, int& tk1, int& tj0, int& tj1) {
  if (cu - HALF_W > 0) return false;
  const int h = P / 2;
  const int kp_lo = max(0, cu - HALF_W + h - 1);
  const int kp_hi = min(h - 1, cu + HALF_W + h - 1);
  tk0 = kp_lo / TK;
  tk1 = kp_hi / TK;
  tj0 = (cv - HALF_W + h) / TJ;
  tj1 = (cv + HALF_W + h) / TJ;
  return true;
}

// Line blocks of lb whole lines touched by a sample centred on cell (cu, cv): the
// half-plane lines k' = cu + du + P/2 - 1 <= P/2 - 1 it reaches, in blocks of lb.
__device__ __forceinline__ bool block_range(int cu, int P, int lb, int& b0, int& b1) {
  if (cu - HALF_W > 0) return false;
  const int h = P / 2;
  const int kp_lo = max(0, cu - HALF_W + h - 1);
  const int kp_hi = min(h - 1, cu + HALF_W + h - 1);
  b0 = kp_lo / lb;
  b1 = kp_hi / lb;
  return true;
}

// Count (pass 0) or scatter (pass 1) the entries of one half grid: per tile of TK x TJ
// cells (lb = 0), or per block of lb whole lines (the fused gridding + transform passes).
// With rec (line blocks only), the scatter pass writes self-contained records instead.
__device__ void bin_pass(const InstDesc& d, const float2* __restrict__ uv, const float* __restrict__ w_in,
                         bool beam, int pass, int* cnt, int* __restrict__ ent, int lb,
                         GridRec* __restrict__ rec = nullptr, const float2* __restrict__ vis = nullptr,
                         const float* __restrict__ wts = nullptr) {
  const int N = d.N, P = beam ? 2 * N : N;
  const int ntj = lb ? 1 : P / TJ;
  for (int k = threadIdx.x; k < d.n_vis; k += blockDim.x) {
    const float2 q = uv[d.vis_off + k];
    const Sample s = prep_sample(q.x, q.y, w_in[d.vis_off + k], d.scale, N);
    if (!s.keep) continue;
    const int cu = beam ? s.cu2 : s.cu, cv = beam ? s.cv2 : s.cv;
    const int ou = beam ? s.ou2 : s.ou, ov = beam ? s.ov2 : s.ov;
    float2 v = make_float2(1.f, 0.f);
    float wk = 0.f;
    if (rec && pass) {
      wk = wts[d.vis_off + k];
      if (!beam) v = vis ? vis[d.vis_off + k] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int su = m ? -cu : cu, sv = m ? -cv : cv;
      int tk0, tk1, tj0, tj1;
      if (lb) {
        if (!block_range(su, P, lb, tk0, tk1)) continue;
        tj0 = tj1 = 0;
      } else if (!tile_range(su, sv, P, tk0, tk1, tj0, tj1)) {
        continue;
      }
      for (int tk = tk0; tk <= tk1; ++tk)
        for (int tj = tj0; tj <= tj1; ++tj) {
          const int t = tk * ntj + tj;
          const int slot = atomicAdd(&cnt[t], 1);
          if (pass && rec) {
            GridRec r;
            r.cucv = (int)(((unsigned)su << 16) | ((unsigned)sv & 0xffffu));
            r.ouov = (((m ? -ou : ou) + OS / 2) << 8) | ((m ? -ov : ov) + OS / 2);
            r.w = wk;
            r.pad0 = 0;
            r.vr = v.x;
            r.vi = m ? -v.y : v.y;
            r.pad1 = r.pad2 = 0.f;
            rec[slot] = r;
          } else if (pass) {
            ent[slot] = (k << 1) | m;
          }
        }
    }
  }
}

}  // namespace

__global__ void __launch_bounds__(BIN_THREADS)
k_bin(const InstDesc* __restrict__ inst, const float2* __restrict__ uv, const float* __restrict__ w_in,
      Tables T, float* __restrict__ wts, double* __restrict__ b0, int* __restrict__ nkept,
      int* __restrict__ status, float* __restrict__ cnt_scratch,
      int* __restrict__ ent_d, int* __restrict__ ent_b,
      int* __restrict__ tstart_d, int* __restrict__ tcount_d,
      int* __restrict__ tstart_b, int* __restrict__ tcount_b, int fail_inst, int do_beam, int unit_w,
      int lb_elems_d, int lb_elems_b, const float2* __restrict__ vis, GridRec* __restrict__ rec_d,
      GridRec* __restrict__ rec_b) {
  extern __shared__ int lds[];
  __shared__ int wave_tot[BIN_THREADS / 64 + 1];
  __shared__ double red_d[2][BIN_THREADS / 64];
  __shared__ int red_i[BIN_THREADS / 64];
  const int i = blockIdx.x;
  const InstDesc d = inst[i];
  const int N = d.N, tid = threadIdx.x;

  // ---- uniform weighting: sum of w_in per nearest N-grid cell (mirrors included).  Only
  // touched cells of the scratch grid are written (zeroed first), so no dense clear.
  float* cnt = (d.mode == 1 && !unit_w) ? cnt_scratch + d.cnt_off : nullptr;
  if (cnt) {
    for (int k = tid; k < d.n_vis; k += blockDim.x) {
      const float2 q = uv[d.vis_off + k];
      const Sample s = prep_sample(q.x, q.y, w_in[d.vis_off + k], d.scale, N);
      if (!s.keep) continue;
      cnt[(s.cv + N / 2) * N + (s.cu + N / 2)] = 0.0f;
      cnt[(-s.cv + N / 2) * N + (-s.cu + N / 2)] = 0.0f;
    }
    __syncthreads();
    for (int k = tid; k < d.n_vis; k += blockDim.x) {
      const float2 q = uv[d.vis_off + k];
      const float wi = w_in[d.vis_off + k];
      const Sample s = prep_sample(q.x, q.y, wi, d.scale, N);
      if (!s.keep) continue;
      atomicAdd(&cnt[(s.cv + N / 2) * N + (s.cu + N / 2)], wi);
      atomicAdd(&cnt[(-s.cv + N / 2) * N + (-s.cu + N / 2)], wi);
    }
    __syncthreads();
  }

  // ---- per-visibility weights, kept count, B0 of both grids (FP64 sums)
  double sd = 0.0, sb = 0.0;
  int nk = 0;
  for (int k = tid; k < d.n_vis; k += blockDim.x) {
    const float2 q = uv[d.vis_off + k];
    const float wi = w_in[d.vis_off + k];
    const Sample s = prep_sample(q.x, q.y, wi, d.scale, N);
    float w = 0.0f;
    if (s.keep) {
      w = unit_w ? 1.0f : cnt ? wi / cnt[(s.cv + N / 2) * N + (s.cu + N / 2)] : wi;
      ++nk;
      const double wd = 2.0 * (double)w;
      sd += wd * T.tsum[s.ou + OS / 2] * T.tsum[s.ov + OS / 2];
      sb += wd * T.tsum[s.ou2 + OS / 2] * T.tsum[s.ov2 + OS / 2];
    }
    wts[d.vis_off + k] = w;
  }
  __threadfence_block();      // the records written below read these weights back
  sd = wave_sum_d(sd);
  sb = wave_sum_d(sb);
  nk = wave_sum_i(nk);
  if ((tid & 63) == 0) {
    red_d[0][tid >> 6] = sd;
    red_d[1][tid >> 6] = sb;
    red_i[tid >> 6] = nk;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, b = 0.0;
    int n = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { a += red_d[0][w]; b += red_d[1][w]; n += red_i[w]; }
    b0[2 * i + 0] = a * T.inv_corr0_sq;
    b0[2 * i + 1] = b * T.inv_corr0_sq;
    nkept[i] = n;
    if (status) status[i] = (n == 0 ? 1 : 0) | (i == fail_inst ? 8 : 0);
  }

  // ---- counting sort of (sample, tile) entries, dirty grid then beam grid; with
  // lb_elems_* > 0, of (sample, line block) entries for the fused gridding + transform
  // passes, blocks of the lines one transform workgroup of that many points holds
  for (int g = 0; g < (do_beam ? 2 : 1); ++g) {
    const bool beam = g == 1;
    const int P = beam ? 2 * N : N;
    const int le = beam ? lb_elems_b : lb_elems_d;
    int lb = 0;
    if (le) lb = beam ? min(2 * le / P, P / 2) : min(le / P, P / 2);   // real lines (beam) / lines
    const int nt = lb ? (P / 2) / lb : (P / 2 / TK) * (P / TJ);
    const int base = lb ? (beam ? d.blk_base_b : d.blk_base_d) : (beam ? d.tile_base_b : d.tile_base_d);
    int* ent = (beam ? ent_b : ent_d) + d.ent_off;
    int* tstart = (beam ? tstart_b : tstart_d) + base;
    int* tcount = (beam ? tcount_b : tcount_d) + base;
    for (int t = tid; t < nt; t += blockDim.x) lds[t] = 0;
    __syncthreads();
    bin_pass(d, uv, w_in, beam, 0, lds, nullptr, lb);
    __syncthreads();
    for (int t = tid; t < nt; t += blockDim.x) tcount[t] = lds[t];
    __syncthreads();
    block_exclusive_scan(lds, nt, wave_tot);
    for (int t = tid; t < nt; t += blockDim.x) tstart[t] = (int)(d.ent_off) + lds[t];
    __syncthreads();
    bin_pass(d, uv, w_in, beam, 1, lds, ent, lb, lb ? (beam ? rec_b : rec_d) + d.ent_off : nullptr, vis, wts);
    __syncthreads();
  }
}

// Tiles of TK x TJ cells, `chunk` consecutive tiles per workgroup (their metadata
// staged in LDS, so a run of empty tiles is a stream of stores with no dependent global
// loads).  A non-empty tile stages up to GRID_EB of its samples' parameters in LDS, then
// spreads (sample, tap row) pairs over all threads; accumulation is FP64 in LDS (the grid
// correction later amplifies grid rounding by up to ~1e6 in the map corners).  The chunk
// is chosen per context (mi_set_tuning; 8 by default): on a 520 x 1024^2 dirty + beam batch
// 8 measured fastest (32: 1.1 ms slower, the few dense tiles near each uv centre holding
// their workgroup longer; 2-4: more per-workgroup setup).
constexpr int GRID_THREADS = 256;
constexpr int GRID_CHUNK_MAX = 32;   // tiles per workgroup: a tuning choice up to this
constexpr int GRID_EB = 256;
// Row stride of the LDS accumulator.  The seven lanes of one sample add into seven tile
// rows at the same column, which a 64-cell stride puts in one LDS bank; one cell of
// padding per complex row shifts consecutive rows by 4 banks (0.16 ms less for the dirty
// grids of a 520 x 1024^2 batch).  Real (beam) rows stay unpadded: two cells of padding
// there measured no faster.
template <bool REAL> constexpr int acc_stride() { return REAL ? TJ : TJ + 1; }

// Grid cell stores: FP64 complex or complex64 (mi_grid output); the real FP64 beam grid
// (imaginary part zero) is stored two cells at a time.  The FP64 grids are written with
// nontemporal 16-byte stores: each cell is written once and read back only by the next
// kernel, and streaming them past the caches took 0.3 ms off the dirty and 0.45 ms off the
// beam stage of a 520 x 1024^2 batch (the same hint on the transform passes' stores was
// neutral or slower).
typedef double nt_double2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void put2_nt(double* p, double a, double b) {
  const nt_double2 v = {a, b};
  __builtin_nontemporal_store(v, reinterpret_cast<nt_double2*>(p));
}
__device__ __forceinline__ void put_cell(double2* p, double2 v) { put2_nt(&p->x, v.x, v.y); }
__device__ __forceinline__ void put_cell(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }

template <class OutT>
__global__ void __launch_bounds__(GRID_THREADS)
k_grid(const InstDesc* __restrict__ inst, const int* __restrict__ tile_inst, int n_tiles, int beam,
       const float2* __restrict__ vis, const float2* __restrict__ uv, const float* __restrict__ w_in,
       const float* __restrict__ wts, const int* __restrict__ ent,
       const int* __restrict__ tstart, const int* __restrict__ tcount, Tables T,
       OutT* __restrict__ grid, int modulate, int chunk) {
  constexpr bool REAL = std::is_same<OutT, double>::value;
  constexpr int RS = acc_stride<REAL>();
  __shared__ double2 acc[REAL ? TK * RS / 2 : TK * RS];
  double* accr = reinterpret_cast<double*>(acc);       // real grids: one double per cell
  static_assert(!REAL || RS % 2 == 0, "real cell pairs are read as 16 bytes");
  __shared__ double tab[TAB_LEN];
  __shared__ int m_inst[GRID_CHUNK_MAX], m_start[GRID_CHUNK_MAX], m_cnt[GRID_CHUNK_MAX];
  __shared__ int s_kp[GRID_EB], s_j[GRID_EB], s_ou[GRID_EB], s_ov[GRID_EB];
  __shared__ double s_wr[GRID_EB], s_wi[GRID_EB];
  const int tid = threadIdx.x;
  const int g0 = blockIdx.x * chunk;
  if (g0 >= n_tiles) return;
  const int gn = min(chunk, n_tiles - g0);
  for (int t = tid; t < TAB_LEN; t += GRID_THREADS) tab[t] = T.tab[t];
  for (int t = tid; t < gn; t += GRID_THREADS) {
    m_inst[t] = tile_inst[g0 + t];
    m_start[t] = tstart[g0 + t];
    m_cnt[t] = tcount[g0 + t];
  }
  __syncthreads();

  for (int tt = 0; tt < gn; ++tt) {
    const int g = g0 + tt;
    const int i = __builtin_amdgcn_readfirstlane(m_inst[tt]);
    const InstDesc d = inst[i];
    const int N = d.N, P = beam ? 2 * N : N, h = P / 2;
    const int t = g - (beam ? d.tile_base_b : d.tile_base_d);
    const int ntj = P / TJ;
    const int k0 = (t / ntj) * TK, j0 = (t % ntj) * TJ;
    OutT* out = grid + (beam ? d.gb_off : d.gd_off) + (int64_t)k0 * P + j0;
    const int n = __builtin_amdgcn_readfirstlane(m_cnt[tt]);

    if (n == 0) {  // empty tile: plain zero fill
      if constexpr (std::is_same<OutT, double>::value) {   // real cells, two per 16-byte store
        for (int q = tid; q < TK * TJ / 2; q += GRID_THREADS)
          put2_nt(out + (int64_t)(2 * q / TJ) * P + (2 * q % TJ), 0.0, 0.0);
      } else {
        for (int q = tid; q < TK * TJ; q += GRID_THREADS)
          put_cell(out + (int64_t)(q / TJ) * P + (q % TJ), make_double2(0.0, 0.0));
      }
      continue;
    }
    if constexpr (REAL) {
      for (int q = tid; q < TK * RS / 2; q += GRID_THREADS) acc[q] = make_double2(0.0, 0.0);
    } else {
      for (int q = tid; q < TK * RS; q += GRID_THREADS) acc[q] = make_double2(0.0, 0.0);
    }
    const int st = m_start[tt];
    for (int e0 = 0; e0 < n; e0 += GRID_EB) {
      const int ne = min(GRID_EB, n - e0);
      __syncthreads();                                 // acc zeroed / previous stage consumed
      if (tid < ne) {
        const int en = ent[st + e0 + tid];
        const int k = en >> 1;
        const bool mirror = en & 1;
        const int64_t vi = d.vis_off + k;
        const float2 q = uv[vi];
        const Sample sm = prep_sample(q.x, q.y, w_in[vi], d.scale, N);
        int cu = beam ? sm.cu2 : sm.cu, cv = beam ? sm.cv2 : sm.cv;
        int ou = beam ? sm.ou2 : sm.ou, ov = beam ? sm.ov2 : sm.ov;
        float2 v = beam ? make_float2(1.f, 0.f) : vis[vi];
        if (mirror) { cu = -cu; cv = -cv; ou = -ou; ov = -ov; v.y = -v.y; }
        const double w = (double)wts[vi];
        s_kp[tid] = cu + h - 1;
        s_j[tid] = cv + h;
        s_ou[tid] = ou;
        s_ov[tid] = ov;
        s_wr[tid] = w * (double)v.x;
        s_wi[tid] = w * (double)v.y;
      }
      __syncthreads();
      for (int wi = tid; wi < ne * W; wi += GRID_THREADS) {
        const int e = wi / W, du = wi - e * W - HALF_W;
        const int kp = s_kp[e] + du;
        if (kp < k0 || kp >= k0 + TK || kp > h - 1) continue;
        const double tu = tab[du * OS - s_ou[e] + TAB_CENTRE];
        const int jb = s_j[e], ov = s_ov[e];
        const double wr = s_wr[e], wim = s_wi[e];
#pragma unroll
        for (int dv = -HALF_W; dv <= HALF_W; ++dv) {
          const int j = jb + dv;
          if (j < j0 || j >= j0 + TJ) continue;
          const double kk = tu * tab[dv * OS - ov + TAB_CENTRE];
          const int c = (kp - k0) * RS + (j - j0);
          if constexpr (REAL) {
            atomicAdd(accr + c, wr * kk);
          } else {
            double* a = reinterpret_cast<double*>(&acc[c]);
            atomicAdd(a, wr * kk);
            if (!beam) atomicAdd(a + 1, wim * kk);
          }
        }
      }
    }
    __syncthreads();
    if constexpr (REAL) {                                  // real cells, two per 16-byte store
      for (int q = tid; q < TK * TJ / 2; q += GRID_THREADS) {
        const int l = 2 * q / TJ, jj = 2 * q % TJ;
        double2 val = *reinterpret_cast<const double2*>(accr + l * RS + jj);   // RS and jj even
        if (modulate) {
          if (((k0 + l + 1) + (j0 + jj)) & 1) val.x = -val.x;
          else val.y = -val.y;
        }
        put2_nt(out + (int64_t)l * P + jj, val.x, val.y);
      }
    } else {
      for (int q = tid; q < TK * TJ; q += GRID_THREADS) {
        const int l = q / TJ, jj = q % TJ;
        double2 val = acc[l * RS + jj];
        if (modulate && (((k0 + l + 1) + (j0 + jj)) & 1)) { val.x = -val.x; val.y = -val.y; }
        put_cell(out + (int64_t)l * P + jj, val);
      }
    }
    __syncthreads();
  }
}

// Expand FP64 half grids into full centred P x P complex64 grids G[j][i] (mi_grid layout).
__global__ void k_expand_full(const InstDesc* __restrict__ inst, int n_inst, int beam,
                              const double2* __restrict__ half, float2* __restrict__ full,
                              const int64_t* __restrict__ full_off) {
  const int i = blockIdx.y;
  if (i >= n_inst) return;
  const InstDesc d = inst[i];
  const int P = beam ? 2 * d.N : d.N, h = P / 2;
  const double2* H = half + (beam ? d.gb_off : d.gd_off);
  float2* G = full + full_off[i];
  const int64_t tot = (int64_t)P * P;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < tot; q += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(q / P), ii = (int)(q % P);
    const int cu = ii - h, cv = j - h;
    float2 val = make_float2(0.f, 0.f);
    if (ii > 0 && j > 0) {
      if (cu <= 0) {
        const double2 v = H[(int64_t)(ii - 1) * P + j];
        val = make_float2((float)v.x, (float)v.y);
      } else {
        const int mi_ = -cu + h, mj = -cv + h;
        const double2 v = H[(int64_t)(mi_ - 1) * P + mj];
        val = make_float2((float)v.x, -(float)v.y);
      }
    }
    G[q] = val;
  }
}

// ---- host launchers ----
hipError_t launch_bin(const InstDesc* inst, int n_inst, const float2* uv, const float* w_in, const Tables& T,
                      float* wts, double* b0, int* nkept, int* status, float* cnt, int* ent_d, int* ent_b,
                      int* tstart_d, int* tcount_d, int* tstart_b, int* tcount_b, int fail_inst, int do_beam,
                      int unit_w, int lb_elems_d, int lb_elems_b, const float2* vis, GridRec* rec_d,
                      GridRec* rec_b, size_t lds_bytes, hipStream_t st) {
  hipLaunchKernelGGL(k_bin, dim3(n_inst), dim3(BIN_THREADS), lds_bytes, st, inst, uv, w_in, T, wts, b0, nkept,
                     status, cnt, ent_d, ent_b, tstart_d, tcount_d, tstart_b, tcount_b, fail_inst, do_beam, unit_w,
                     lb_elems_d, lb_elems_b, vis, rec_d, rec_b);
  return hipGetLastError();
}

template <class OutT>
hipError_t launch_grid_t(const InstDesc* inst, const int* tile_inst, int n_tiles, int beam, const float2* vis,
                         const float2* uv, const float* w_in, const float* wts, const int* ent, const int* tstart,
                         const int* tcount, const Tables& T, OutT* grid, int modulate, int chunk, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  if (chunk < 1 || chunk > GRID_CHUNK_MAX) return hipErrorInvalidValue;
  const int blocks = (n_tiles + chunk - 1) / chunk;
  hipLaunchKernelGGL((k_grid<OutT>), dim3(blocks), dim3(GRID_THREADS), 0, st, inst, tile_inst, n_tiles, beam, vis,
                     uv, w_in, wts, ent, tstart, tcount, T, grid, modulate, chunk);
  return hipGetLastError();
}

hipError_t launch_grid(const InstDesc* inst, const int* tile_inst, int n_tiles, int beam, const float2* vis,
                       const float2* uv, const float* w_in, const float* wts, const int* ent, const int* tstart,
                       const int* tcount, const Tables& T, double2* grid, int modulate, int chunk, hipStream_t st) {
  return launch_grid_t(inst, tile_inst, n_tiles, beam, vis, uv, w_in, wts, ent, tstart, tcount, T, grid, modulate,
                       chunk, st);
}

hipError_t launch_grid_f32(const InstDesc* inst, const int* tile_inst, int n_tiles, int beam, const float2* vis,
                           const float2* uv, const float* w_in, const float* wts, const int* ent, const int* tstart,
                           const int* tcount, const Tables& T, float2* grid, int modulate, int chunk,
                           hipStream_t st) {
  return launch_grid_t(inst, tile_inst, n_tiles, beam, vis, uv, w_in, wts, ent, tstart, tcount, T, grid, modulate,
                       chunk, st);
}

hipError_t launch_grid_real(const InstDesc* inst, const int* tile_inst, int n_tiles, const float2* uv,
                            const float* w_in, const float* wts, const int* ent, const int* tstart, const int* tcount,
                            const Tables& T, double* grid, int chunk, hipStream_t st) {
  return launch_grid_t(inst, tile_inst, n_tiles, 1, nullptr, uv, w_in, wts, ent, tstart, tcount, T, grid, 1, chunk,
                       st);
}

hipError_t launch_expand_full(const InstDesc* inst, int n_inst, int beam, const double2* half, float2* full,
                              const int64_t* full_off, hipStream_t st) {
  hipLaunchKernelGGL(k_expand_full, dim3(256, n_inst), dim3(256), 0, st, inst, n_inst, beam, half, full, full_off);
  return hipGetLastError();
}

__global__ void k_fill_u32(unsigned* p, int64_t n, unsigned v) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
    p[q] = v;
}

hipError_t launch_fill_u32(unsigned* p, int64_t n, unsigned v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)b), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace mi
