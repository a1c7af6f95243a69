// LDS-resident Stockham FFTs for the imaging transform and its adjoint (gfx950, FP64).
//
// Sec. 3.2.3: an inverse FFT of the gridded visibilities gives the dirty image (with the
// disk at the centre, Algorithm 1).  The centred transform
//   I[y][x] = sum G[j][i] exp(+2 pi i ((i-P/2)(x-P/2) + (j-P/2)(y-P/2)) / P)
// is computed for even P as (-1)^(x+y) IDFT[(-1)^(i+j) G], so no shift passes are needed:
// the gridder applies (-1)^(i+j) when it flushes a tile and the last pass applies
// (-1)^(x+y) together with the grid correction 1/(corr(x) corr(y)) and 1/B0.
//
// Precision: the correction divides by corr(x) corr(y), about 1e-6 in the map corners for
// the prolate spheroidal kernel, so rounding in the grid and the transform is amplified by
// up to ~1e6 there.  Grid, transform and correction therefore run in FP64; inputs and
// output images are FP32.
//
// The grid is Hermitian, so only the half plane u <= 0 is stored: P/2 lines (u index
// i = 1..P/2; i = 0 is never touched by the 7-tap kernel and is zero), each P cells long
// in v.  Two passes, each LDS-resident and reading/writing whole contiguous blocks:
//   pass A  (k_fft_a): nl lines per workgroup, length-P complex FFT along v, written as
//           one contiguous block Yb[line_block][y][line % nl] over the same footprint;
//   pass B  (k_fft_b_c2r): ny rows y per workgroup; rebuilds the Hermitian spectrum
//           along u from the blocks, length-P FFT, real part, correction, normalisation.
// The beam's grid is also real and even, which k_fft_a_real / k_fft_b_c2r_sym use to halve
// its transform work and bytes (see there).  In the imaging calls pass A is fused with the
// gridding (k_grid_fft_a, k_grid_fft_a_real: the block's samples are gridded straight into
// LDS); the separate pass A kernels serve grids built elsewhere (the w-projection gridder).
// The adjoint runs the mirror image (k_fft_b_r2c then k_fft_a_fwd); mi_ifft2 uses
// k_fft_c2c_t twice on full complex arrays.
//
// Twiddles come from a table exp(+2 pi i t / 8192) computed on the host in FP64.
#include <algorithm>

#include "mi_internal.h"
#include "fft_lds.h"

namespace mi {

namespace {

template <int ELEMS>
__device__ __forceinline__ int lines_per_block(int P) {
  const int nl = ELEMS / P;
  return nl > P / 2 ? P / 2 : nl;
}

// Rows per workgroup of the real-valued passes: two rows share one complex FFT.
template <int ELEMS>
__device__ __forceinline__ int rows_per_block(int P) {
  const int ny = 2 * ELEMS / P;
  return ny > P ? P : ny;
}

// Real lines per workgroup of the beam's pass A: two real lines share one complex FFT.
template <int ELEMS>
__device__ __forceinline__ int real_lines_per_block(int P) {
  const int nr = 2 * ELEMS / P;
  return nr > P / 2 ? P / 2 : nr;
}

constexpr int LDS_PADDED(int elems) { return elems + elems / 8; }
// Two 512-thread workgroups of the small block share a CU (LDS 2 x 72 KB), which needs
// 4 waves per SIMD, i.e. at most 128 VGPRs.
#define FFT_WAVES_PER_EU(ELEMS) ((ELEMS) <= 4096 ? 4 : 2)

}  // namespace

// The four inverse passes below are persistent: a workgroup takes work items w =
// blockIdx.x, blockIdx.x + gridDim.x, ... and issues the global loads of its next item into
// registers as soon as the current one is staged in LDS, so those loads are in flight
// during the transform and the stores (LDS barriers do not wait for global loads).  That
// only holds if nothing waits for them early: the vector memory counter completes loads
// and stores in order, and where the compiler cannot count what was issued after the load
// it needs, it waits for everything.  Hence no global load inside a transform (twiddles in
// registers, TwRegs), prefetched values kept raw until staging, only the record fields
// that are used loaded, unconditional loads, and store loops with a fixed number of
// unconditional rounds.

// Pass A (inverse, dirty grid): half-grid lines -> FFT along v -> contiguous block Yb[b][y][l].
template <int ELEMS, int THREADS>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(FFT_WAVES_PER_EU(ELEMS))))
k_fft_a(const InstDesc* __restrict__ inst, const FftWork* __restrict__ work, int n_work, double2* grid, Tables T) {
  __shared__ double2 buf[LDS_PADDED(ELEMS)];
  constexpr int NPT = ELEMS / THREADS;
  constexpr int NPF = NPT / 2;                 // prefetched half; the rest is loaded at staging
  double2 r[NPF];
  auto fetch = [&](int wi) {
    const FftWork wk = work[wi];
    const InstDesc d = inst[wk.inst];
    const int P = d.N, n = lines_per_block<ELEMS>(P) * P;
    const double2* blk = grid + d.gd_off + (int64_t)wk.first * P;
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      const int q = threadIdx.x + i * THREADS;
      if (q < n) {
        const double2 v = blk[q];
        r[i] = make_double2(v.x, v.y);   // component copy keeps r[] in registers
      }
    }
  };
  int w = blockIdx.x;
  if (w < n_work) fetch(w);
  TwRegs<ELEMS, THREADS> twr;
  for (; w < n_work; w += gridDim.x) {
    const FftWork wk = work[w];
    const InstDesc d = inst[wk.inst];
    const int P = d.N, log2P = ilog2(P);
    const int nl = lines_per_block<ELEMS>(P), log2nl = ilog2(nl);
    const int n = nl * P;
    double2* blk = grid + d.gd_off + (int64_t)wk.first * P;
#pragma unroll
    for (int i = NPF; i < NPT; ++i) {
      const int q = threadIdx.x + i * THREADS;
      if (q < n) buf[pd(q)] = blk[q];
    }
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      const int q = threadIdx.x + i * THREADS;
      if (q < n) buf[pd(q)] = r[i];
    }
    twr.ensure(log2P, T.twiddle);
    __syncthreads();
    if (w + (int)gridDim.x < n_work) fetch(w + gridDim.x);
    lds_fft<ELEMS, THREADS>(buf, log2P, nl, +1.0, T.twiddle, twr);
    // a fixed number of unconditional store rounds (n is a power of two; for P < 128 the
    // extra rounds repeat elements with identical values), so that the compiler can count
    // them and a later wait for an older load does not wait for these stores too
#pragma unroll
    for (int rd = 0; rd < ELEMS / THREADS; ++rd) {
      const int q = (threadIdx.x + rd * THREADS) & (n - 1);
      const int y = q >> log2nl, l = q & (nl - 1);
      blk[q] = buf[pd((l << log2P) + y)];
    }
    __syncthreads();
  }
}

// Pass B (inverse, complex-to-real, dirty image): rows y0..y0+ny-1, two rows per complex
// line: Z = X1 + i X2 with X1, X2 Hermitian along u, so Re IDFT(Z) and Im IDFT(Z) are the
// two real rows.  Element (line k', row y) of the blocked layout is at
// (k'/nl) nl P + y nl + k' % nl.
template <int ELEMS, int THREADS>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(FFT_WAVES_PER_EU(ELEMS))))
k_fft_b_c2r(const InstDesc* __restrict__ inst, const FftWork* __restrict__ work, int n_work,
            const double2* __restrict__ yb, const double* __restrict__ b0, Tables T, float* __restrict__ out) {
  __shared__ double2 buf[LDS_PADDED(ELEMS)];
  constexpr int NPT = ELEMS / 2 / THREADS;
  double2 r1[NPT], r2[NPT];
  auto fetch = [&](int wi) {
    const FftWork wk = work[wi];
    const InstDesc d = inst[wk.inst];
    const int P = d.N, h = P / 2;
    const int nl = lines_per_block<ELEMS>(P), log2nl = ilog2(nl);
    const int nz = rows_per_block<ELEMS>(P) / 2, log2pb = ilog2(nz * nl);
    const double2* src = yb + d.gd_off;
    // unconditional loads (lanes past the item's h * nz elements, only for P < 128, load
    // duplicates that staging ignores): a load under a lane condition leaves the compiler
    // unsure at later joins whether it is still pending, and it then waits for everything
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int q = (threadIdx.x + i * THREADS) & (h * nz - 1);
      const int b = q >> log2pb, r = q & ((1 << log2pb) - 1);
      const int zl = r >> log2nl, l = r & (nl - 1);
      const int64_t e = (int64_t)b * nl * P + (int64_t)(wk.first + 2 * zl) * nl + l;
      const double2 v1 = src[e], v2 = src[e + nl];
      r1[i] = make_double2(v1.x, v1.y);
      r2[i] = make_double2(v2.x, v2.y);
    }
  };
  int w = blockIdx.x;
  if (w < n_work) fetch(w);
  // the first item's loads settled here, so that the staging of every later item (reached
  // with the previous item's stores still in flight) waits only for its prefetch
  __builtin_amdgcn_s_waitcnt(0);
  TwRegs<ELEMS, THREADS> twr;
  for (; w < n_work; w += gridDim.x) {
    const FftWork wk = work[w];
    const InstDesc d = inst[wk.inst];
    const int P = d.N, log2P = ilog2(P), h = P / 2;
    const int nl = lines_per_block<ELEMS>(P), log2nl = ilog2(nl);
    const int ny = rows_per_block<ELEMS>(P), nz = ny / 2, log2pb = ilog2(nz * nl);
    const int y0 = wk.first;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {            // registers read by every lane, LDS written for the item's elements
      const int qi = threadIdx.x + i * THREADS, q = qi & (h * nz - 1);
      const int b = q >> log2pb, r = q & ((1 << log2pb) - 1);
      const int zl = r >> log2nl, l = r & (nl - 1);
      const double2 v1 = r1[i], v2 = r2[i];
      const int k = b * nl + l + 1;            // u frequency index 1..P/2
      const int row = zl << log2P;
      // u = 0 column (k = P/2): real by symmetry
      const double2 za = k < h ? make_double2(v1.x - v2.y, v1.y + v2.x) : make_double2(v1.x, v2.x);
      const double2 zb = make_double2(v1.x + v2.y, v2.x - v1.y);
      if (qi < h * nz) {
        buf[pd(row + k)] = za;
        if (k < h) buf[pd(row + P - k)] = zb;
      }
    }
    for (int zl = threadIdx.x; zl < nz; zl += THREADS) buf[pd(zl << log2P)] = make_double2(0.0, 0.0);
    twr.ensure(log2P, T.twiddle);
    __syncthreads();
    fetch(min(w + (int)gridDim.x, n_work - 1));   // after the last item: a harmless reload
    lds_fft<ELEMS, THREADS>(buf, log2P, nz, +1.0, T.twiddle, twr);
    const double bd = b0[2 * wk.inst];
    const double inv_b0 = bd > 0.0 ? 1.0 / bd : 0.0;
    const double* ic = T.inv_corr + (P - 64);
    float* o = out + d.img_off + (int64_t)y0 * P;
    // Output phase with a fixed number of rounds: when the item holds fewer pixels (P < 128)
    // the extra rounds repeat earlier ones with identical values.  All correction factors are
    // loaded before the first store and every store is unconditional, so no load here waits
    // behind a store and the next item's staging waits only for its own prefetch (the vector
    // memory counter completes in order and counts stores too).
    constexpr int NRD = ELEMS / 4 / THREADS;
    const int nq4 = nz * P / 4;                                    // a power of two
    double cx[NRD][4], cy[NRD][2];
#pragma unroll
    for (int rd = 0; rd < NRD; ++rd) {
      const int q = 4 * ((threadIdx.x + rd * THREADS) & (nq4 - 1));
      const int x = q & (P - 1), y = y0 + 2 * (q >> log2P);
      cy[rd][0] = ic[y];
      cy[rd][1] = ic[y + 1];
#pragma unroll
      for (int e = 0; e < 4; ++e) cx[rd][e] = ic[x + e];
    }
#pragma unroll
    for (int rd = 0; rd < NRD; ++rd) {   // pixels x .. x + 3 of rows y0 + 2 zl, + 1
      const int q = 4 * ((threadIdx.x + rd * THREADS) & (nq4 - 1));
      const int zl = q >> log2P, x = q & (P - 1);
      const int y = y0 + 2 * zl;
      const double ry = cy[rd][0] * inv_b0, ry1 = cy[rd][1] * inv_b0;
      float fa[4], fb[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        double s0 = cx[rd][e] * ry, s1 = cx[rd][e] * ry1;
        if ((x + e + y) & 1) s0 = -s0;
        else s1 = -s1;
        const double2 z = buf[pd(q + e)];
        fa[e] = (float)(z.x * s0);
        fb[e] = (float)(z.y * s1);
      }
      *reinterpret_cast<float4*>(o + ((2 * zl) << log2P) + x) = make_float4(fa[0], fa[1], fa[2], fa[3]);
      *reinterpret_cast<float4*>(o + ((2 * zl + 1) << log2P) + x) = make_float4(fb[0], fb[1], fb[2], fb[3]);
    }
    __syncthreads();
  }
}

// Fused gridding + pass A.  A workgroup owns one block of whole half-grid lines: it
// accumulates the block's gridded samples (7 x 7 prolate-spheroidal taps, FP64 LDS atomics)
// straight into the LDS lines, each tap already carrying the (-1)^(i+j) modulation,
// transforms along v and writes the block once in pass A's blocked layout, so the half grid never goes to HBM and
// back.  The block's entries are self-contained records (cells, offsets, weight, value)
// written by k_bin; work item w covers line block rec_block(w), whose entries are
// tstart[b] .. tstart[b] + tcount[b] - 1.
// Thread t of a round takes entry t / 7 and v tap t % 7 - 3 and adds that cell in each of
// the sample's seven lines: the seven threads of a sample touch seven consecutive cells of
// a line (different LDS banks).  The next work item's range and its first round of records
// are loaded into registers before the current transform, so their latency hides behind it.
// Only the fields the gridder uses are loaded (12 + 8 bytes): a loaded register that is
// never read is free for reuse at once, and overwriting it means waiting for the load, which
// turns the next item's prefetch into a stall.
struct RecRegs { int3 a; float2 b; };

__device__ __forceinline__ RecRegs load_rec(const GridRec* __restrict__ rec, int i) {
  const int* p = reinterpret_cast<const int*>(rec + i);
  RecRegs r;
  r.a = *reinterpret_cast<const int3*>(p);
  r.b = *reinterpret_cast<const float2*>(p + 4);
  return r;
}

template <bool REAL>
__device__ __forceinline__ void grid_rec(double2* buf, const double* tab, const RecRegs& r, int dv, int h, int first,
                                         int lines, int log2P) {
  const int cu = r.a.x >> 16, cv = (int)(short)(r.a.x & 0xffff);
  const int ou = ((r.a.y >> 8) & 0xff) - OS / 2, ov = (r.a.y & 0xff) - OS / 2;
  const double w = (double)__int_as_float(r.a.z);
  const double wr = w * (double)r.b.x, wim = w * (double)r.b.y;
  // the v tap and all seven u taps are read before any accumulation, so that the table
  // reads overlap instead of each one waiting behind the previous tap's LDS atomics (every
  // index lies in [0, TAB_LEN) for |ou|, |ov| <= OS / 2)
  const double tv = tab[dv * OS - ov + TAB_CENTRE];
  double tu[W];
#pragma unroll
  for (int k = 0; k < W; ++k) tu[k] = tab[(k - HALF_W) * OS - ou + TAB_CENTRE];
  const int j = cv + dv + h;
  // REAL: real line l is the real (l even) or imaginary (l odd) part of complex line l / 2
  double* row = reinterpret_cast<double*>(buf);
#pragma unroll
  for (int du = -HALF_W; du <= HALF_W; ++du) {
    const int kp = cu + du + h - 1, l = kp - first;
    if (l < 0 || l >= lines || kp > h - 1) continue;
    // the (-1)^(i + j) modulation of the transform (u index i = kp + 1) goes with each tap
    const double kk = ((kp + 1 + j) & 1) ? -(tu[du + HALF_W] * tv) : tu[du + HALF_W] * tv;
    if (REAL) {
      atomicAdd(row + 2 * pd(((l >> 1) << log2P) + j) + (l & 1), wr * kk);
    } else {
      double* a = row + 2 * pd((l << log2P) + j);
      atomicAdd(a, wr * kk);
      atomicAdd(a + 1, wim * kk);
    }
  }
}

// The line block (index of its record range) of work item w of a fused first pass: blocks
// are numbered instance by instance, the work list deals them out in another order.
template <int ELEMS, bool REAL>
__device__ __forceinline__ int rec_block(const InstDesc* __restrict__ inst, const FftWork* __restrict__ work, int w) {
  const FftWork wk = work[w];
  const InstDesc& d = inst[wk.inst];
  if (REAL) return d.blk_base_b + (wk.first >> ilog2(real_lines_per_block<ELEMS>(2 * d.N)));
  return d.blk_base_d + (wk.first >> ilog2(lines_per_block<ELEMS>(d.N)));
}

// One work item's gridding: round 0 from the prefetched registers, later rounds loaded here.
template <int THREADS, bool REAL>
__device__ __forceinline__ void grid_block(double2* buf, const double* tab, const GridRec* __restrict__ rec,
                                           const RecRegs& r0, int st, int cnt, int P, int first, int lines) {
  constexpr int PER = THREADS / W;
  const int h = P / 2, log2P = ilog2(P);
  const int eo = threadIdx.x / W, dv = threadIdx.x - eo * W - HALF_W;
  if (eo < PER && eo < cnt) grid_rec<REAL>(buf, tab, r0, dv, h, first, lines, log2P);
  for (int e = PER + eo; e - eo < cnt; e += PER)
    if (eo < PER && e < cnt) grid_rec<REAL>(buf, tab, load_rec(rec, st + e), dv, h, first, lines, log2P);
}

template <int ELEMS, int THREADS>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(FFT_WAVES_PER_EU(ELEMS))))
k_grid_fft_a(const InstDesc* __restrict__ inst, const FftWork* __restrict__ work, int n_work,
             const GridRec* __restrict__ rec, const int* __restrict__ tstart, const int* __restrict__ tcount,
             double2* grid, Tables T) {
  __shared__ double2 buf[LDS_PADDED(ELEMS)];
  __shared__ double tab[TAB_LEN];
  for (int t = threadIdx.x; t < TAB_LEN; t += THREADS) tab[t] = T.tab[t];
  constexpr int PER = THREADS / W;
  const int eo = threadIdx.x / W;
  int w = blockIdx.x;
  int st = 0, cnt = 0;
  RecRegs r0{};
  if (w < n_work) {
    const int bk = rec_block<ELEMS, false>(inst, work, w);
    st = tstart[bk];
    cnt = tcount[bk];
    if (eo < PER && eo < cnt) r0 = load_rec(rec, st + eo);
  }
  // settled once: every later item then waits for its prefetched records only, not for the
  // previous item's stores (the first item's path would otherwise decide the wait)
  __builtin_amdgcn_s_waitcnt(0);
  TwRegs<ELEMS, THREADS> twr;
  for (; w < n_work; w += gridDim.x) {
    const int wn = w + gridDim.x;
    const int bn = wn < n_work ? rec_block<ELEMS, false>(inst, work, wn) : 0;
    const int stn = wn < n_work ? tstart[bn] : 0, cntn = wn < n_work ? tcount[bn] : 0;
    const FftWork wk = work[w];
    const InstDesc d = inst[wk.inst];
    const int P = d.N, log2P = ilog2(P);
    const int nl = lines_per_block<ELEMS>(P), log2nl = ilog2(nl);
    const int n = nl * P;
    twr.ensure(log2P, T.twiddle);
    for (int q = threadIdx.x; q < n; q += THREADS) buf[pd(q)] = make_double2(0.0, 0.0);
    __syncthreads();
    grid_block<THREADS, false>(buf, tab, rec, r0, st, cnt, P, wk.first, nl);
    if (eo < PER && eo < cntn) r0 = load_rec(rec, stn + eo);       // the next item's first round
    st = stn;
    cnt = cntn;
    __syncthreads();
    lds_fft<ELEMS, THREADS>(buf, log2P, nl, +1.0, T.twiddle, twr);
    double2* blk = grid + d.gd_off + (int64_t)wk.first * P;
    // a fixed number of unconditional store rounds (n is a power of two; for P < 128 the
    // extra rounds repeat elements with identical values), so that the compiler can count
    // them and a later wait for an older load does not wait for these stores too
#pragma unroll
    for (int rd = 0; rd < ELEMS / THREADS; ++rd) {
      const int q = (threadIdx.x + rd * THREADS) & (n - 1);
      const int y = q >> log2nl, l = q & (nl - 1);
      blk[q] = buf[pd((l << log2P) + y)];
    }
    __syncthreads();
  }
}

// The beam's fused gridding + pass A: real lines accumulated two per complex LDS line, then
// the same transform and slot separation as k_fft_a_real.
template <int ELEMS, int THREADS>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(FFT_WAVES_PER_EU(ELEMS))))
k_grid_fft_a_real(const InstDesc* __restrict__ inst, const FftWork* __restrict__ work, int n_work,
                  const GridRec* __restrict__ rec, const int* __restrict__ tstart, const int* __restrict__ tcount,
                  double* grid, Tables T) {
  __shared__ double2 buf[LDS_PADDED(ELEMS)];
  __shared__ double tab[TAB_LEN];
  for (int t = threadIdx.x; t < TAB_LEN; t += THREADS) tab[t] = T.tab[t];
  constexpr int PER = THREADS / W;
  const int eo = threadIdx.x / W;
  int w = blockIdx.x;
  int st = 0, cnt = 0;
  RecRegs r0{};
  if (w < n_work) {
    const int bk = rec_block<ELEMS, true>(inst, work, w);
    st = tstart[bk];
    cnt = tcount[bk];
    if (eo < PER && eo < cnt) r0 = load_rec(rec, st + eo);
  }
  // settled once: every later item then waits for its prefetched records only, not for the
  // previous item's stores (the first item's path would otherwise decide the wait)
  __builtin_amdgcn_s_waitcnt(0);
  TwRegs<ELEMS, THREADS> twr;
  for (; w < n_work; w += gridDim.x) {
    const int wn = w + gridDim.x;
    const int bn = wn < n_work ? rec_block<ELEMS, true>(inst, work, wn) : 0;
    const int stn = wn < n_work ? tstart[bn] : 0, cntn = wn < n_work ? tcount[bn] : 0;
    const FftWork wk = work[w];
    const InstDesc d = inst[wk.inst];
    const int P = 2 * d.N, log2P = ilog2(P), h = P / 2;
    const int nr = real_lines_per_block<ELEMS>(P), log2nr = ilog2(nr), nc = nr / 2;
    const int n = nc * P;
    twr.ensure(log2P, T.twiddle);
    for (int q = threadIdx.x; q < n; q += THREADS) buf[pd(q)] = make_double2(0.0, 0.0);
    __syncthreads();
    grid_block<THREADS, true>(buf, tab, rec, r0, st, cnt, P, wk.first, nr);
    if (eo < PER && eo < cntn) r0 = load_rec(rec, stn + eo);
    st = stn;
    cnt = cntn;
    __syncthreads();
    lds_fft<ELEMS, THREADS>(buf, log2P, nc, +1.0, T.twiddle, twr);
    double2* o = reinterpret_cast<double2*>(grid + d.gb_off + (int64_t)wk.first * P);   // nr x P/2 complex
    const int log2nc = log2nr - 1;
    // fixed, unconditional store rounds as in k_grid_fft_a (nc h is a power of two)
#pragma unroll
    for (int rd = 0; rd < ELEMS / 2 / THREADS; ++rd) {   // slot sl of lines 2c and 2c + 1
      const int q = (threadIdx.x + rd * THREADS) & (nc * h - 1);
      const int sl = q >> log2nc, c = q & (nc - 1);
      const int row = c << log2P;
      const double2 Z = buf[pd(row + sl)];
      double2 ya, yb;
      if (sl == 0) {
        const double2 Zh = buf[pd(row + h)];
        ya = make_double2(Z.x, Zh.x);
        yb = make_double2(Z.y, Zh.y);
      } else {
        const double2 Zm = buf[pd(row + P - sl)];
        ya = make_double2(0.5 * (Z.x + Zm.x), 0.5 * (Z.y - Zm.y));
        yb = make_double2(0.5 * (Z.y + Zm.y), 0.5 * (Zm.x - Z.x));
      }
      o[(sl << log2nr) + 2 * c] = ya;
      o[(sl << log2nr) + 2 * c + 1] = yb;
    }
    __syncthreads();
  }
}

// The beam: its grid is real and even (w K at the samples and their mirrors), so
//  * each half-grid line g_k(v) is real, and its transform along v has Y_k(P - y) =
//    conj Y_k(y): rows y = 0..P/2 carry everything, and Y_k(0), Y_k(P/2) are real;
//  * the beam is point-symmetric about (P/2, P/2): B[P - y][x] = B[y][(P - x) mod P].
// Pass A packs two real lines into one complex FFT and stores, per line, P/2 complex
// slots (slot 0 = (Y(0), Y(P/2)), slot s = Y(s)) over the same footprint as its P real
// inputs; pass B transforms rows 0..P/2 only and writes each of them twice, at y and
// mirrored at P - y, so the stored beam is exactly symmetric.

// Beam pass A: real half-grid lines -> FFT along v of line pairs -> separated spectra,
// slots 0..P/2-1, blocked layout Yb[b][s][l] (complex, nr lines per block).
template <int ELEMS, int THREADS>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(FFT_WAVES_PER_EU(ELEMS))))
k_fft_a_real(const InstDesc* __restrict__ inst, const FftWork* __restrict__ work, int n_work, double* grid,
             Tables T) {
  __shared__ double2 buf[LDS_PADDED(ELEMS)];
  constexpr int NPT = ELEMS / THREADS / 2;       // pairs of consecutive v per thread
  double2 ra[NPT], rb[NPT];
  auto fetch = [&](int wi) {
    const FftWork wk = work[wi];
    const InstDesc d = inst[wk.inst];
    const int P = 2 * d.N, log2P = ilog2(P);
    const int nc = real_lines_per_block<ELEMS>(P) / 2;
    const double* blk = grid + d.gb_off + (int64_t)wk.first * P;     // nr real lines of P
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int q = threadIdx.x + i * THREADS;      // pair index: line pair c, v = 2 (q % (P/2))
      if (q < nc * P / 2) {
        const int c = q >> (log2P - 1), v = 2 * (q & (P / 2 - 1));
        const double2* a = reinterpret_cast<const double2*>(blk + ((int64_t)(2 * c) << log2P) + v);
        const double2 x = a[0], y = a[P / 2];
        ra[i] = make_double2(x.x, x.y);
        rb[i] = make_double2(y.x, y.y);
      }
    }
  };
  int w = blockIdx.x;
  if (w < n_work) fetch(w);
  TwRegs<ELEMS, THREADS> twr;
  for (; w < n_work; w += gridDim.x) {
    const FftWork wk = work[w];
    const InstDesc d = inst[wk.inst];
    const int P = 2 * d.N, log2P = ilog2(P), h = P / 2;
    const int nr = real_lines_per_block<ELEMS>(P), log2nr = ilog2(nr), nc = nr / 2;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int q = threadIdx.x + i * THREADS;
      if (q < nc * P / 2) {
        buf[pd(2 * q)] = make_double2(ra[i].x, rb[i].x);
        buf[pd(2 * q + 1)] = make_double2(ra[i].y, rb[i].y);
      }
    }
    twr.ensure(log2P, T.twiddle);
    __syncthreads();
    if (w + (int)gridDim.x < n_work) fetch(w + gridDim.x);
    lds_fft<ELEMS, THREADS>(buf, log2P, nc, +1.0, T.twiddle, twr);
    double2* o = reinterpret_cast<double2*>(grid + d.gb_off + (int64_t)wk.first * P);   // nr x P/2 complex
    const int log2nc = log2nr - 1;
    // fixed, unconditional store rounds as in k_grid_fft_a (nc h is a power of two)
#pragma unroll
    for (int rd = 0; rd < ELEMS / 2 / THREADS; ++rd) {   // slot sl of lines 2c and 2c + 1
      const int q = (threadIdx.x + rd * THREADS) & (nc * h - 1);
      const int sl = q >> log2nc, c = q & (nc - 1);
      const int row = c << log2P;
      const double2 Z = buf[pd(row + sl)];
      double2 ya, yb;
      if (sl == 0) {
        const double2 Zh = buf[pd(row + h)];
        ya = make_double2(Z.x, Zh.x);
        yb = make_double2(Z.y, Zh.y);
      } else {
        const double2 Zm = buf[pd(row + P - sl)];
        // first line (Z + conj Zm) / 2, second line -i (Z - conj Zm) / 2
        ya = make_double2(0.5 * (Z.x + Zm.x), 0.5 * (Z.y - Zm.y));
        yb = make_double2(0.5 * (Z.y + Zm.y), 0.5 * (Zm.x - Z.x));
      }
      o[(sl << log2nr) + 2 * c] = ya;
      o[(sl << log2nr) + 2 * c + 1] = yb;
    }
    __syncthreads();
  }
}

// Beam pass B: rows y0..y0+ny-1 (only those <= P/2) from the slots, Hermitian completion
// along u, FFT, real part, correction, normalisation; row y is stored at y and, for
// 0 < y < P/2, mirrored at P - y; the right half of row P/2 mirrors its left half.
template <int ELEMS, int THREADS>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(FFT_WAVES_PER_EU(ELEMS))))
k_fft_b_c2r_sym(const InstDesc* __restrict__ inst, const FftWork* __restrict__ work, int n_work,
                const double* __restrict__ grid, const double* __restrict__ b0, Tables T,
                float* __restrict__ out) {
  __shared__ double2 buf[LDS_PADDED(ELEMS)];
  constexpr int NPT = ELEMS / 2 / THREADS;
  double2 r1[NPT], r2[NPT];
  // As in k_fft_b_c2r, every global load and store below is unconditional (lanes without an
  // element of their own load or store duplicates), so that the compiler can count the
  // memory operations in flight instead of waiting for all of them.
  auto fetch = [&](int wi) {
    const FftWork wk = work[wi];
    const InstDesc d = inst[wk.inst];
    const int P = 2 * d.N, h = P / 2;
    const int nr = real_lines_per_block<ELEMS>(P), log2nr = ilog2(nr);
    const int nz = rows_per_block<ELEMS>(P) / 2, log2pb = ilog2(nz * nr);
    const double2* src = reinterpret_cast<const double2*>(grid + d.gb_off);
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int q = (threadIdx.x + i * THREADS) & (h * nz - 1);
      const int b = q >> log2pb, r = q & ((1 << log2pb) - 1);
      const int zl = r >> log2nr, l = r & (nr - 1);
      const int ya = wk.first + 2 * zl;
      const double2* e = src + (int64_t)b * nr * h + l;
      // ya and P/2 are even, so row P/2 always starts a pair (and is the last row); slot
      // row 0 holds rows 0 (real part) and P/2 (imaginary part).  The raw slots are kept:
      // selecting from them here would wait for the loads at once.
      const int a1 = ya < h ? ya * nr : 0, a2 = ya < h ? (ya + 1) * nr : 0;
      const double2 u1 = e[a1], u2 = e[a2];
      r1[i] = make_double2(u1.x, u1.y);
      r2[i] = make_double2(u2.x, u2.y);
    }
  };
  int w = blockIdx.x;
  if (w < n_work) fetch(w);
  __builtin_amdgcn_s_waitcnt(0);           // see k_fft_b_c2r
  TwRegs<ELEMS, THREADS> twr;
  for (; w < n_work; w += gridDim.x) {
    const FftWork wk = work[w];
    const InstDesc d = inst[wk.inst];
    const int P = 2 * d.N, log2P = ilog2(P), h = P / 2;
    const int nr = real_lines_per_block<ELEMS>(P), log2nr = ilog2(nr);
    const int ny = rows_per_block<ELEMS>(P), nz = ny / 2, log2pb = ilog2(nz * nr);
    const int y0 = wk.first;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int qi = threadIdx.x + i * THREADS, q = qi & (h * nz - 1);
      const int b = q >> log2pb, r = q & ((1 << log2pb) - 1);
      const int zl = r >> log2nr, l = r & (nr - 1);
      const int ya = y0 + 2 * zl;
      const double2 u1 = r1[i], u2 = r2[i];
      double2 v1 = u1, v2 = u2;            // rows ya, ya + 1
      if (ya == 0) v1.y = 0.0;             // rows 0 and 1
      if (ya >= h) {                       // row P/2 alone, or past it
        v1 = make_double2(ya == h ? u1.y : 0.0, 0.0);
        v2 = make_double2(0.0, 0.0);
      }
      const int k = b * nr + l + 1;        // u frequency index 1..P/2
      const int row = zl << log2P;
      // u = 0 column (k = P/2): real by symmetry
      const double2 za = k < h ? make_double2(v1.x - v2.y, v1.y + v2.x) : make_double2(v1.x, v2.x);
      const double2 zb = make_double2(v1.x + v2.y, v2.x - v1.y);
      if (qi < h * nz) {
        buf[pd(row + k)] = za;
        if (k < h) buf[pd(row + P - k)] = zb;
      }
    }
    for (int zl = threadIdx.x; zl < nz; zl += THREADS) buf[pd(zl << log2P)] = make_double2(0.0, 0.0);
    twr.ensure(log2P, T.twiddle);
    __syncthreads();
    fetch(min(w + (int)gridDim.x, n_work - 1));   // after the last item: a harmless reload
    lds_fft<ELEMS, THREADS>(buf, log2P, nz, +1.0, T.twiddle, twr);
    const double bd = b0[2 * wk.inst + 1];
    const double inv_b0 = bd > 0.0 ? 1.0 / bd : 0.0;
    const double* ic = T.inv_corr + (P - 64);
    float* o = out + d.beam_off;
    // Output rounds: pixels x, x + 1 of rows ya, ya + 1 (ya <= P/2).  The item's npair row
    // pairs (nz, or 1 for the item holding row P/2 alone) make npair P/2 pixel pairs, a
    // power of two; a fixed number of rounds covers them, the extra rounds repeating
    // earlier ones.  All correction factors are loaded before the first store.
    constexpr int NRD = ELEMS / 2 / THREADS;
    const int npair = (min(ny, h + 1 - y0) + 1) / 2;
    const int nq2 = npair * P / 2;
    double cx[NRD][2], cy[NRD][2];
#pragma unroll
    for (int rd = 0; rd < NRD; ++rd) {
      const int q = 2 * ((threadIdx.x + rd * THREADS) & (nq2 - 1));
      const int x = q & (P - 1), ya = y0 + 2 * (q >> log2P);
#pragma unroll
      for (int e = 0; e < 2; ++e) {        // row P/2: its right half from the left half
        const int xs = (ya == h && x + e > h) ? P - x - e : x + e;
        cx[rd][e] = ic[xs];
      }
      cy[rd][0] = ic[ya];
      cy[rd][1] = ic[ya + 1];
    }
#pragma unroll
    for (int rd = 0; rd < NRD; ++rd) {
      const int q = 2 * ((threadIdx.x + rd * THREADS) & (nq2 - 1));
      const int zl = q >> log2P, x = q & (P - 1);
      const int ya = y0 + 2 * zl;
      const int row = zl << log2P;
      const bool mid = ya == h;            // row P/2 alone: no second row, no mirror row
      const double ra = cy[rd][0] * inv_b0, rb = cy[rd][1] * inv_b0;
      float fa[2], fb[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int xs = (mid && x + e > h) ? P - x - e : x + e;
        double sa = cx[rd][e] * ra, sb = cx[rd][e] * rb;
        if ((xs + ya) & 1) sa = -sa;
        else sb = -sb;
        const double2 z = buf[pd(row + xs)];
        fa[e] = (float)(z.x * sa);
        fb[e] = mid ? fa[e] : (float)(z.y * sb);
      }
      // stores: row ya; row ya + 1 (row P/2: row P/2 again, same values); the mirror of row
      // ya at P - ya (row 0: itself, same values) and of row ya + 1 at P - ya - 1 (row P/2:
      // the mirrored half of row P/2, whose values equal those of its left half)
      const int yb = mid ? ya : ya + 1;
      *reinterpret_cast<float2*>(o + (ya << log2P) + x) = make_float2(fa[0], fa[1]);
      *reinterpret_cast<float2*>(o + (yb << log2P) + x) = make_float2(fb[0], fb[1]);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int xm = (P - x - e) & (P - 1);
        if (ya > 0) o[((P - ya) << log2P) + xm] = fa[e];
        else o[x + e] = fa[e];
        o[((P - yb) << log2P) + xm] = fb[e];
      }
    }
    __syncthreads();
  }
}

// Adjoint pass B^T: image rows -> pre-correction and (-1)^(x+y) -> forward FFT along x ->
// keep u frequencies 1..P/2 -> blocked layout.  Two real rows per complex line, separated
// after the transform by X1 = (Z[k] + conj Z[-k]) / 2, X2 = (Z[k] - conj Z[-k]) / 2i.
// Persistent with the next item's image rows prefetched into registers, like the inverse.
template <int ELEMS, int THREADS>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(FFT_WAVES_PER_EU(ELEMS))))
k_fft_b_r2c(const InstDesc* __restrict__ inst, const FftWork* __restrict__ work, int n_work,
            const float* __restrict__ img, Tables T, double2* __restrict__ yb) {
  __shared__ double2 buf[LDS_PADDED(ELEMS)];
  constexpr int NPT = ELEMS / THREADS;
  float ra[NPT], rb[NPT];
  auto fetch = [&](int wi) {
    const FftWork wk = work[wi];
    const InstDesc d = inst[wk.inst];
    const int P = d.N, log2P = ilog2(P);
    const int nz = rows_per_block<ELEMS>(P) / 2;
    const float* src = img + d.img_off + (int64_t)wk.first * P;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int q = threadIdx.x + i * THREADS;
      if (q < nz * P) {
        const int zl = q >> log2P, x = q & (P - 1);
        const float* r0 = src + ((int64_t)(2 * zl) << log2P) + x;
        ra[i] = r0[0];
        rb[i] = r0[P];
      }
    }
  };
  int w = blockIdx.x;
  if (w < n_work) fetch(w);
  TwRegs<ELEMS, THREADS> twr;
  for (; w < n_work; w += gridDim.x) {
    const FftWork wk = work[w];
    const InstDesc d = inst[wk.inst];
    const int P = d.N, log2P = ilog2(P), h = P / 2;
    const int nl = lines_per_block<ELEMS>(P), log2nl = ilog2(nl);
    const int ny = rows_per_block<ELEMS>(P), nz = ny / 2;
    const int y0 = wk.first;
    const double* ic = T.inv_corr + (P - 64);
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int q = threadIdx.x + i * THREADS;
      if (q < nz * P) {
        const int zl = q >> log2P, x = q & (P - 1);
        const int y = y0 + 2 * zl;
        double s = ic[x] * ic[y], s2 = ic[x] * ic[y + 1];
        if ((x + y) & 1) s = -s;
        else s2 = -s2;
        buf[pd(q)] = make_double2((double)ra[i] * s, (double)rb[i] * s2);
      }
    }
    twr.ensure(log2P, T.twiddle);
    __syncthreads();
    if (w + (int)gridDim.x < n_work) fetch(w + gridDim.x);
    lds_fft<ELEMS, THREADS>(buf, log2P, nz, -1.0, T.twiddle, twr);
    double2* dst = yb + d.gd_off;
    const int nblk = h / nl, per_blk = nz * nl, log2pb = ilog2(per_blk);   // powers of two
    for (int q = threadIdx.x; q < nblk * per_blk; q += THREADS) {
      const int b = q >> log2pb, r = q & (per_blk - 1);
      const int zl = r >> log2nl, l = r & (nl - 1);
      const int k = b * nl + l + 1;
      const double2 A = buf[pd((zl << log2P) + k)];
      const double2 B = buf[pd((zl << log2P) + ((P - k) & (P - 1)))];
      // X1 = (A + conj B) / 2,  X2 = -i (A - conj B) / 2
      const double2 x1 = make_double2(0.5 * (A.x + B.x), 0.5 * (A.y - B.y));
      const double2 x2 = make_double2(0.5 * (A.y + B.y), -0.5 * (A.x - B.x));
      const int64_t e = (int64_t)b * nl * P + (int64_t)(y0 + 2 * zl) * nl + l;
      dst[e] = x1;
      dst[e + nl] = x2;
    }
    __syncthreads();
  }
}

// Adjoint pass A^T: blocked layout -> forward FFT along v -> (-1)^(i+j) -> half grid lines.
// Persistent; half of the next item is prefetched (within 128 VGPRs), as in pass A.
template <int ELEMS, int THREADS>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(FFT_WAVES_PER_EU(ELEMS))))
k_fft_a_fwd(const InstDesc* __restrict__ inst, const FftWork* __restrict__ work, int n_work, Tables T,
            double2* grid) {
  __shared__ double2 buf[LDS_PADDED(ELEMS)];
  constexpr int NPT = ELEMS / THREADS;
  constexpr int NPF = NPT / 2;
  double2 r[NPF];
  auto fetch = [&](int wi) {
    const FftWork wk = work[wi];
    const InstDesc d = inst[wk.inst];
    const int P = d.N, n = lines_per_block<ELEMS>(P) * P;
    const double2* blk = grid + d.gd_off + (int64_t)wk.first * P;
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      const int q = threadIdx.x + i * THREADS;
      if (q < n) {
        const double2 v = blk[q];
        r[i] = make_double2(v.x, v.y);   // component copy keeps r[] in registers
      }
    }
  };
  int w = blockIdx.x;
  if (w < n_work) fetch(w);
  TwRegs<ELEMS, THREADS> twr;
  for (; w < n_work; w += gridDim.x) {
    const FftWork wk = work[w];
    const InstDesc d = inst[wk.inst];
    const int P = d.N, log2P = ilog2(P);
    const int nl = lines_per_block<ELEMS>(P), log2nl = ilog2(nl);
    const int n = nl * P;
    double2* blk = grid + d.gd_off + (int64_t)wk.first * P;
#pragma unroll
    for (int i = NPF; i < NPT; ++i) {
      const int q = threadIdx.x + i * THREADS;
      if (q < n) buf[pd(((q & (nl - 1)) << log2P) + (q >> log2nl))] = blk[q];
    }
#pragma unroll
    for (int i = 0; i < NPF; ++i) {
      const int q = threadIdx.x + i * THREADS;
      if (q < n) buf[pd(((q & (nl - 1)) << log2P) + (q >> log2nl))] = r[i];
    }
    twr.ensure(log2P, T.twiddle);
    __syncthreads();
    if (w + (int)gridDim.x < n_work) fetch(w + gridDim.x);
    lds_fft<ELEMS, THREADS>(buf, log2P, nl, -1.0, T.twiddle, twr);
    for (int q = threadIdx.x; q < n; q += THREADS) {
      const int l = q >> log2P, j = q & (P - 1);
      double2 v = buf[pd(q)];
      if (((wk.first + l + 1) + j) & 1) { v.x = -v.x; v.y = -v.y; }
      blk[q] = v;
    }
    __syncthreads();
  }
}

// Generic complex lines -> FFT -> transposed write, for mi_ifft2 (two passes).
// src lines of length P (stride P), nl lines per block; dst[y * P + line].
// pre: multiply input (line, n) by (-1)^(line+n); post: output (y, line) by (-1)^(y+line).
template <int ELEMS, int THREADS, class TIn, class TOut>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(FFT_WAVES_PER_EU(ELEMS))))
k_fft_c2c_t(const int* __restrict__ n_arr, const int64_t* __restrict__ offs, const FftWork* __restrict__ work,
            const TIn* __restrict__ src, TOut* __restrict__ dst, Tables T, double s, int pre, int post) {
  __shared__ double2 buf[LDS_PADDED(ELEMS)];
  const FftWork wk = work[blockIdx.x];
  const int P = n_arr[wk.inst], log2P = ilog2(P);
  int nl = ELEMS / P;
  if (nl > P) nl = P;
  const int log2nl = ilog2(nl);
  const int64_t off = offs[wk.inst];
  const TIn* in = src + off + (int64_t)wk.first * P;
  const int n = nl * P;
  // staging in fixed rounds (n <= ELEMS, a power of two), every load issued before the first
  // LDS write (lanes past n load a duplicate, unused): one wait instead of one round trip per
  // element
  constexpr int NPT = ELEMS / THREADS;
  TIn v[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) v[k] = in[(threadIdx.x + k * THREADS) & (n - 1)];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int q = threadIdx.x + k * THREADS;
    if (q >= n) continue;
    double2 d = make_double2((double)v[k].x, (double)v[k].y);
    if (pre && (((q >> log2P) + wk.first + (q & (P - 1))) & 1)) { d.x = -d.x; d.y = -d.y; }
    buf[pd(q)] = d;
  }
  __syncthreads();
  lds_fft<ELEMS, THREADS>(buf, log2P, nl, s, T.twiddle);
  TOut* out = dst + off;
  for (int q = threadIdx.x; q < n; q += THREADS) {
    const int y = q >> log2nl, l = q & (nl - 1);
    double2 v = buf[pd((l << log2P) + y)];
    const int line = wk.first + l;
    if (post && ((y + line) & 1)) { v.x = -v.x; v.y = -v.y; }
    TOut o;
    o.x = v.x;
    o.y = v.y;
    out[(int64_t)y * P + line] = o;
  }
}

// ---- host launchers.  elems selects the LDS block: 4096 complex doubles (72 KB with
// padding, 512 threads, two workgroups per CU) or 8192 (144 KB, 512 threads, needed only
// for P = 8192).

// Persistent passes: as many workgroups as are resident at once (or fewer items).
template <class Kern>
int resident_grid(Kern k, int threads, int n_work, int n_cu) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  return std::min(n_work, per_cu * n_cu);
}
#define MI_FFT_PERSISTENT(KERNEL, ...)                                                                    \
  do {                                                                                                    \
    if (elems == 8192)                                                                                    \
      hipLaunchKernelGGL((KERNEL<8192, 512>), dim3(resident_grid(KERNEL<8192, 512>, 512, n_work, n_cu)),  \
                         dim3(512), 0, st, __VA_ARGS__);                                                  \
    else                                                                                                  \
      hipLaunchKernelGGL((KERNEL<4096, 512>), dim3(resident_grid(KERNEL<4096, 512>, 512, n_work, n_cu)),  \
                         dim3(512), 0, st, __VA_ARGS__);                                                  \
  } while (0)

hipError_t launch_fft_a(int elems, int n_cu, const InstDesc* inst, const FftWork* work, int n_work, double2* grid,
                        const Tables& T, hipStream_t st) {
  if (n_work <= 0) return hipSuccess;
  MI_FFT_PERSISTENT(k_fft_a, inst, work, n_work, grid, T);
  return hipGetLastError();
}
hipError_t launch_grid_fft_a(int elems, int n_cu, const InstDesc* inst, const FftWork* work, int n_work,
                             const GridRec* rec, const int* tstart, const int* tcount, double2* grid, const Tables& T,
                             hipStream_t st) {
  if (n_work <= 0) return hipSuccess;
  MI_FFT_PERSISTENT(k_grid_fft_a, inst, work, n_work, rec, tstart, tcount, grid, T);
  return hipGetLastError();
}
hipError_t launch_grid_fft_a_real(int elems, int n_cu, const InstDesc* inst, const FftWork* work, int n_work,
                                  const GridRec* rec, const int* tstart, const int* tcount, double* grid,
                                  const Tables& T, hipStream_t st) {
  if (n_work <= 0) return hipSuccess;
  MI_FFT_PERSISTENT(k_grid_fft_a_real, inst, work, n_work, rec, tstart, tcount, grid, T);
  return hipGetLastError();
}
hipError_t launch_fft_b_c2r(int elems, int n_cu, const InstDesc* inst, const FftWork* work, int n_work,
                            const double2* yb, const double* b0, const Tables& T, float* out, hipStream_t st) {
  if (n_work <= 0) return hipSuccess;
  MI_FFT_PERSISTENT(k_fft_b_c2r, inst, work, n_work, yb, b0, T, out);
  return hipGetLastError();
}
hipError_t launch_fft_a_real(int elems, int n_cu, const InstDesc* inst, const FftWork* work, int n_work,
                             double* grid, const Tables& T, hipStream_t st) {
  if (n_work <= 0) return hipSuccess;
  MI_FFT_PERSISTENT(k_fft_a_real, inst, work, n_work, grid, T);
  return hipGetLastError();
}
hipError_t launch_fft_b_c2r_sym(int elems, int n_cu, const InstDesc* inst, const FftWork* work, int n_work,
                                const double* grid, const double* b0, const Tables& T, float* out, hipStream_t st) {
  if (n_work <= 0) return hipSuccess;
  MI_FFT_PERSISTENT(k_fft_b_c2r_sym, inst, work, n_work, grid, b0, T, out);
  return hipGetLastError();
}
hipError_t launch_fft_b_r2c(int elems, int n_cu, const InstDesc* inst, const FftWork* work, int n_work,
                            const float* img, const Tables& T, double2* yb, hipStream_t st) {
  if (n_work <= 0) return hipSuccess;
  MI_FFT_PERSISTENT(k_fft_b_r2c, inst, work, n_work, img, T, yb);
  return hipGetLastError();
}
hipError_t launch_fft_a_fwd(int elems, int n_cu, const InstDesc* inst, const FftWork* work, int n_work,
                            const Tables& T, double2* grid, hipStream_t st) {
  if (n_work <= 0) return hipSuccess;
  MI_FFT_PERSISTENT(k_fft_a_fwd, inst, work, n_work, T, grid);
  return hipGetLastError();
}
hipError_t launch_fft_c2c_t_f2d(int elems, const int* n_arr, const int64_t* offs, const FftWork* work, int n_work,
                                const float2* src, double2* dst, const Tables& T, double s, int pre, int post,
                                hipStream_t st) {
  if (n_work <= 0) return hipSuccess;
  if (elems == 8192)
    hipLaunchKernelGGL((k_fft_c2c_t<8192, 512, float2, double2>), dim3(n_work), dim3(512), 0, st, n_arr, offs, work,
                       src, dst, T, s, pre, post);
  else
    hipLaunchKernelGGL((k_fft_c2c_t<4096, 512, float2, double2>), dim3(n_work), dim3(512), 0, st, n_arr, offs, work,
                       src, dst, T, s, pre, post);
  return hipGetLastError();
}
hipError_t launch_fft_c2c_t_d2d(int elems, const int* n_arr, const int64_t* offs, const FftWork* work, int n_work,
                                const double2* src, double2* dst, const Tables& T, double s, int pre, int post,
                                hipStream_t st) {
  if (n_work <= 0) return hipSuccess;
  if (elems == 8192)
    hipLaunchKernelGGL((k_fft_c2c_t<8192, 512, double2, double2>), dim3(n_work), dim3(512), 0, st, n_arr, offs, work,
                       src, dst, T, s, pre, post);
  else
    hipLaunchKernelGGL((k_fft_c2c_t<4096, 512, double2, double2>), dim3(n_work), dim3(512), 0, st, n_arr, offs, work,
                       src, dst, T, s, pre, post);
  return hipGetLastError();
}
hipError_t launch_fft_c2c_t_d2f(int elems, const int* n_arr, const int64_t* offs, const FftWork* work, int n_work,
                                const double2* src, float2* dst, const Tables& T, double s, int pre, int post,
                                hipStream_t st) {
  if (n_work <= 0) return hipSuccess;
  if (elems == 8192)
    hipLaunchKernelGGL((k_fft_c2c_t<8192, 512, double2, float2>), dim3(n_work), dim3(512), 0, st, n_arr, offs, work,
                       src, dst, T, s, pre, post);
  else
    hipLaunchKernelGGL((k_fft_c2c_t<4096, 512, double2, float2>), dim3(n_work), dim3(512), 0, st, n_arr, offs, work,
                       src, dst, T, s, pre, post);
  return hipGetLastError();
}

}  // namespace mi
