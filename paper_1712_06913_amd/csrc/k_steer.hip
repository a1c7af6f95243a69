// Steer CLEAN (gfx950): the Steer-Dewdney-Ito CLEAN that the paper names as MUSER's
// deconvolver (Sec. 2; Sec. 4.3; Algorithm 1's improved_clean runs it with the loop gain
// 0.1 until the peak reaches the sky level).  One iteration of an image:
//   peak = max |R| (max R for positive-only), stop if peak <= threshold;
//   C = R on the pixels with |R| >= trim peak (R >= trim peak), 0 elsewhere;
//   D = C convolved with the dirty beam (linear: D[y][x] = sum_q C[q] B[y - q_y + N][x - q_x + N]);
//   alpha = gain peak / max |D|;  model += alpha C;  R -= alpha D.
//
// The convolution is a 2N x 2N circular one, which equals the linear one on the cropped
// rows and columns N..2N-1 (no index wraps there), computed by FP32 FFTs in LDS with
// twiddles computed in FP64 and rounded once; the spectra go between the passes as FP32.
// There is no grid correction here to amplify rounding: the FP32 transforms put an error of
// about 1e-7 of max |D| into D, so alpha D, whose largest value is gain x peak, is off by
// about 1e-8 of the peak per iteration, against the 1e-5 x peak to which each selection is
// checked and the 1e-4 x peak of the maps:
//   k_st_rows     real rows of C (N nonzero of 2N) -> row spectra, two rows per complex
//                 FFT, kx = 0..N kept (Hermitian), written as blocks of RB rows;
//   k_st_cols     per column kx: FFT along y, times the beam spectrum, inverse FFT, rows
//                 N..2N-1 written back over the column's inputs;
//   k_st_rows_inv per row: Hermitian completion, inverse FFT, columns N..2N-1 = D, max |D|;
//   k_st_update   alpha, the model and residual updates, the next peak.
// The beam spectrum is made once per call by the same row and column passes, and the
// restore (model convolved with the fitted clean-beam Gaussian, plus R) reuses all three.
// Every image of the batch advances in lockstep, one launch per pass and iteration; an
// image that has stopped (iteration cap, peak at the threshold, or D = 0) skips its work.
//
// Control words per image (zeroed before the first launch): peak keys of iterations with
// even / odd index, the max |D| key, and the count of selected pixels per iteration.  Keys
// are order-preserving 32-bit images of float values, 0 meaning "none": iteration k's rows
// pass clears the key that iteration k's update will fill (it last held iteration k - 1's
// peak, read by then) and the max |D| key.
#include <type_traits>

#include "mi_internal.h"
#include "fft_lds.h"

namespace mi {

constexpr int ST_THREADS = 512;
// Complex floats staged per workgroup: 4096 (36 KB with padding; at 72 VGPRs three
// workgroups share a compute unit) for transforms up to 4096 points, 8192 (72 KB) for
// 8192-point ones (N = 4096).
constexpr int st_lds(int elems) { return elems + elems / 8; }

namespace {

__device__ __forceinline__ unsigned fkey(float v) {
  const unsigned b = __float_as_uint(v);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float fkey_val(unsigned k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__device__ __forceinline__ unsigned wave_max(unsigned v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, o));
  return v;
}

// Block-wide maximum of a key, then one atomic per block.
__device__ __forceinline__ void block_atomic_max(unsigned v, unsigned* sh, unsigned* dst) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned m = 0u;
    for (int w = 0; w < ST_THREADS / 64; ++w) m = max(m, sh[w]);
    if (m) atomicMax(dst, m);
  }
}

// Whether image i takes part in iteration k (and its peak if it does).
__device__ __forceinline__ bool st_active(const SteerArgs& A, const SteerInst& s, int i, float& peak) {
  if (A.k >= s.ncycle) return false;
  const unsigned key = A.ctl[s.ctl_off + (A.k & 1)];
  if (key == 0u) return false;
  peak = fkey_val(key);
  const float thr = A.thr_dev ? A.thr_dev[i] : s.thr;
  return peak > thr;
}

// The selection test, the same arithmetic in the rows and the update pass.
__device__ __forceinline__ bool st_sel(float v, double tp, int posonly) {
  return posonly ? (double)v >= tp : (double)fabsf(v) >= tp;
}

}  // namespace

// Forward row transforms of RB rows (RB/2 complex lines of P = 2N points).
//   MODE 0: C = the selected residual pixels (rows of N, padded), iteration launches;
//   MODE 1: the model (rows of N, padded);
//   MODE 2: the dirty beam (2N rows of 2N);
//   MODE 3: the clean-beam Gaussian exp(-(a dx^2 + b dx dy + c dy^2)) at dx = x - N,
//           dy = y - N (2N rows of 2N).
template <int MODE, int ST_ELEMS>
__global__ void __launch_bounds__(ST_THREADS) k_st_rows(SteerArgs A) {
  __shared__ float2 buf[st_lds(ST_ELEMS)];
  __shared__ unsigned n_sel;
  const FftWork wk = A.work[blockIdx.x];
  const int i = wk.inst;
  const InstDesc d = A.inst[i];
  const SteerInst s = A.sti[i];
  const int N = d.N, P = 2 * N, log2P = d.log2N + 1, RB = s.rb, nl = RB / 2;
  TwRegs<ST_ELEMS, ST_THREADS> twr;               // issued before the data loads, waited for with them
  twr.load(log2P, A.T.twiddle);
  const int y0 = wk.first;
  double tp = 0.0;
  if (MODE == 0) {
    if (y0 == 0 && threadIdx.x == 0) {
      A.ctl[s.ctl_off + ((A.k + 1) & 1)] = 0u;     // filled by this iteration's update
      A.ctl[s.ctl_off + 2] = 0u;                   // filled by this iteration's rows_inv
    }
    float peak;
    if (!st_active(A, s, i, peak)) return;
    tp = (double)A.trim * (double)peak;
    if (threadIdx.x == 0) n_sel = 0u;
    __syncthreads();
  }
  const int Lin = (MODE <= 1) ? N : P;
  double ga = 0.0, gb = 0.0, gc = 0.0;
  if (MODE == 3) {
    ga = A.cbeam[6 * i + 0];
    gb = A.cbeam[6 * i + 1];
    gc = A.cbeam[6 * i + 2];
  }
  unsigned cnt = 0u;
  // staging in fixed rounds (nl P <= ST_ELEMS), all loads first and then the LDS writes: one
  // wait per thread instead of one memory round trip per element
  constexpr int NPT = ST_ELEMS / ST_THREADS;
  using LT = typename std::conditional<MODE == 1, double, float>::type;
  LT ld[NPT][2];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int q = threadIdx.x + k * ST_THREADS;
    const int l = q >> log2P, x = q & (P - 1);
    const bool in = q < nl * P && x < Lin;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int y = y0 + 2 * l + h;
      if (MODE == 0) ld[k][h] = in ? A.R[d.img_off + (int64_t)y * N + x] : 0.0f;
      else if (MODE == 1) ld[k][h] = in ? A.model[d.img_off + (int64_t)y * N + x] : 0.0;
      else if (MODE == 2) ld[k][h] = in ? A.beam[d.beam_off + (int64_t)y * P + x] : 0.0f;
      else ld[k][h] = 0;
    }
  }
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int q = threadIdx.x + k * ST_THREADS;
    if (q >= nl * P) continue;
    const int l = q >> log2P, x = q & (P - 1);
    double v[2] = {0.0, 0.0};
    if (x < Lin) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int y = y0 + 2 * l + h;
        if (MODE == 0) {
          const float r = ld[k][h];
          const bool sel = st_sel(r, tp, A.posonly);
          cnt += sel ? 1u : 0u;
          v[h] = sel ? (double)r : 0.0;
        } else if (MODE == 1 || MODE == 2) {
          v[h] = (double)ld[k][h];
        } else {
          const double dx = (double)(x - N), dy = (double)(y - N);
          v[h] = exp(-(dx * (ga * dx + gb * dy) + gc * dy * dy));
        }
      }
    }
    buf[pd(q)] = make_float2((float)v[0], (float)v[1]);
  }
  if (MODE == 0) {
    for (int o = 32; o > 0; o >>= 1) cnt += (unsigned)__shfl_xor((int)cnt, o);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(&n_sel, cnt);
  }
  __syncthreads();
  if (MODE == 0 && threadIdx.x == 0 && n_sel) atomicAdd(&A.ctl[s.ctl_off + 4 + A.k], n_sel);
  lds_fft<ST_ELEMS, ST_THREADS>(buf, log2P, nl, -1.0, A.T.twiddle, twr);
  // separate the two rows of each line: Xa = (Z(k) + conj Z(P-k)) / 2, Xb = (Z(k) - conj Z(P-k)) / 2i
  const int log2RB = __builtin_ctz(RB);
  float2* out = A.X + s.x_off + (int64_t)(y0 >> log2RB) * (N + 1) * RB;
  for (int q = threadIdx.x; q < (N + 1) * RB; q += ST_THREADS) {
    const int kx = q >> log2RB, r = q & (RB - 1), l = r >> 1;
    const float2 Z = buf[pd(l * P + kx)];
    const float2 Zm = buf[pd(l * P + ((P - kx) & (P - 1)))];
    out[q] = (r & 1) ? make_float2(0.5f * (Z.y + Zm.y), 0.5f * (Zm.x - Z.x))
                     : make_float2(0.5f * (Z.x + Zm.x), 0.5f * (Z.y - Zm.y));
  }
}

// Column transforms of up to ST_ELEMS / P columns kx0.. of the blocked row spectra.
//   MODE 0: the spectrum of a 2N-row image: FFT along y, scaled by 1/P^2, stored column by
//           column in S;
//   MODE 1: convolution: rows 0..N-1 (the rest is zero), FFT, times S, inverse FFT, rows
//           N..2N-1 written back over rows 0..N-1 of the same columns.
template <int MODE, int ST_ELEMS>
__global__ void __launch_bounds__(ST_THREADS) k_st_cols(SteerArgs A) {
  __shared__ float2 buf[st_lds(ST_ELEMS)];
  const FftWork wk = A.work[blockIdx.x];
  const int i = wk.inst;
  const InstDesc d = A.inst[i];
  const SteerInst s = A.sti[i];
  if (A.iter) {
    float peak;
    if (!st_active(A, s, i, peak)) return;
  }
  const int N = d.N, P = 2 * N, log2P = d.log2N + 1, RB = s.rb, log2RB = __builtin_ctz(RB);
  TwRegs<ST_ELEMS, ST_THREADS> twr;               // issued before the data loads, waited for with them
  twr.load(log2P, A.T.twiddle);
  const int kx0 = wk.first;
  const int nc = min(ST_ELEMS >> log2P, N + 1 - kx0);
  const int Rin = MODE == 0 ? P : N;
  float2* X = A.X + s.x_off;
  // element q = (yb nc + c) RB + r: row yb RB + r of column kx0 + c; for each block of rows
  // the nc columns' entries are contiguous in memory.  nc is a power of two (the block's
  // column count, or 1 for the last column kx = N: N is a multiple of it), so q splits by
  // shifts
  const int run = nc * RB, log2run = __builtin_ctz(nc) + log2RB;
  // staging in fixed rounds (nc P <= ST_ELEMS elements), all loads before the LDS writes
  constexpr int NPT = ST_ELEMS / ST_THREADS;
  float2 sv[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int q = threadIdx.x + k * ST_THREADS;
    const int yb = q >> log2run, rem = q & (run - 1), c = rem >> log2RB, r = rem & (RB - 1);
    const int y = (yb << log2RB) + r;
    // an unconditional load (element 0 where nothing is read), then the selection: a load
    // under a lane condition would be waited for inside its branch
    const bool in = q < (P / RB) * run && y < Rin;
    const float2 t = X[in ? (int64_t)yb * (N + 1) * RB + (int64_t)(kx0 + c) * RB + r : 0];
    sv[k] = in ? t : make_float2(0.0f, 0.0f);
  }
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int q = threadIdx.x + k * ST_THREADS;
    const int yb = q >> log2run, rem = q & (run - 1), c = rem >> log2RB, r = rem & (RB - 1);
    if (q < (P / RB) * run) buf[pd((c << log2P) + (yb << log2RB) + r)] = sv[k];
  }
  __syncthreads();
  lds_fft<ST_ELEMS, ST_THREADS>(buf, log2P, nc, -1.0, A.T.twiddle, twr);
  float2* Sc = A.S + s.s_off + (int64_t)kx0 * P;
  if (MODE == 0) {
    const float sc = 1.0f / ((float)P * (float)P);     // a power of two: exact
    for (int q = threadIdx.x; q < nc * P; q += ST_THREADS) {
      const float2 v = buf[pd(q)];
      Sc[q] = make_float2(v.x * sc, v.y * sc);
    }
    return;
  }
  for (int q = threadIdx.x; q < nc * P; q += ST_THREADS) buf[pd(q)] = cmul(buf[pd(q)], Sc[q]);
  __syncthreads();
  lds_fft<ST_ELEMS, ST_THREADS>(buf, log2P, nc, +1.0, A.T.twiddle, twr);
  for (int q = threadIdx.x; q < (N / RB) * run; q += ST_THREADS) {
    const int yb = q >> log2run, rem = q & (run - 1), c = rem >> log2RB, r = rem & (RB - 1);
    const int y = (yb << log2RB) + r;
    X[(int64_t)yb * (N + 1) * RB + (int64_t)(kx0 + c) * RB + r] = buf[pd((c << log2P) + N + y)];
  }
}

// Inverse row transforms of RB rows j0.. of the convolution (complex-to-real, two rows per
// complex FFT), keeping columns N..2N-1.
//   MODE 0: D = the result, and its max |D| into the image's control word;
//   MODE 1: the restored image R + result.
template <int MODE, int ST_ELEMS>
__global__ void __launch_bounds__(ST_THREADS) k_st_rows_inv(SteerArgs A) {
  __shared__ float2 buf[st_lds(ST_ELEMS)];
  __shared__ unsigned red[ST_THREADS / 64];
  const FftWork wk = A.work[blockIdx.x];
  const int i = wk.inst;
  const InstDesc d = A.inst[i];
  const SteerInst s = A.sti[i];
  if (A.iter) {
    float peak;
    if (!st_active(A, s, i, peak)) return;
  }
  const int N = d.N, P = 2 * N, log2P = d.log2N + 1, RB = s.rb, nl = RB / 2, log2nl = __builtin_ctz(nl);
  TwRegs<ST_ELEMS, ST_THREADS> twr;               // issued before the data loads, waited for with them
  twr.load(log2P, A.T.twiddle);
  const int j0 = wk.first;
  const float2* in = A.X + s.x_off + (int64_t)(j0 / RB) * (N + 1) * RB;
  // staging in fixed rounds ((N + 1) nl <= ST_ELEMS / 2 + nl elements), all loads before
  // the LDS writes
  constexpr int NPT = ST_ELEMS / 2 / ST_THREADS + 1;
  float2 sa[NPT], sb[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int q = threadIdx.x + k * ST_THREADS;
    const int kx = q >> log2nl, l = q & (nl - 1);
    const bool ok = q < (N + 1) * nl;
    sa[k] = ok ? in[kx * RB + 2 * l] : make_float2(0.0f, 0.0f);
    sb[k] = ok ? in[kx * RB + 2 * l + 1] : make_float2(0.0f, 0.0f);
  }
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int q = threadIdx.x + k * ST_THREADS;
    if (q >= (N + 1) * nl) continue;
    const int kx = q >> log2nl, l = q & (nl - 1);
    float2 a = sa[k], b = sb[k];
    if (kx == 0 || kx == N) { a.y = 0.0f; b.y = 0.0f; }    // real by symmetry
    const int row = l << log2P;
    buf[pd(row + kx)] = make_float2(a.x - b.y, a.y + b.x);
    if (kx > 0 && kx < N) buf[pd(row + P - kx)] = make_float2(a.x + b.y, b.x - a.y);
  }
  __syncthreads();
  lds_fft<ST_ELEMS, ST_THREADS>(buf, log2P, nl, +1.0, A.T.twiddle, twr);
  unsigned m = 0u;
  const int log2N = d.log2N;
  for (int q = threadIdx.x; q < nl * N; q += ST_THREADS) {
    const int l = q >> log2N, x = q & (N - 1);
    const float2 z = buf[pd((l << log2P) + N + x)];
    const int64_t o = d.img_off + (int64_t)(j0 + 2 * l) * N + x;
    if (MODE == 0) {
      A.D[o] = z.x;
      A.D[o + N] = z.y;
      m = max(m, fkey(fmaxf(fabsf(z.x), fabsf(z.y))));
    } else {
      A.restored[o] = (float)((double)A.R[o] + z.x);
      A.restored[o + N] = (float)((double)A.R[o + N] + z.y);
    }
  }
  if (MODE == 0) block_atomic_max(m, red, &A.ctl[s.ctl_off + 2]);
}

// Residual initialisation: R = dirty, model = 0, the first peak.
__global__ void __launch_bounds__(ST_THREADS) k_st_init(SteerArgs A) {
  __shared__ unsigned red[ST_THREADS / 64];
  const FftWork wk = A.work[blockIdx.x];
  const int i = wk.inst;
  const InstDesc d = A.inst[i];
  const SteerInst s = A.sti[i];
  const int64_t n2 = (int64_t)d.N * d.N;
  const int64_t p = (int64_t)wk.first + 4 * threadIdx.x;
  if (wk.first == 0 && threadIdx.x == 0 && A.ncyc_out) A.ncyc_out[i] = 0;
  unsigned best = 0u;
  if (p < n2) {
    const float4 r = *reinterpret_cast<const float4*>(A.dirty + d.img_off + p);
    *reinterpret_cast<float4*>(A.R + d.img_off + p) = r;
    double* m = A.model + d.img_off + p;
    m[0] = m[1] = m[2] = m[3] = 0.0;
    const float v[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) best = max(best, fkey(A.posonly ? v[j] : fabsf(v[j])));
  }
  block_atomic_max(best, red, &A.ctl[s.ctl_off + 0]);
}

// Iteration update over 4 pixels per thread: alpha, model += alpha C, R -= alpha D, the
// selection bits (optional) and the next peak.
__global__ void __launch_bounds__(ST_THREADS) k_st_update(SteerArgs A) {
  __shared__ unsigned red[ST_THREADS / 64];
  const FftWork wk = A.work[blockIdx.x];
  const int i = wk.inst;
  const InstDesc d = A.inst[i];
  const SteerInst s = A.sti[i];
  float peak;
  if (!st_active(A, s, i, peak)) return;
  const float dmax = fkey_val(A.ctl[s.ctl_off + 2]);
  if (!(dmax > 0.0f)) return;                 // nothing to subtract: the image stops here
  const double alpha = (double)A.gain * (double)peak / (double)dmax;
  const double tp = (double)A.trim * (double)peak;
  const int64_t n2 = (int64_t)d.N * d.N;
  const int64_t p = (int64_t)wk.first + 4 * threadIdx.x;
  if (wk.first == 0 && threadIdx.x == 0) {
    if (A.log) {
      double* lg = A.log + s.log_off + 3 * (int64_t)A.k;
      lg[0] = (double)peak;
      lg[1] = alpha;
      lg[2] = (double)A.ctl[s.ctl_off + 4 + A.k];
    }
    if (A.ncyc_out) A.ncyc_out[i] = A.k + 1;
  }
  unsigned best = 0u, nib = 0u;
  if (p < n2) {
    float4* rp = reinterpret_cast<float4*>(A.R + d.img_off + p);
    const float4 r = *rp;
    const float4 dd = *reinterpret_cast<const float4*>(A.D + d.img_off + p);
    double* m = A.model + d.img_off + p;
    const float v[4] = {r.x, r.y, r.z, r.w};
    const float dv[4] = {dd.x, dd.y, dd.z, dd.w};
    float o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (st_sel(v[j], tp, A.posonly)) {
        m[j] += alpha * (double)v[j];
        nib |= 1u << j;
      }
      o[j] = (float)((double)v[j] - alpha * (double)dv[j]);
      best = max(best, fkey(A.posonly ? o[j] : fabsf(o[j])));
    }
    *rp = make_float4(o[0], o[1], o[2], o[3]);
  }
  if (A.mask) {
    // 8 threads x 4 pixels = one 32-bit word, bit b = pixel 32 w + b
    unsigned word = nib << (4 * (threadIdx.x & 7));
    word |= (unsigned)__shfl_xor((int)word, 1);
    word |= (unsigned)__shfl_xor((int)word, 2);
    word |= (unsigned)__shfl_xor((int)word, 4);
    if ((threadIdx.x & 7) == 0 && p < n2) A.mask[s.mask_off + (int64_t)A.k * (n2 >> 5) + (p >> 5)] = word;
  }
  block_atomic_max(best, red, &A.ctl[s.ctl_off + ((A.k + 1) & 1)]);
}

// ---- host launchers ----
static hipError_t st_launch(const void* k, int n_blocks, const SteerArgs& A, hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  SteerArgs a = A;
  void* args[] = {&a};
  return hipLaunchKernel(k, dim3(n_blocks), dim3(ST_THREADS), args, 0, st);
}

#define MI_ST_PICK(KERNEL, MODE) \
  (elems == 8192 ? reinterpret_cast<const void*>(&KERNEL<MODE, 8192>) : reinterpret_cast<const void*>(&KERNEL<MODE, 4096>))

hipError_t launch_st_rows(int mode, int elems, int n_blocks, const SteerArgs& A, hipStream_t st) {
  const void* k = mode == 0   ? MI_ST_PICK(k_st_rows, 0)
                  : mode == 1 ? MI_ST_PICK(k_st_rows, 1)
                  : mode == 2 ? MI_ST_PICK(k_st_rows, 2)
                              : MI_ST_PICK(k_st_rows, 3);
  return st_launch(k, n_blocks, A, st);
}

hipError_t launch_st_cols(int mode, int elems, int n_blocks, const SteerArgs& A, hipStream_t st) {
  const void* k = mode == 0 ? MI_ST_PICK(k_st_cols, 0) : MI_ST_PICK(k_st_cols, 1);
  return st_launch(k, n_blocks, A, st);
}

hipError_t launch_st_rows_inv(int mode, int elems, int n_blocks, const SteerArgs& A, hipStream_t st) {
  const void* k = mode == 0 ? MI_ST_PICK(k_st_rows_inv, 0) : MI_ST_PICK(k_st_rows_inv, 1);
  return st_launch(k, n_blocks, A, st);
}

hipError_t launch_st_init(int n_blocks, const SteerArgs& A, hipStream_t st) {
  return st_launch(reinterpret_cast<const void*>(&k_st_init), n_blocks, A, st);
}

hipError_t launch_st_update(int n_blocks, const SteerArgs& A, hipStream_t st) {
  return st_launch(reinterpret_cast<const void*>(&k_st_update), n_blocks, A, st);
}

}  // namespace mi
