// LDS-resident Stockham FFT primitives shared by the transform kernels (internal header,
// not part of the ABI).  Everything sits in an unnamed namespace: each kernel source that
// includes it gets its own inlined copy.
//
// A radix-R pass over nl lines of P points in LDS (line stride P, one padding element per
// 8 against bank conflicts) reads butterfly b's inputs x[b + m P/R] and writes
// y[(b/L) L R + b%L + q L] after twiddling by w^m, w = exp(s 2 pi i (b%L)/(L R)); twiddles
// come from the FP64 table exp(+2 pi i t / 8192) and their powers by recurrence.  The
// values are double2 (FP64) or float2 (FP32): the twiddles are always computed in FP64.
#pragma once

#include "mi_internal.h"

namespace mi {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// multiply by s*i (s = +1 or -1)
__device__ __forceinline__ double2 mul_si(double2 a, double s) { return make_double2(-s * a.y, s * a.x); }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 mul_si(float2 a, double s) {
  const float f = (float)s;
  return make_float2(-f * a.y, f * a.x);
}

// A twiddle (computed in FP64) in the precision of the data.
template <typename V> __device__ __forceinline__ V tw_as(double2 w);
template <> __device__ __forceinline__ double2 tw_as<double2>(double2 w) { return w; }
template <> __device__ __forceinline__ float2 tw_as<float2>(double2 w) { return make_float2((float)w.x, (float)w.y); }

template <int R, typename V> __device__ __forceinline__ void small_dft(V* x, double s);

template <> __device__ __forceinline__ void small_dft<2, double2>(double2* x, double) {
  double2 a = x[0], b = x[1];
  x[0] = cadd(a, b);
  x[1] = csub(a, b);
}
template <> __device__ __forceinline__ void small_dft<2, float2>(float2* x, double) {
  float2 a = x[0], b = x[1];
  x[0] = cadd(a, b);
  x[1] = csub(a, b);
}

template <typename V> __device__ __forceinline__ void dft4(V* x, double s) {
  V t0 = cadd(x[0], x[2]), t1 = csub(x[0], x[2]);
  V t2 = cadd(x[1], x[3]), t3 = mul_si(csub(x[1], x[3]), s);
  x[0] = cadd(t0, t2);
  x[2] = csub(t0, t2);
  x[1] = cadd(t1, t3);
  x[3] = csub(t1, t3);
}
template <> __device__ __forceinline__ void small_dft<4, double2>(double2* x, double s) { dft4(x, s); }
template <> __device__ __forceinline__ void small_dft<4, float2>(float2* x, double s) { dft4(x, s); }

template <typename V> __device__ __forceinline__ void dft8(V* x, double s) {
  V e[4] = {x[0], x[2], x[4], x[6]};
  V o[4] = {x[1], x[3], x[5], x[7]};
  dft4(e, s);
  dft4(o, s);
  const double r = 0.70710678118654752440;
  // w8^q = exp(s i pi q / 4)
  V o1 = cmul(o[1], tw_as<V>(make_double2(r, s * r)));
  V o2 = mul_si(o[2], s);
  V o3 = cmul(o[3], tw_as<V>(make_double2(-r, s * r)));
  x[0] = cadd(e[0], o[0]);
  x[4] = csub(e[0], o[0]);
  x[1] = cadd(e[1], o1);
  x[5] = csub(e[1], o1);
  x[2] = cadd(e[2], o2);
  x[6] = csub(e[2], o2);
  x[3] = cadd(e[3], o3);
  x[7] = csub(e[3], o3);
}
template <> __device__ __forceinline__ void small_dft<8, double2>(double2* x, double s) { dft8(x, s); }
template <> __device__ __forceinline__ void small_dft<8, float2>(float2* x, double s) { dft8(x, s); }

// LDS index with one padding element per 8: strided butterfly stores of 16-byte elements
// otherwise land on the same banks.  (A further element per line, against conflicts in
// the staging and the transposed stores, measured slower overall.)
__device__ __forceinline__ int pd(int i) { return i + (i >> 3); }

// One Stockham radix-R pass over nl lines of P points held in LDS (line stride P).
// L = product of the radices already applied.  Butterfly b of a line reads x[b + m P/R]
// and writes y[(b/L) L R + b%L + q L] after twiddling by w^m, w = exp(s 2 pi i (b%L)/(L R));
// w comes from the FP64 table and its powers by recurrence in FP64, each rounded once to
// the data's precision (V = double2 or float2).
// wreg: when not null, the twiddle exp(+2 pi i j / (L R)) shared by all of this thread's
// butterflies in the pass (TwRegs); otherwise read from the table.
template <int R, int ELEMS, int THREADS, typename V>
__device__ __forceinline__ void stockham_pass(V* buf, int log2P, int log2L, int nl, double s,
                                              const double2* __restrict__ tw, const double2* wreg = nullptr) {
  constexpr int BPT = (ELEMS / THREADS / R) > 0 ? ELEMS / THREADS / R : 1;
  constexpr int LOG2R = R == 8 ? 3 : (R == 4 ? 2 : 1);
  const int log2nb = log2P - LOG2R;
  const int nb = 1 << log2nb;
  const int total = nl << log2nb;
  const int L = 1 << log2L;
  const int tw_shift = (13 - log2L - LOG2R);   // table length 8192 = 2^13
  V x[BPT][R];
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = threadIdx.x + q * THREADS;
    if (b < total) {
      const int line = b >> log2nb, bb = b & (nb - 1);
      const int base = (line << log2P) + bb;
#pragma unroll
      for (int m = 0; m < R; ++m) x[q][m] = buf[pd(base + (m << log2nb))];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = threadIdx.x + q * THREADS;
    if (b < total) {
      const int line = b >> log2nb, bb = b & (nb - 1);
      const int j = bb & (L - 1), blk = bb >> log2L;
      if (L > 1) {
        double2 w1 = wreg ? *wreg : tw[j << tw_shift];
        w1.y *= s;
        double2 w = w1;
        x[q][1] = cmul(x[q][1], tw_as<V>(w));
#pragma unroll
        for (int m = 2; m < R; ++m) {
          w = cmul(w, w1);
          x[q][m] = cmul(x[q][m], tw_as<V>(w));
        }
      }
      small_dft<R, V>(x[q], s);
      const int base = (line << log2P) + (blk << (log2L + LOG2R)) + j;
#pragma unroll
      for (int m = 0; m < R; ++m) buf[pd(base + (m << log2L))] = x[q][m];
    }
  }
  __syncthreads();
}

// log2 of the radix of the next pass when rem of log2P bits are left: radix 8 while more
// than 4 bits remain, then 4 (4 bits as 4 x 4, 2 bits), 8 (3 bits) or 2 (1 bit).
__device__ __forceinline__ int pass_log2r(int rem) { return (rem == 4 || rem == 2) ? 2 : (rem == 1 ? 1 : 3); }

// Full length-P FFT (sign s) of nl lines in LDS; nl * P <= ELEMS.
template <int ELEMS, int THREADS, typename V>
__device__ __forceinline__ void lds_fft(V* buf, int log2P, int nl, double s, const double2* __restrict__ tw) {
  int done = 0, rem = log2P;
  while (rem > 0) {
    const int r = pass_log2r(rem);
    if (r == 3) stockham_pass<8, ELEMS, THREADS>(buf, log2P, done, nl, s, tw);
    else if (r == 2) stockham_pass<4, ELEMS, THREADS>(buf, log2P, done, nl, s, tw);
    else stockham_pass<2, ELEMS, THREADS>(buf, log2P, done, nl, s, tw);
    done += r;
    rem -= r;
  }
}

// Twiddles held in registers.  A pass's twiddle depends only on the thread, P and the
// pass, not on the data, so a kernel loads its threads' twiddles before its data and its
// transforms then issue no global loads: a global load inside a transform waits for its
// own round trip, pass after pass, and also for every older load and store of the
// workgroup (the vector memory counter completes in order), e.g. a persistent kernel's
// prefetch of its next item.  Covers P = 4 .. 4096 in 4096-point workgroups of at least
// 512 threads: at most four passes (radix 8 or 4), the first without twiddles, and in each
// pass P / R <= THREADS, so the butterflies b and b + THREADS of a thread share
// j = (b mod P/R) mod L and one twiddle per pass serves them all.  Larger workgroups keep
// the table reads.
template <int ELEMS, int THREADS>
struct TwRegs {
  static constexpr bool ON = ELEMS <= 4096 && THREADS >= 512;
  static constexpr int NP = 3;                                             // passes after the first
  double2 w[NP];
  int log2P = -1;

  // Issue the loads for line length 2^lp (the first use waits for them).
  __device__ __forceinline__ void load(int lp, const double2* __restrict__ tw) {
    if (!ON) return;
    log2P = lp;
    int done = 0, rem = lp;
#pragma unroll
    for (int p = 0; p <= NP; ++p) {
      if (rem > 0) {
        const int r = pass_log2r(rem);
        if (p > 0) {
          const int j = ((int)threadIdx.x & ((1 << (lp - r)) - 1)) & ((1 << done) - 1);
          w[p - 1] = tw[j << (13 - done - r)];
        }
        done += r;
        rem -= r;
      }
    }
  }

  // Persistent kernels: load when the line length changes, and settle the loads there, once
  // per line length; otherwise the compiler cannot tell at a twiddle's use whether the load
  // that wrote it is still pending and waits for every outstanding memory operation there,
  // i.e. for the prefetch the twiddles are meant to let the transform overlap.
  __device__ __forceinline__ void ensure(int lp, const double2* __restrict__ tw) {
    if (!ON || lp == log2P) return;
    load(lp, tw);
    __builtin_amdgcn_s_waitcnt(0);
  }
};

// lds_fft with the twiddles of t (loaded by t.ensure for this log2P and sign).
template <int ELEMS, int THREADS, typename V>
__device__ __forceinline__ void lds_fft(V* buf, int log2P, int nl, double s, const double2* __restrict__ tw,
                                        const TwRegs<ELEMS, THREADS>& t) {
  if constexpr (!TwRegs<ELEMS, THREADS>::ON) {
    lds_fft<ELEMS, THREADS>(buf, log2P, nl, s, tw);
  } else {
    int done = 0, rem = log2P;
#pragma unroll
    for (int p = 0; p <= TwRegs<ELEMS, THREADS>::NP; ++p) {
      if (rem > 0) {
        const int r = pass_log2r(rem);
        const double2* wr = &t.w[p > 0 ? p - 1 : 0];
        if (r == 3) stockham_pass<8, ELEMS, THREADS>(buf, log2P, done, nl, s, tw, wr);
        else stockham_pass<4, ELEMS, THREADS>(buf, log2P, done, nl, s, tw, wr);
        done += r;
        rem -= r;
      }
    }
  }
}

__device__ __forceinline__ int ilog2(int v) { return 31 - __clz(v); }

}  // namespace
}  // namespace mi
