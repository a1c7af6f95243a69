// Hogbom CLEAN, clean-beam fit and restore (gfx950).
//
// Algorithm 1 (improved_clean) finds the strength and position of the map peak and
// repeats a CLEAN step and a new peak search until the peak falls to the sky level;
// Sec. 4.3 fixes the loop gain at 0.1.  The loop here is classic Hogbom CLEAN:
//   p = argmax |R| (ties: lowest y*N + x), stop if |R[p]| <= thr,
//   f = gain R[p] (FP64), model[p] += f, R -= f beam[y - p_y + N][x - p_x + N].
//
// k_clean is one persistent, cooperatively launched kernel.  Each image is owned by a
// team of G workgroups; member m keeps pixels [m N^2/G, (m+1) N^2/G) of the residual in
// LDS for the whole loop.  One iteration per member: fused subtract + local argmax over
// its LDS chunk, a wave/workgroup reduction of packed 64-bit keys
//   (|R| bits << 32) | ((2^24 - 1 - index) << 8) | sign
// whose maximum is the largest |R| with the lowest index on ties, one slot store, and a
// team barrier (agent-scope release/acquire on a monotone counter); every member then
// reduces all G slots itself, so all members agree on the pick without a second barrier.
// Slots are double-buffered by barrier parity.  When the team's workgroups sit on one XCD
// (blocks b = x + 8 r run on XCD x), the barrier traffic stays in that XCD's L2.
//
// Restore (Algorithm 1's clean beam, gpu_cpsf): k_beamfit fits a Gaussian to the beam's
// main lobe (4-connected region around (N, N) with beam > 0.35) by FP64 least squares on
// ln(beam); k_clean then adds each component times that Gaussian (truncated where it
// drops below 1e-12) to its LDS chunk after the loop, and writes the restored image.
#include "mi_internal.h"

namespace mi {

constexpr int CL_THREADS = 1024;
constexpr int CL_WAVES = CL_THREADS / 64;
constexpr int RESTORE_RMAX = 64;
constexpr int FIT_HALF = 63;                 // fit box half-width (pixels)
constexpr int FIT_BOX = 2 * FIT_HALF + 1;


namespace {

__device__ __forceinline__ unsigned long long make_key(float r, int idx, int posonly) {
  const unsigned b = __float_as_uint(r);
  unsigned k32, sgn = 0u;
  if (posonly) {
    k32 = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  } else {
    k32 = b & 0x7fffffffu;
    sgn = b >> 31;
  }
  return ((unsigned long long)k32 << 32) | ((unsigned long long)(0xFFFFFFu - (unsigned)idx) << 8) | sgn;
}

__device__ __forceinline__ void decode_key(unsigned long long key, int posonly, int& idx, float& val) {
  idx = (int)(0xFFFFFFu - (unsigned)((key >> 8) & 0xFFFFFFu));
  const unsigned k32 = (unsigned)(key >> 32);
  if (posonly) {
    const unsigned b = (k32 & 0x80000000u) ? (k32 & 0x7fffffffu) : ~k32;
    val = __uint_as_float(b);
  } else {
    val = __uint_as_float(k32 | ((unsigned)(key & 1ull) << 31));
  }
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long t = __shfl_xor(v, o);
    v = t > v ? t : v;
  }
  return v;
}

// Workgroup max of a key; result returned to every thread.
__device__ unsigned long long block_max_key(unsigned long long k, unsigned long long* red) {
  k = wave_max_u64(k);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = k;
  __syncthreads();
  if (wave == 0) {
    unsigned long long v = lane < CL_WAVES ? red[lane] : 0ull;
    v = wave_max_u64(v);
    if (lane == 0) red[CL_WAVES] = v;
  }
  __syncthreads();
  const unsigned long long r = red[CL_WAVES];
  __syncthreads();
  return r;
}

// Local argmax over the chunk (initial search, no subtraction).
__device__ unsigned long long chunk_argmax(const float* R, int chunk, int c0, int posonly) {
  float bv = 0.f;
  int bi = -1;
  float ba = -1.f;
  for (int q = threadIdx.x; q < chunk; q += CL_THREADS) {
    const float r = R[q];
    const float a = posonly ? r : fabsf(r);
    if (bi < 0 || a > ba) { ba = a; bv = r; bi = c0 + q; }
  }
  return bi < 0 ? 0ull : make_key(bv, bi, posonly);
}

// Fused beam subtraction and local argmax.
__device__ unsigned long long chunk_subtract_argmax(float* R, int chunk, int c0, int log2N, int N,
                                                    const float* __restrict__ bm, float f, int py, int px,
                                                    int posonly) {
  const int twoN = 2 * N;
  float bv = 0.f;
  int bi = -1;
  float ba = -1.f;
  const float* bwin = bm + (int64_t)(N - py) * twoN + (N - px);   // beam[y - py + N][x - px + N]
  for (int q = threadIdx.x; q < chunk; q += CL_THREADS) {
    const int g = c0 + q;
    const int y = g >> log2N, x = g & (N - 1);
    const float r = R[q] - f * bwin[(int64_t)y * twoN + x];
    R[q] = r;
    const float a = posonly ? r : fabsf(r);
    if (bi < 0 || a > ba) { ba = a; bv = r; bi = g; }
  }
  return bi < 0 ? 0ull : make_key(bv, bi, posonly);
}

// Team barrier: every member arrives once per call; `target` = G * (calls so far + 1).
// The wait is bounded: after BARRIER_SPIN_LIMIT polls (seconds) the workgroup gives up and
// returns false, so a broken launch ends instead of spinning forever.
constexpr unsigned BARRIER_SPIN_LIMIT = 1u << 24;

__device__ __forceinline__ bool team_barrier(unsigned* bar, unsigned target, int* flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    int ok = 1;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > BARRIER_SPIN_LIMIT) { ok = 0; break; }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *flag = ok;
  }
  __syncthreads();
  return *flag != 0;
}

}  // namespace

__global__ void __launch_bounds__(CL_THREADS)
k_clean(CleanArgs A) {
  extern __shared__ float R[];
  __shared__ unsigned long long red[CL_WAVES + 1];
  __shared__ int bar_ok;
  const int G = A.G;
  int team, member;
  if (A.xcd_map) {
    const int x = blockIdx.x & 7, r = blockIdx.x >> 3;
    team = (r / G) * 8 + x;
    member = r % G;
  } else {
    team = blockIdx.x / G;
    member = blockIdx.x % G;
  }
  unsigned* bar = A.bar + team;
  unsigned long long* slots = A.slots + (size_t)team * 2 * G;
  unsigned nbar = 0;
  const int tid = threadIdx.x;

  for (int ti = A.team_off[team]; ti < A.team_off[team + 1]; ++ti) {
    const int img = A.team_imgs[ti];
    const InstDesc d = A.inst[img];
    const int N = d.N, log2N = d.log2N;
    const int chunk = (N * N) / G;
    const int c0 = member * chunk;
    const float* dirty = A.dirty + d.img_off + c0;
    for (int q = tid; q < chunk; q += CL_THREADS) R[q] = dirty[q];
    if (A.model) {
      double* m = A.model + d.img_off + c0;
      for (int q = tid; q < chunk; q += CL_THREADS) m[q] = 0.0;
    }
    __syncthreads();
    const int niter = A.niter[img];
    const float thr = A.thr ? A.thr[img] : 0.0f;
    const float* bm = A.beam + d.beam_off;
    unsigned long long key = block_max_key(chunk_argmax(R, chunk, c0, A.posonly), red);
    int it = 0;
    for (; it < niter; ++it) {
      const int par = nbar & 1;
      if (tid == 0)
        __hip_atomic_store(&slots[par * G + member], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ++nbar;
      if (!team_barrier(bar, nbar * (unsigned)G, &bar_ok)) {
        if (tid == 0 && A.status) atomicOr(&A.status[img], 16);
        return;
      }
      unsigned long long k = 0ull;
      for (int m = tid; m < G; m += 64)
        if (tid < 64) {
          unsigned long long t = __hip_atomic_load(&slots[par * G + m], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          k = t > k ? t : k;
        }
      if (tid < 64) {
        k = wave_max_u64(k);
        if (tid == 0) red[CL_WAVES] = k;
      }
      __syncthreads();
      const unsigned long long best = red[CL_WAVES];
      __syncthreads();
      int p;
      float val;
      decode_key(best, A.posonly, p, val);
      if (!(fabsf(val) > thr)) break;
      const double f = (double)A.gain * (double)val;
      if (tid == 0) {
        if (A.model && p >= c0 && p < c0 + chunk) A.model[d.img_off + p] += f;
        if (member == 0 && A.comp_idx) {
          A.comp_idx[A.comp_off[img] + it] = p;
          A.comp_flux[A.comp_off[img] + it] = f;
        }
      }
      key = block_max_key(chunk_subtract_argmax(R, chunk, c0, log2N, N, bm, (float)f, p >> log2N, p & (N - 1),
                                                A.posonly), red);
    }
    if (member == 0 && tid == 0 && A.ncomp) A.ncomp[img] = it;
    __syncthreads();
    float* ro = A.resid + d.img_off + c0;
    for (int q = tid; q < chunk; q += CL_THREADS) ro[q] = R[q];

    if (A.restored && A.cbeam) {
      // all components must be visible to every member
      ++nbar;
      if (!team_barrier(bar, nbar * (unsigned)G, &bar_ok)) {
        if (tid == 0 && A.status) atomicOr(&A.status[img], 16);
        return;
      }
      const float ga = (float)A.cbeam[6 * img + 0], gb = (float)A.cbeam[6 * img + 1],
                  gc = (float)A.cbeam[6 * img + 2];
      const int rr = A.rrad[img];
      const int side = 2 * rr + 1;
      const int row_lo = c0 >> log2N, row_hi = (c0 + chunk - 1) >> log2N;
      for (int i = 0; i < it; ++i) {
        const int p = __hip_atomic_load(&A.comp_idx[A.comp_off[img] + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int py = p >> log2N, px = p & (N - 1);
        if (py + rr < row_lo || py - rr > row_hi) continue;
        const unsigned long long fb = __hip_atomic_load(
            reinterpret_cast<unsigned long long*>(&A.comp_flux[A.comp_off[img] + i]), __ATOMIC_RELAXED,
            __HIP_MEMORY_SCOPE_AGENT);
        const float f = (float)__longlong_as_double((long long)fb);
        for (int w = tid; w < side * side; w += CL_THREADS) {
          const int dy = w / side - rr, dx = w % side - rr;
          const int y = py + dy, x = px + dx;
          if (y < 0 || y >= N || x < 0 || x >= N) continue;
          const int g = (y << log2N) + x;
          if (g < c0 || g >= c0 + chunk) continue;
          const float e = (float)dx * (ga * (float)dx + gb * (float)dy) + gc * (float)dy * (float)dy;
          atomicAdd(&R[g - c0], f * expf(-e));
        }
      }
      __syncthreads();
      float* rs = A.restored + d.img_off + c0;
      for (int q = tid; q < chunk; q += CL_THREADS) rs[q] = R[q];
    }
    __syncthreads();
  }
}

// Clean-beam fit: one workgroup per instance.
__global__ void __launch_bounds__(CL_THREADS)
k_beamfit(const InstDesc* __restrict__ inst, const float* __restrict__ beam, double* __restrict__ cbeam,
          int* __restrict__ rrad, int* __restrict__ status) {
  __shared__ unsigned char lab[FIT_BOX * FIT_BOX];
  __shared__ int changed;
  __shared__ double red[8][CL_WAVES];
  __shared__ int cnt[3][CL_WAVES];
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
  for (int q = threadIdx.x; q < side * side; q += CL_THREADS) lab[q] = 0;
  __syncthreads();
  if (threadIdx.x == 0) lab[hb * side + hb] = bval(hb * side + hb) > thr ? 1 : 0;
  __syncthreads();
  for (;;) {
    if (threadIdx.x == 0) changed = 0;
    __syncthreads();
    for (int q = threadIdx.x; q < side * side; q += CL_THREADS) {
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
  for (int q = threadIdx.x; q < side * side; q += CL_THREADS) {
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
      for (int w = 0; w < CL_WAVES; ++w) t[k] += red[k][w];
    }
    for (int w = 0; w < CL_WAVES; ++w) { nxy += cnt[0][w]; nx += cnt[1][w]; ny += cnt[2][w]; }
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

// Degrid (prediction / adjoint): one thread per visibility of instance blockIdx.y; FP64
// tap sums over the FP64 forward spectrum (same cancellation argument as the imager).
__global__ void k_degrid(const InstDesc* __restrict__ inst, const float2* __restrict__ uv,
                         const float* __restrict__ w_in, const float* __restrict__ wts,
                         const double* __restrict__ b0, const double2* __restrict__ fgrid, Tables T,
                         int adjoint, float2* __restrict__ out) {
  __shared__ double tab[TAB_LEN];
  for (int t = threadIdx.x; t < TAB_LEN; t += blockDim.x) tab[t] = T.tab[t];
  __syncthreads();
  const int i = blockIdx.y;
  const InstDesc d = inst[i];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n_vis) return;
  const int64_t vi = d.vis_off + k;
  const float2 q = uv[vi];
  const Sample s = prep_sample(q.x, q.y, w_in[vi], d.scale, d.N);
  double2 acc = make_double2(0.0, 0.0);
  if (s.keep) {
    const int P = d.N, h = P / 2;
    const double2* F = fgrid + d.gd_off;
    for (int dv = -HALF_W; dv <= HALF_W; ++dv) {
      const double tv = tab[dv * OS - s.ov + TAB_CENTRE];
      double2 row = make_double2(0.0, 0.0);
      for (int du = -HALF_W; du <= HALF_W; ++du) {
        const double tu = tab[du * OS - s.ou + TAB_CENTRE];
        const int a = s.cu + du, b = s.cv + dv;
        double2 f;
        if (a <= 0) {
          f = F[(int64_t)(a + h - 1) * P + (b + h)];
        } else {
          f = F[(int64_t)(-a + h - 1) * P + (-b + h)];
          f.y = -f.y;
        }
        row.x += tu * f.x;
        row.y += tu * f.y;
      }
      acc.x += tv * row.x;
      acc.y += tv * row.y;
    }
    if (adjoint) {
      const double bd = b0[2 * i];
      const double sc = bd > 0.0 ? 2.0 * (double)wts[vi] / bd : 0.0;
      acc.x *= sc;
      acc.y *= sc;
    }
  }
  out[vi] = make_float2((float)acc.x, (float)acc.y);
}

// ---- host launchers ----
hipError_t clean_max_blocks_per_cu(size_t lds_bytes, int* nb) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, reinterpret_cast<const void*>(k_clean), CL_THREADS,
                                                      lds_bytes);
}

hipError_t launch_clean(const CleanArgs& A, int n_blocks, size_t lds_bytes, hipStream_t st) {
  CleanArgs a = A;
  void* args[] = {&a};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_clean), dim3(n_blocks), dim3(CL_THREADS), args,
                                    lds_bytes, st);
}

hipError_t launch_beamfit(const InstDesc* inst, int n_inst, const float* beam, double* cbeam, int* rrad,
                          int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_beamfit, dim3(n_inst), dim3(CL_THREADS), 0, st, inst, beam, cbeam, rrad, status);
  return hipGetLastError();
}

hipError_t launch_degrid(const InstDesc* inst, int n_inst, int max_nvis, const float2* uv, const float* w_in,
                         const float* wts, const double* b0, const double2* fgrid, const Tables& T, int adjoint,
                         float2* out, hipStream_t st) {
  if (max_nvis <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_degrid, dim3((max_nvis + 255) / 256, n_inst), dim3(256), 0, st, inst, uv, w_in, wts, b0,
                     fgrid, T, adjoint, out);
  return hipGetLastError();
}

}  // namespace mi
