// Hogbom CLEAN, clean-beam fit and restore (gfx950).
//
// Algorithm 1 (improved_clean) finds the strength and position of the map peak and
// repeats a CLEAN step and a new peak search until the peak falls to the sky level;
// Sec. 4.3 fixes the loop gain at 0.1.  The loop here is classic Hogbom CLEAN:
//   p = argmax |R| (ties: lowest y*N + x), stop if |R[p]| <= thr,
//   f = gain R[p] (FP64), model[p] += f, R -= f beam[y - p_y + N][x - p_x + N].
//
// k_clean is one persistent, cooperatively launched kernel.  Each image is owned by a
// team of G workgroups (G chosen per image size so every member holds the same number of
// pixels); member m keeps pixels [m N^2/G, (m+1) N^2/G) of the residual in registers for
// the whole loop.  A per-block table gives each block its team and member, and teams of
// one launch may have different sizes (a mixed-size batch runs in one launch).  One
// iteration per member: window subtraction fused with the local maximum, 32-bit value
// keys reduced across the wave (DPP) and the workgroup (LDS), a search for the lowest
// index only in the wave holding the maximum, and one exchange of packed 64-bit keys
//   (|R| bits << 32) | ((2^24 - 1 - index) << 8) | (seq << 1) | sign
// through the team's slots; every member reduces all G slots itself, so all agree on the
// pick without a second round.  Teams of up to 32 workgroups sit on one XCD (blocks b with
// equal b % 8 share an XCD), so their beam windows share that XCD's L2.
//
// Beam reads: 16-byte raw buffer loads; window rows above the pick read the point-mirrored
// beam row when the beam is exactly symmetric (checked per call by k_beam_symcheck), which
// halves the distinct beam lines a central window touches.
//
// Restore (Algorithm 1's clean beam, gpu_cpsf): k_beamfit (k_beam.hip) fits a Gaussian to
// the beam's main lobe by FP64 least squares on ln(beam); k_clean then adds each component
// times that Gaussian (truncated where it drops below 1e-12) to its chunk, staged through
// LDS, and writes the restored image.
#include <algorithm>

#include "mi_internal.h"

namespace mi {

constexpr int CL_THREADS = 1024;
constexpr int CL_WAVES = CL_THREADS / 64;
// Word 3 of a raw buffer resource descriptor on gfx9-family GPUs (untyped dword access).
constexpr int BUFFER_RSRC_WORD3 = 0x00020000;


namespace {

// ---- team communication.  Slots hold 64-bit keys
//   (peak bits << 32) | ((2^24 - 1 - index) << 8) | (seq << 1) | sign
// where seq is a 7-bit barrier sequence number.  All shared words (slots, component list)
// are accessed with agent-scope relaxed atomics, which are coherent per location across
// CUs and XCDs; ordering between them is made explicit with s_waitcnt vmcnt(0).  No
// release/acquire fences are used: on this GPU those write back and invalidate the whole
// L2, which would also evict the beam window every iteration.  The LOCAL variant only
// changes team placement (all members of a team on one XCD, sharing its L2).
__device__ __forceinline__ void wait_vm() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Shared words use agent scope (sc1) in both placements: workgroup-scope (sc0) accesses are
// not coherent between CUs of one XCD on this GPU outside threadgroup-split mode.
#define MI_TEAM_SCOPE __HIP_MEMORY_SCOPE_AGENT

template <bool LOCAL>
__device__ __forceinline__ unsigned long long ld_shared_u64(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, MI_TEAM_SCOPE);
}

template <bool LOCAL>
__device__ __forceinline__ unsigned ld_shared_u32(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, MI_TEAM_SCOPE);
}

template <bool LOCAL>
__device__ __forceinline__ void st_shared_u64(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, MI_TEAM_SCOPE);
}

template <bool LOCAL>
__device__ __forceinline__ void st_shared_u32(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, MI_TEAM_SCOPE);
}

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

// Wave-wide maximum of a 32-bit unsigned value, returned uniform: DPP steps within each
// row of 16 lanes (quad swaps, half-row and row mirrors), then the four row results.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false));   // [1,0,3,2]
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false));   // [2,3,0,1]
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xF, 0xF, false));  // half mirror
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x140, 0xF, 0xF, false));  // row mirror
  const unsigned r0 = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
  const unsigned r1 = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
  const unsigned r2 = (unsigned)__builtin_amdgcn_readlane((int)v, 32);
  const unsigned r3 = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
  return max(max(r0, r1), max(r2, r3));
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  const unsigned hi = wave_max_u32((unsigned)(v >> 32));
  const unsigned lo = wave_max_u32((unsigned)(v >> 32) == hi ? (unsigned)v : 0u);
  return ((unsigned long long)hi << 32) | lo;
}

// Order-preserving 32-bit key of a peak candidate: |r| bits (all pixels) or the signed
// float's total order (positive-only picks).  Empty lanes give the smallest keys.
__device__ __forceinline__ unsigned value_key(float r, int posonly) {
  const unsigned b = __float_as_uint(r);
  if (posonly) return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return (b & 0x80000000u) ? 0u : b;                  // r = |R| >= 0, or -1 when empty
}

__device__ __forceinline__ float key_value(unsigned k32, int posonly) {
  if (posonly) return __uint_as_float((k32 & 0x80000000u) ? (k32 & 0x7fffffffu) : ~k32);
  return __uint_as_float(k32);
}

// Team exchange, run by one whole wave with its workgroup key wk (uniform): publish it for
// barrier `seq`, poll the team's G slots until all carry `seq`, and leave their maximum in
// *out (~0 if the wait timed out).  `ordered`: wait for this wave's earlier stores
// (component list) before publishing.
constexpr unsigned POLL_LIMIT = 1u << 22;     // polls per wait (seconds): a hang becomes an abort

// `poll_limit` bounds every wait; `skip_publish` (failure-path tests only, set from the
// host) leaves this member's slot unwritten so that every member of the team times out.
template <bool LOCAL>
__device__ __forceinline__ void team_exchange(unsigned long long* slots, int G, int member, unsigned seq,
                                              unsigned long long wk, unsigned long long* out, bool ordered,
                                              unsigned poll_limit, bool skip_publish) {
  const int lane = threadIdx.x & 63;
  const unsigned s7 = seq & 127u;
  unsigned long long* sl = slots + (seq & 1u) * G;
  if (lane == 0 && !skip_publish) {
    if (ordered) wait_vm();
    st_shared_u64<LOCAL>(sl + member, (wk & ~0xFEull) | ((unsigned long long)s7 << 1));
  }
  unsigned long long k = 0ull;
  bool timed_out = false;
  for (int m0 = 0; m0 < G; m0 += 64) {
    const int m = m0 + lane;
    bool done = m >= G;
    unsigned spins = 0;
    unsigned long long v = 0ull;
    while (true) {
      if (!done) {
        v = ld_shared_u64<LOCAL>(sl + m);
        done = ((unsigned)(v >> 1) & 127u) == s7;
      }
      if (__all(done)) break;
      if (++spins > poll_limit) { timed_out = true; break; }
    }
    if (m < G && done) k = v > k ? v : k;
  }
  k = wave_max_u64(k);
  if (lane == 0) *out = timed_out ? ~0ull : k;
}

// Window subtraction R -= f beam[window].  Group g of a thread covers 4 pixels of one row;
// groups g < K read the point-mirrored beam row (highest address first, so the 16-byte
// load's components come reversed), the others the direct row.  Offsets live in the VGPR
// operand, which the buffer range check covers: a group past the image's range reads
// zeros.  A scheduling barrier between batches keeps at most LB loads in flight, which
// bounds the registers next to the PPT residual values.
template <int NS, int LB>
__device__ __forceinline__ void sub_window(float* R, __amdgpu_buffer_rsrc_t rs, unsigned vd, unsigned vm, int K,
                                           float f) {
  constexpr unsigned GSTEP = 2u * 4u * CL_THREADS * 4u;   // bytes between load steps (2 STEP floats)
#pragma unroll
  for (int s0 = 0; s0 < NS; s0 += LB) {
    float4 bv[LB];
#pragma unroll
    for (int s = 0; s < LB; ++s) {
      const int g = s0 + s;
      const unsigned vo = g < K ? vm - GSTEP * g : vd + GSTEP * g;
      bv[s] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)vo, 0, 0));
    }
#pragma unroll
    for (int s = 0; s < LB; ++s) {
      const int g = s0 + s;
      const bool m = g < K;
      R[4 * g + 0] = fmaf(-f, m ? bv[s].w : bv[s].x, R[4 * g + 0]);
      R[4 * g + 1] = fmaf(-f, m ? bv[s].z : bv[s].y, R[4 * g + 1]);
      R[4 * g + 2] = fmaf(-f, m ? bv[s].y : bv[s].z, R[4 * g + 2]);
      R[4 * g + 3] = fmaf(-f, m ? bv[s].x : bv[s].w, R[4 * g + 3]);
    }
    if (s0 + LB < NS) __builtin_amdgcn_sched_barrier(0);
  }
}

}  // namespace

// Residual in registers: thread t of member m owns 4-pixel groups at
// c0 + 4 (t + CL_THREADS s) + j, s < PPT/4, j < 4 (c0 = m N^2/G).  For N <= 1024 and G <= N,
// c0 is a row start and a step of 4 CL_THREADS = 4096 pixels is 4096/N whole rows, i.e.
// 8192 floats further into the beam window: each group is one 16-byte buffer load at a
// uniform (SGPR) offset from a fixed per-thread offset.
template <int PPT, bool LOCAL, bool WIN>
__global__ void __launch_bounds__(CL_THREADS)
k_clean(CleanArgs A) {
  static_assert(PPT % 4 == 0, "4 pixels per load");
  constexpr int NS = PPT / 4;
  constexpr int LB = NS < 8 ? NS : 8;
  extern __shared__ float Rl[];                       // restore staging (when requested)
  __shared__ unsigned long long red_k[CL_WAVES + 2];  // [0..1] team key by parity, [2..] wave keys
  __shared__ unsigned red_v[CL_WAVES];                // wave peak-value keys
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int2 bm = A.blk[blockIdx.x];
  const int team = __builtin_amdgcn_readfirstlane(bm.x), member = __builtin_amdgcn_readfirstlane(bm.y);
  if (team < 0) return;                               // idle slot of the launch
  const int G = A.team_G[team];
  unsigned long long* slots = A.slots + A.team_slot[team];
  unsigned seq = 0;
  const unsigned poll_limit = A.poll_limit ? A.poll_limit : POLL_LIMIT;
  const float NaN = __uint_as_float(0x7fc00000u);
  const int posonly = A.posonly;

  for (int ti = A.team_off[team]; ti < A.team_off[team + 1]; ++ti) {
    const int img = __builtin_amdgcn_readfirstlane(A.team_imgs[ti]);
    const InstDesc d = A.inst[img];
    const int N = d.N, log2N = d.log2N, twoN = 2 * N;
    const int chunk = (N * N) / G;
    const int c0 = member * chunk;
    constexpr int STEP = 4 * CL_THREADS;              // pixels per load step
    const int smax = (chunk + STEP - 1) / STEP;       // uniform
    const bool tvalid = 4 * tid < chunk;              // false only when chunk < STEP
    const int t4 = 4 * tid;
    const unsigned vtb = tvalid ? (unsigned)(((t4 >> log2N) * twoN + (t4 & (N - 1))) * 4) : 0u;
    const int row0 = c0 >> log2N;
    float R[PPT];
    {
      const float* dsrc = A.dirty + d.img_off + c0 + t4;
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int j = 0; j < 4; ++j) R[4 * s + j] = (s < smax && tvalid) ? dsrc[s * STEP + j] : NaN;
    }
    if (A.model) {
      double* m = A.model + d.img_off + c0 + t4;
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (s < smax && tvalid)
#pragma unroll
          for (int j = 0; j < 4; ++j) m[s * STEP + j] = 0.0;
      wait_vm();                                      // zeros land before any model atomic
    }
    __syncthreads();
    const int niter = A.niter[img];
    const float thr = A.thr ? A.thr[img] : 0.0f;
    const int64_t coff = A.comp_off[img];
    const float* bimg = A.beam + d.beam_off;
    // one resource over this image's beam; offsets are bytes from its first pixel
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(bimg), 0,
                                                                        16 * N * N, BUFFER_RSRC_WORD3);
    // mirrored reads need the beam exactly symmetric and each wave's 256 pixels of a load
    // step inside one row (N >= 256), so the choice is uniform per wave and step
    const bool sym = N >= 256 && A.asym[img] == 0;
    const int yw = row0 + __builtin_amdgcn_readfirstlane(t4 >> log2N);   // this wave's row at step 0
    const int RS = STEP >> log2N, log2RS = 12 - log2N;   // rows per load step (STEP = 2^12)
    // peak-search box: pixel (x, y) of group s, component j is x = xt + j, y = yt + s RS
    const int4 wb = WIN ? A.win[img] : make_int4(0, 0, N, N);
    const bool windowed = WIN && (wb.x > 0 || wb.y > 0 || wb.z < N || wb.w < N);   // uniform
    const int xt = t4 & (N - 1), yt = (c0 + t4) >> log2N;
    auto in_win = [&](int s, int j) {
      return (unsigned)(xt + j - wb.x) < (unsigned)(wb.z - wb.x) &&
             (unsigned)(yt + s * RS - wb.y) < (unsigned)(wb.w - wb.y);
    };
    float f = 0.0f;                                   // pending pick (none yet)
    int py = N / 2, px = N / 2;
    int it = 0;
    bool aborted = false;
    for (;; ++it) {
      // apply the pending pick and find the local peak.  Pixels a thread does not own hold
      // NaN (fma keeps NaN, fmaxf ignores it); their loads either stay inside this image's
      // beam or lie past the resource's range, which returns zero.
      // group s of this thread: row y = yw + s RS (+ lane row for N < 256), column x.
      // Direct: beam[y - py + N][x - px + N ..]; mirrored (rows y < py of a symmetric beam):
      // beam[N + py - y][N + px - x - 3 ..] read as one 16-byte load, components reversed.
      const unsigned vd = (unsigned)(((N - py + row0) * twoN + (N - px)) * 4) + vtb;
      const unsigned vm = (unsigned)(((N + py - row0) * twoN + (N + px - 3)) * 4) - vtb;
      // groups s < K lie in rows y < py: uniform per wave (one row per wave and step)
      int K = 0;
      if (sym && py > yw) K = min(NS, (py - yw + RS - 1) >> log2RS);
      K = __builtin_amdgcn_readfirstlane(K);
      sub_window<NS, LB>(R, rs, vd, vm, K, f);
      float best = posonly ? -INFINITY : -1.0f;
      if (windowed) {
#pragma unroll
        for (int k = 0; k < PPT; ++k)
          if (in_win(k >> 2, k & 3)) best = fmaxf(best, posonly ? R[k] : fabsf(R[k]));
      } else if (posonly) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) best = fmaxf(best, R[k]);
      } else {
#pragma unroll
        for (int k = 0; k < PPT; ++k) best = fmaxf(best, fabsf(R[k]));
      }
      if (it == niter) break;
      // peak value: wave maxima of the 32-bit value keys, then the workgroup maximum
      const unsigned wk32 = wave_max_u32(value_key(best, posonly));
      if (lane == 0) red_v[wave] = wk32;
      ++seq;
      __syncthreads();
      const unsigned lv = lane < CL_WAVES ? red_v[lane] : 0u;
      const unsigned wg32 = wave_max_u32(lv);
      const int n_tied = __popcll(__ballot(lane < CL_WAVES && lv == wg32));
      // only a wave holding the workgroup maximum locates it: the first 4-pixel group s in
      // which some lane matches, the lowest such lane, the lowest pixel in its group
      unsigned long long key = 0ull;
      if (wk32 == wg32) {
        const float wv = key_value(wg32, posonly);
        bool found = false;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          if (!found && s < smax) {
            unsigned long long mj[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
              mj[j] = __ballot((posonly ? R[4 * s + j] : fabsf(R[4 * s + j])) == wv && (!windowed || in_win(s, j)));
            const unsigned long long m = mj[0] | mj[1] | mj[2] | mj[3];
            if (m) {
              found = true;
              const int L = __builtin_ctzll(m);
              const int j = ((mj[0] >> L) & 1ull) ? 0 : ((mj[1] >> L) & 1ull) ? 1 : ((mj[2] >> L) & 1ull) ? 2 : 3;
              const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(R[4 * s + 0]), L));
              const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(R[4 * s + 1]), L));
              const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(R[4 * s + 2]), L));
              const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(R[4 * s + 3]), L));
              const float rv = j == 0 ? r0 : j == 1 ? r1 : j == 2 ? r2 : r3;
              key = make_key(rv, c0 + 4 * (64 * wave + L + CL_THREADS * s) + j, posonly);
            }
          }
        }
      }
      const bool stall = A.test_stall && member == 0;
      if (n_tied == 1) {
        if (wk32 == wg32) team_exchange<LOCAL>(slots, G, member, seq, key, &red_k[seq & 1u], false, poll_limit, stall);
      } else {                                        // several waves hold the maximum
        if (lane == 0) red_k[2 + wave] = key;
        __syncthreads();
        if (wave == 0) {
          const unsigned long long wk = wave_max_u64(lane < CL_WAVES ? red_k[2 + lane] : 0ull);
          team_exchange<LOCAL>(slots, G, member, seq, wk, &red_k[seq & 1u], false, poll_limit, stall);
        }
      }
      __syncthreads();
      // the team key is the same in every lane: keep it (and all that follows) uniform
      const unsigned long long tk = red_k[seq & 1u];
      const unsigned long long tkey =
          ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(tk >> 32)) << 32) |
          (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)tk);
      if (tkey == ~0ull) { aborted = true; break; }
      int p;
      float val;
      decode_key(tkey, posonly, p, val);
      if (!(fabsf(val) > thr)) break;
      const double fd = (double)A.gain * (double)val;
      if (tid == 0) {
        // fire-and-forget: same-thread atomics to one address apply in program order
        if (A.model && p >= c0 && p < c0 + chunk) atomicAdd(A.model + d.img_off + p, fd);
        if (member == 0 && A.comp_idx) {
          st_shared_u32<LOCAL>(reinterpret_cast<unsigned*>(A.comp_idx + coff + it), (unsigned)p);
          st_shared_u64<LOCAL>(reinterpret_cast<unsigned long long*>(A.comp_flux + coff + it),
                               (unsigned long long)__double_as_longlong(fd));
        }
      }
      f = (float)fd;
      py = p >> log2N;
      px = p & (N - 1);
    }
    if (aborted) {
      // this member leaves the kernel: every image still on the team's list (this one
      // included) is left incomplete, so each of them is flagged
      if (tid == 0 && A.status)
        for (int tj = ti; tj < A.team_off[team + 1]; ++tj) atomicOr(&A.status[A.team_imgs[tj]], 16);
      return;
    }
    if (member == 0 && tid == 0 && A.ncomp) A.ncomp[img] = it;
    {
      float* ro = A.resid + d.img_off + c0 + t4;
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (s < smax && tvalid)
#pragma unroll
          for (int j = 0; j < 4; ++j) ro[s * STEP + j] = R[4 * s + j];
    }
    if (A.restored && A.cbeam) {
      // every member needs the whole component list: one more exchange, ordered after
      // member 0's component stores
      ++seq;
      __syncthreads();
      if (wave == 0) team_exchange<LOCAL>(slots, G, member, seq, 0ull, &red_k[seq & 1u], true, poll_limit, false);
      __syncthreads();
      if (red_k[seq & 1u] == ~0ull) {
        if (tid == 0 && A.status)
          for (int tj = ti; tj < A.team_off[team + 1]; ++tj) atomicOr(&A.status[A.team_imgs[tj]], 16);
        return;
      }
      const float ga = (float)A.cbeam[6 * img + 0], gb = (float)A.cbeam[6 * img + 1],
                  gc = (float)A.cbeam[6 * img + 2];
      const int rr = A.rrad[img];
      const int side = 2 * rr + 1;
      // the chunk goes through LDS in parts of sub pixels (sub a multiple of STEP or the
      // whole chunk); each part rescans the component list
      const int sub = chunk < A.sub_px ? chunk : A.sub_px;
      for (int p0 = 0; p0 < chunk; p0 += sub) {
        const int g_lo = c0 + p0, g_hi = g_lo + sub;   // this part: pixels [g_lo, g_hi)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int q = 4 * (tid + CL_THREADS * s);     // chunk-local index of the group
          if (s < smax && tvalid && q >= p0 && q < p0 + sub)
#pragma unroll
            for (int j = 0; j < 4; ++j) Rl[q - p0 + j] = R[4 * s + j];
        }
        __syncthreads();
        const int row_lo = g_lo >> log2N, row_hi = (g_hi - 1) >> log2N;
        for (int i = 0; i < it; ++i) {
          const int p = (int)ld_shared_u32<LOCAL>(reinterpret_cast<const unsigned*>(A.comp_idx + coff + i));
          const int cy = p >> log2N, cx = p & (N - 1);
          if (cy + rr < row_lo || cy - rr > row_hi) continue;
          const float fc = (float)__longlong_as_double(
              (long long)ld_shared_u64<LOCAL>(reinterpret_cast<const unsigned long long*>(A.comp_flux + coff + i)));
          for (int w = tid; w < side * side; w += CL_THREADS) {
            const int dy = w / side - rr, dx = w % side - rr;
            const int y = cy + dy, x = cx + dx;
            if (y < 0 || y >= N || x < 0 || x >= N) continue;
            const int g = (y << log2N) + x;
            if (g < g_lo || g >= g_hi) continue;
            const float e = (float)dx * (ga * (float)dx + gb * (float)dy) + gc * (float)dy * (float)dy;
            atomicAdd(&Rl[g - g_lo], fc * expf(-e));
          }
        }
        __syncthreads();
        float* rs = A.restored + d.img_off + g_lo;
        for (int q = tid; q < sub; q += CL_THREADS) rs[q] = Rl[q];
        __syncthreads();
      }
    }
  }
}

// ---- host launchers ----
// Windowed peak searches run a separate instantiation, so the unwindowed kernel's code and
// register allocation are untouched by the window tests.
#define MI_CLEAN_KERNEL(PPT, LOCAL)                                                     \
  (win ? reinterpret_cast<const void*>(&k_clean<PPT, LOCAL, true>)                    \
       : reinterpret_cast<const void*>(&k_clean<PPT, LOCAL, false>))

static const void* clean_kernel(int ppt, bool local, bool win) {
  switch (ppt) {
    case 4: return local ? MI_CLEAN_KERNEL(4, true) : MI_CLEAN_KERNEL(4, false);
    case 8: return local ? MI_CLEAN_KERNEL(8, true) : MI_CLEAN_KERNEL(8, false);
    case 16: return local ? MI_CLEAN_KERNEL(16, true) : MI_CLEAN_KERNEL(16, false);
    case 32: return local ? MI_CLEAN_KERNEL(32, true) : MI_CLEAN_KERNEL(32, false);
    case 64: return local ? MI_CLEAN_KERNEL(64, true) : MI_CLEAN_KERNEL(64, false);
    default: return nullptr;
  }
}

hipError_t clean_max_blocks_per_cu(int ppt, bool local, bool win, size_t lds, int* nb) {
  const void* k = clean_kernel(ppt, local, win);
  if (!k) return hipErrorInvalidValue;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, k, CL_THREADS, lds);
}

hipError_t launch_clean(const CleanArgs& A, int ppt, bool local, int n_blocks, size_t lds, hipStream_t st) {
  const void* k = clean_kernel(ppt, local, A.win != nullptr);
  if (!k) return hipErrorInvalidValue;
  CleanArgs a = A;
  void* args[] = {&a};
  return hipLaunchCooperativeKernel(k, dim3(n_blocks), dim3(CL_THREADS), args, lds, st);
}

}  // namespace mi
