// Disk centering and phase correction (gfx950), Sec. 4.2: the cleaned map is correlated
// with a simulated solar disk, the correlation peak gives the disk's offset from the field
// centre, and the visibilities' phases are corrected by that offset.  Choices the paper
// leaves open: a uniform disk of the given radius (pixels) centred on pixel (N/2, N/2);
// circular correlation C[d] = sum_x map[x] disk[x - d] through plain FP64 DFTs (the
// transforms run in k_fft.hip; two real maps of equal size share one complex transform,
// Z = A + i B, separated in the spectrum by Hermitian symmetry: A^(k) = (Z^(k) +
// conj Z^(-k)) / 2, B^(k) = (Z^(k) - conj Z^(-k)) / 2i, and the two correlations come back
// as the real and imaginary parts of one inverse transform); the peak is the largest Re C, ties to the lowest linear
// index, wrapped to [-N/2, N/2), refined per axis by the parabola through the peak and its
// neighbours; the correction multiplies each visibility by exp(+2 pi i (u dl + v dm)).
#include <algorithm>

#include "mi_internal.h"

namespace mi {

constexpr int CTR_THREADS = 1024;
constexpr int CTR_WAVES = CTR_THREADS / 64;

// map (float32, packed N^2 per instance) -> X (double2), disk model -> D (double2)
__global__ void __launch_bounds__(256)
k_corr_prep(const InstDesc* __restrict__ inst, const float* __restrict__ images, const double* __restrict__ radius_px,
            double2* __restrict__ X, double2* __restrict__ D) {
  const int i = blockIdx.y;
  const InstDesc d = inst[i];
  const int N = d.N, h = N / 2;
  const double r2 = radius_px[i] * radius_px[i];
  const int64_t n = (int64_t)N * N;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256) {
    const int y = (int)(q >> d.log2N), x = (int)(q & (N - 1));
    const double dx = x - h, dy = y - h;
    if (X) X[d.img_off + q] = make_double2((double)images[d.img_off + q], 0.0);          // null: maps paired
    if (D) D[d.img_off + q] = make_double2(dx * dx + dy * dy <= r2 ? 1.0 : 0.0, 0.0);   // null: model cached
  }
}

// maps of a slot -> Z = A + i B (double2)
__global__ void __launch_bounds__(256)
k_corr_prep_pair(const CorrSlot* __restrict__ slots, const InstDesc* __restrict__ inst, const float* __restrict__ images,
                 double2* __restrict__ Z) {
  const CorrSlot sl = slots[blockIdx.y];
  const int64_t n = (int64_t)sl.N * sl.N;
  const float* a = images + inst[sl.a].img_off;
  const float* b = sl.b >= 0 ? images + inst[sl.b].img_off : nullptr;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
    Z[sl.off + q] = make_double2((double)a[q], b ? (double)b[q] : 0.0);
}

// W = A^ conj(DA) + i B^ conj(DB) from the slot's spectrum Z^ (out of place: Z^(-k) is read
// by another thread); a slot with one map has Z^ = A^.
__global__ void __launch_bounds__(256)
k_corr_mul_pair(const CorrSlot* __restrict__ slots, const InstDesc* __restrict__ inst, const double2* __restrict__ Z,
                const double2* __restrict__ D, double2* __restrict__ W) {
  const CorrSlot sl = slots[blockIdx.y];
  const int N = sl.N;
  const int64_t n = (int64_t)N * N;
  const double2* z = Z + sl.off;
  const double2* da = D + inst[sl.a].img_off;
  const double2* db = sl.b >= 0 ? D + inst[sl.b].img_off : nullptr;
  double2* w = W + sl.off;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256) {
    const double2 zk = z[q], ea = da[q];
    if (!db) {
      w[q] = make_double2(zk.x * ea.x + zk.y * ea.y, zk.y * ea.x - zk.x * ea.y);
      continue;
    }
    const int ky = (int)(q >> sl.log2N), kx = (int)(q & (N - 1));
    const double2 zm = z[(int64_t)((N - ky) & (N - 1)) * N + ((N - kx) & (N - 1))];
    const double2 fa = make_double2(0.5 * (zk.x + zm.x), 0.5 * (zk.y - zm.y));     // (Z + conj Zm) / 2
    const double2 fb = make_double2(0.5 * (zk.y + zm.y), 0.5 * (zm.x - zk.x));     // (Z - conj Zm) / 2i
    const double2 eb = db[q];
    const double2 pa = make_double2(fa.x * ea.x + fa.y * ea.y, fa.y * ea.x - fa.x * ea.y);   // A^ conj(DA)
    const double2 pb = make_double2(fb.x * eb.x + fb.y * eb.y, fb.y * eb.x - fb.x * eb.y);   // B^ conj(DB)
    w[q] = make_double2(pa.x - pb.y, pa.y + pb.x);                                      // pa + i pb
  }
}

namespace {
__device__ __forceinline__ double parabola(double cm, double c0, double cp) {
  const double den = cm - 2.0 * c0 + cp;
  return den < 0.0 ? (cm - cp) / (2.0 * den) : 0.0;
}
}  // namespace

// Peak of Re C per instance (one workgroup each) -> offsets (dl, dm) in radians.
__global__ void __launch_bounds__(CTR_THREADS)
k_corr_peak(const InstDesc* __restrict__ inst, const double2* __restrict__ C, const int64_t* __restrict__ c_off,
            double* __restrict__ offsets) {
  __shared__ double sv[CTR_WAVES];
  __shared__ int si[CTR_WAVES];
  const int i = blockIdx.x;
  const InstDesc d = inst[i];
  const int N = d.N;
  const int64_t n = (int64_t)N * N;
  // instance i's correlation: the real (c_off even) or imaginary (odd) part of its slot,
  // whose complex values start at c_off / 2
  const double* c = reinterpret_cast<const double*>(C + (c_off[i] >> 1)) + (c_off[i] & 1);
  double best = -INFINITY;
  int bi = 0x7fffffff;
  for (int64_t q = threadIdx.x; q < n; q += CTR_THREADS) {
    const double v = c[2 * q];
    if (v > best) { best = v; bi = (int)q; }     // ascending q per thread: first maximum kept
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(best, o);
    const int oi = __shfl_xor(bi, o);
    if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { sv[wave] = best; si[wave] = bi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    best = sv[0];
    bi = si[0];
    for (int w = 1; w < CTR_WAVES; ++w)
      if (sv[w] > best || (sv[w] == best && si[w] < bi)) { best = sv[w]; bi = si[w]; }
    const int py = bi >> d.log2N, px = bi & (N - 1);
    const double c0 = c[2 * (int64_t)bi];
    const double fx = parabola(c[2 * ((int64_t)py * N + ((px - 1) & (N - 1)))], c0,
                               c[2 * ((int64_t)py * N + ((px + 1) & (N - 1)))]);
    const double fy = parabola(c[2 * ((int64_t)((py - 1) & (N - 1)) * N + px)], c0,
                               c[2 * ((int64_t)((py + 1) & (N - 1)) * N + px)]);
    const int ix = px >= N / 2 ? px - N : px, iy = py >= N / 2 ? py - N : py;
    const double cell = d.scale / (double)N;
    offsets[2 * i] = ((double)ix + fx) * cell;
    offsets[2 * i + 1] = ((double)iy + fy) * cell;
  }
}

// vis *= exp(+2 pi i (u dl + v dm)), FP64 phase, per instance offsets on the device.
__global__ void __launch_bounds__(256)
k_phase_shift(const InstDesc* __restrict__ inst, float2* __restrict__ vis, const float2* __restrict__ uv,
              const double* __restrict__ offsets) {
  const int i = blockIdx.y;
  const InstDesc d = inst[i];
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= d.n_vis) return;
  const int64_t vi = d.vis_off + k;
  const float2 q = uv[vi];
  const double ph = 2.0 * 3.14159265358979323846 * ((double)q.x * offsets[2 * i] + (double)q.y * offsets[2 * i + 1]);
  double sn, cs;
  sincos(ph, &sn, &cs);
  const float2 v = vis[vi];
  vis[vi] = make_float2((float)((double)v.x * cs - (double)v.y * sn), (float)((double)v.x * sn + (double)v.y * cs));
}

hipError_t launch_corr_prep(const InstDesc* inst, int n_inst, int max_N, const float* images, const double* radius_px,
                            double2* X, double2* D, hipStream_t st) {
  const int blocks = std::max(1, std::min(1024, max_N * max_N / 2048));
  hipLaunchKernelGGL(k_corr_prep, dim3(blocks, n_inst), dim3(256), 0, st, inst, images, radius_px, X, D);
  return hipGetLastError();
}
hipError_t launch_corr_peak(const InstDesc* inst, int n_inst, const double2* C, const int64_t* c_off, double* offsets,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_corr_peak, dim3(n_inst), dim3(CTR_THREADS), 0, st, inst, C, c_off, offsets);
  return hipGetLastError();
}
hipError_t launch_corr_prep_pair(const CorrSlot* slots, int n_slots, const InstDesc* inst, int max_N, const float* images,
                                 double2* Z, hipStream_t st) {
  const int blocks = std::max(1, std::min(1024, max_N * max_N / 2048));
  hipLaunchKernelGGL(k_corr_prep_pair, dim3(blocks, n_slots), dim3(256), 0, st, slots, inst, images, Z);
  return hipGetLastError();
}
hipError_t launch_corr_mul_pair(const CorrSlot* slots, int n_slots, const InstDesc* inst, int max_N, const double2* Z,
                                const double2* D, double2* W, hipStream_t st) {
  const int blocks = std::max(1, std::min(1024, max_N * max_N / 2048));
  hipLaunchKernelGGL(k_corr_mul_pair, dim3(blocks, n_slots), dim3(256), 0, st, slots, inst, Z, D, W);
  return hipGetLastError();
}
hipError_t launch_phase_shift(const InstDesc* inst, int n_inst, int max_nvis, float2* vis, const float2* uv,
                              const double* offsets, hipStream_t st) {
  if (max_nvis <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_phase_shift, dim3((max_nvis + 255) / 256, n_inst), dim3(256), 0, st, inst, vis, uv, offsets);
  return hipGetLastError();
}

}  // namespace mi
