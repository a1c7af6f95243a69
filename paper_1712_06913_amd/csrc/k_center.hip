// Disk centering and phase correction (gfx950), Sec. 4.2: the cleaned map is correlated
// with a simulated solar disk, the correlation peak gives the disk's offset from the field
// centre, and the visibilities' phases are corrected by that offset.  Choices the paper
// leaves open: a uniform disk of the given radius (pixels) centred on pixel (N/2, N/2);
// circular correlation C[d] = sum_x map[x] disk[x - d] through plain FP64 DFTs (the
// transforms run in k_fft.hip); the peak is the largest Re C, ties to the lowest linear
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
    X[d.img_off + q] = make_double2((double)images[d.img_off + q], 0.0);
    if (D) D[d.img_off + q] = make_double2(dx * dx + dy * dy <= r2 ? 1.0 : 0.0, 0.0);   // null: model cached
  }
}

// A[q] *= conj(B[q])
__global__ void __launch_bounds__(256)
k_corr_mul(double2* __restrict__ A, const double2* __restrict__ B, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256) {
    const double2 a = A[q], b = B[q];
    A[q] = make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
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
k_corr_peak(const InstDesc* __restrict__ inst, const double2* __restrict__ C, double* __restrict__ offsets) {
  __shared__ double sv[CTR_WAVES];
  __shared__ int si[CTR_WAVES];
  const int i = blockIdx.x;
  const InstDesc d = inst[i];
  const int N = d.N;
  const int64_t n = (int64_t)N * N;
  const double2* c = C + d.img_off;
  double best = -INFINITY;
  int bi = 0x7fffffff;
  for (int64_t q = threadIdx.x; q < n; q += CTR_THREADS) {
    const double v = c[q].x;
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
    const double c0 = c[bi].x;
    const double fx = parabola(c[(int64_t)py * N + ((px - 1) & (N - 1))].x, c0, c[(int64_t)py * N + ((px + 1) & (N - 1))].x);
    const double fy = parabola(c[(int64_t)((py - 1) & (N - 1)) * N + px].x, c0, c[(int64_t)((py + 1) & (N - 1)) * N + px].x);
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
hipError_t launch_corr_mul(double2* A, const double2* B, int64_t n, hipStream_t st) {
  const int64_t blocks = std::min<int64_t>(65536, (n + 255) / 256);
  hipLaunchKernelGGL(k_corr_mul, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, st, A, B, n);
  return hipGetLastError();
}
hipError_t launch_corr_peak(const InstDesc* inst, int n_inst, const double2* C, double* offsets, hipStream_t st) {
  hipLaunchKernelGGL(k_corr_peak, dim3(n_inst), dim3(CTR_THREADS), 0, st, inst, C, offsets);
  return hipGetLastError();
}
hipError_t launch_phase_shift(const InstDesc* inst, int n_inst, int max_nvis, float2* vis, const float2* uv,
                              const double* offsets, hipStream_t st) {
  if (max_nvis <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_phase_shift, dim3((max_nvis + 255) / 256, n_inst), dim3(256), 0, st, inst, vis, uv, offsets);
  return hipGetLastError();
}

}  // namespace mi
