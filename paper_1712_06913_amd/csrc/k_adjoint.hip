// Degridding: the prediction operator and the adjoint of the imaging operator (gfx950).
#include "mi_internal.h"

namespace mi {

__global__ void __launch_bounds__(256) k_degrid(const InstDesc* __restrict__ inst, const float2* __restrict__ uv,
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

hipError_t launch_degrid(const InstDesc* inst, int n_inst, int max_nvis, const float2* uv, const float* w_in,
                         const float* wts, const double* b0, const double2* fgrid, const Tables& T, int adjoint,
                         float2* out, hipStream_t st) {
  if (max_nvis <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_degrid, dim3((max_nvis + 255) / 256, n_inst), dim3(256), 0, st, inst, uv, w_in, wts, b0,
                     fgrid, T, adjoint, out);
  return hipGetLastError();
}

}  // namespace mi
