// Host-side FP64 construction of the gridding convolution function tables.
//
// Sec. 3.2.3 names a truncated prolate spheroidal gridding function (Schwab) without
// printing its coefficients.  It is computed here from its defining eigen-problem:
//   integral_{-1}^{1} (1 - t^2)^alpha cos(c nu t) psi(t) dt = lambda psi(nu),
// discretised by Nystrom on Gauss-Legendre nodes and solved by cyclic Jacobi rotations of
// the symmetrised matrix; the leading (largest) eigenpair gives psi.  Then
//   C(D) = (1 - (2D/W)^2)^alpha psi(2D/W),  T[t] = C(t/OS) / C(0),
//   corr_P(x') = (1/OS) sum_t T[t] cos(2 pi t x' / (OS P))       (grid correction),
//   Tsum(o) = sum_d T[d OS - o]                                      (B0 normalisation).
#include <cmath>
#include <vector>

#include "mi_tables.h"

namespace mi {

namespace {

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;                    // P_0, P_1
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);     // P_n'(z)
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Eigen-decomposition of a symmetric matrix a (n x n, row-major) by cyclic Jacobi.
void jacobi_eigen(int n, std::vector<double>& a, std::vector<double>& evals, std::vector<double>& v) {
  v.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int p = 0; p < n; ++p) {
      diag += a[(size_t)p * n + p] * a[(size_t)p * n + p];
      for (int q = p + 1; q < n; ++q) off += a[(size_t)p * n + q] * a[(size_t)p * n + q];
    }
    if (off <= 1e-32 * diag) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[(size_t)p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {           // columns p, q
          const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
          a[(size_t)k * n + p] = c * akp - s * akq;
          a[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {           // rows p, q
          const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
          a[(size_t)p * n + k] = c * apk - s * aqk;
          a[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
          v[(size_t)k * n + p] = c * vkp - s * vkq;
          v[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  evals.resize(n);
  for (int i = 0; i < n; ++i) evals[i] = a[(size_t)i * n + i];
}

}  // namespace

HostTables build_host_tables(int W, int os, double alpha, int n_nodes) {
  HostTables H;
  const double c = M_PI * W / 2.0;
  std::vector<double> t, wq;
  gauss_legendre(n_nodes, t, wq);
  std::vector<double> d(n_nodes), sq(n_nodes);
  for (int k = 0; k < n_nodes; ++k) {
    d[k] = wq[k] * std::pow(1.0 - t[k] * t[k], alpha);
    sq[k] = std::sqrt(d[k]);
  }
  std::vector<double> a((size_t)n_nodes * n_nodes);
  for (int i = 0; i < n_nodes; ++i)
    for (int k = 0; k < n_nodes; ++k) a[(size_t)i * n_nodes + k] = sq[i] * std::cos(c * t[i] * t[k]) * sq[k];
  std::vector<double> ev, vec;
  jacobi_eigen(n_nodes, a, ev, vec);
  int lead = 0;
  for (int i = 1; i < n_nodes; ++i)
    if (ev[i] > ev[lead]) lead = i;
  const double lam = ev[lead];
  std::vector<double> psi_nodes(n_nodes);
  for (int k = 0; k < n_nodes; ++k) psi_nodes[k] = vec[(size_t)k * n_nodes + lead] / sq[k];
  // psi(nu) = (1/lambda) sum_k d_k cos(c nu t_k) psi(t_k)
  auto psi = [&](double nu) {
    double s = 0.0;
    for (int k = 0; k < n_nodes; ++k) s += d[k] * std::cos(c * nu * t[k]) * psi_nodes[k];
    return s / lam;
  };
  const int half = os * W / 2;
  std::vector<double> tab(2 * half + 1);
  for (int i = -half; i <= half; ++i) {
    const double eta = 2.0 * ((double)i / os) / W;
    const double e2 = 1.0 - eta * eta;
    tab[i + half] = e2 <= 0.0 ? 0.0 : std::pow(e2, alpha) * psi(eta);
  }
  const double t0 = tab[half];
  for (double& v : tab) v /= t0;
  H.tab = tab;
  // corr(0) and Tsum
  double s0 = 0.0;
  for (double v : tab) s0 += v;
  const double corr0 = s0 / os;
  H.corr0 = corr0;
  const int hw = (W - 1) / 2;
  H.tsum.assign(os + 1, 0.0);
  for (int o = -os / 2; o <= os / 2; ++o) {
    double s = 0.0;
    for (int dd = -hw; dd <= hw; ++dd) s += tab[dd * os - o + half];
    H.tsum[o + os / 2] = s;
  }
  // 1/corr for P = 64 .. 8192 (block for P starts at P - 64 in a flat array)
  H.inv_corr.assign(2 * 8192 - 64, 0.0);
  for (int P = 64; P <= 8192; P *= 2) {
    for (int x = 0; x <= P / 2; ++x) {
      const int xp = x - P / 2;            // <= 0; corr is even in x'
      double s = tab[half];
      for (int i = 1; i <= half; ++i) s += 2.0 * tab[half + i] * std::cos(2.0 * M_PI * i * xp / ((double)os * P));
      const double corr = s / os;
      H.inv_corr[(P - 64) + x] = 1.0 / corr;
      if (x > 0 && x < P / 2) H.inv_corr[(P - 64) + (P - x)] = 1.0 / corr;
    }
  }
  // twiddles exp(+2 pi i t / 8192)
  H.twiddle.resize(2 * 8192);
  for (int k = 0; k < 8192; ++k) {
    H.twiddle[2 * k] = std::cos(2.0 * M_PI * k / 8192.0);
    H.twiddle[2 * k + 1] = std::sin(2.0 * M_PI * k / 8192.0);
  }
  return H;
}

}  // namespace mi
