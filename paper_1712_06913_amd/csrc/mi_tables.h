// Host-side FP64 tables of the gridding convolution function (internal).
#pragma once
#include <vector>

namespace mi {

struct HostTables {
  std::vector<double> tab;       // T[t + OS W/2] = C(t/OS)/C(0)
  std::vector<double> tsum;      // Tsum(o), o = -OS/2..OS/2
  std::vector<double> inv_corr;  // 1/corr for P = 64..8192, block for P at offset P - 64
  std::vector<double> twiddle;   // interleaved cos/sin of 2 pi t / 8192
  double corr0 = 0.0;
};

HostTables build_host_tables(int W, int os, double alpha, int n_nodes);

}  // namespace mi
