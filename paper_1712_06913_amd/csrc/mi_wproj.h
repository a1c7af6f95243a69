// Internal definitions of the w-projection gridder (not part of the ABI).
#pragma once

#include "mi_internal.h"

namespace mi {

constexpr int WP_M = 64;        // field points per axis in the kernel construction (minus one, symmetric)
constexpr int WP_OS = 16;       // kernel table points per cell
constexpr int WP_SMAX = 63;     // largest kernel support (cells)
constexpr int WP_ENT = 20;      // (sample, tile) entries per visibility: 2 samples x at most 5 x 2 tiles

// One w-plane of one (N, cell) group of instances.
struct WPlane {
  int N;            // image size of the group
  int S;            // support in cells (odd)
  double w;         // plane's w (wavelengths)
  double cell;      // pixel size dl (rad)
  int64_t off;      // first table entry (complex doubles); (S WP_OS + 1)^2 entries, [dv][du]
};

// Per instance: its group's plane 0, number of planes, plane spacing.
struct WInst {
  int plane0;
  int n_planes;
  double dw;
};

}  // namespace mi
