// Internal definitions shared by the HIP kernels and the host library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mi {

// Gridding convolution function: prolate spheroidal, support W = 7 cells, alpha = 1,
// tabulated at OS = 128 points per cell (Sec. 3.2.3).
constexpr int W = 7;
constexpr int HALF_W = 3;             // taps d = -3..3
constexpr int OS = 128;
constexpr int TAB_CENTRE = OS * W / 2;  // 448
constexpr int TAB_LEN = 2 * TAB_CENTRE + 1;  // 897
constexpr int N_MIN = 64;
constexpr int N_MAX = 4096;
constexpr int P_MAX = 2 * N_MAX;      // largest transform length (beam grid)

// Gridding tiles on the half plane: TK lines (fixed u) x TJ cells along v.
constexpr int TK = 16;
constexpr int TJ = 64;
// Entries (sample, tile) per input visibility: 2 samples x at most 2 x 2 tiles.
constexpr int ENT_PER_VIS = 8;

// FFT kernels stage 4096 complex doubles in LDS per workgroup (8192 for P = 8192).
constexpr int FFT_ELEMS_SMALL = 4096;
constexpr int FFT_ELEMS_LARGE = 8192;
constexpr int CLEAN_RESTORE_SUB_PX = 32768;   // restore staging: 128 KB of LDS

// Per-instance descriptor, built on the host when a plan is created.
struct InstDesc {
  int64_t vis_off;     // first visibility
  int64_t img_off;     // N*N image offset (floats)
  int64_t beam_off;    // (2N)^2 beam offset (floats)
  int64_t gd_off;      // dirty half grid offset (complex): N/2 * N
  int64_t gb_off;      // beam half grid offset (elements): N * 2N per instance
  int64_t ent_off;     // entry-list offset (ENT_PER_VIS * n_vis per instance)
  int64_t cnt_off;     // uniform-weight count scratch offset (floats, N*N) or -1
  double scale;        // N * dl = 1 / du (u in wavelengths -> cells)
  int32_t n_vis;
  int32_t N;
  int32_t log2N;
  int32_t mode;        // 0 natural, 1 uniform
  int32_t tile_base_d; // first dirty tile of this instance
  int32_t tile_base_b; // first beam tile of this instance
  int32_t blk_base_d;  // first dirty line block (fused gridding + first transform pass)
  int32_t blk_base_b;  // first beam line block
};

// Device-side constant tables (computed on the host in FP64).
struct Tables {
  const double* tab;       // kernel table, TAB_LEN values, tab[TAB_CENTRE] = 1
  const double* tsum;      // sum_d T[d OS - o] for o = -OS/2..OS/2 (index o + OS/2)
  const double2* twiddle;  // exp(+2 pi i t / P_MAX), t = 0..P_MAX-1
  const double* inv_corr;  // 1/corr for every P = 64..8192: block for P starts at P - 64
  double inv_corr0_sq;     // 1 / corr(0)^2
};

// An entry of the fused gridding + first transform pass: one sample (or its Hermitian
// mirror) for one block of lines, with everything its taps need, read as two 16-byte loads.
struct GridRec {
  int cucv;        // (cu << 16) | (cv & 0xffff): the nearest cell (mirror: negated)
  int ouov;        // ((ou + OS/2) << 8) | (ov + OS/2): the oversampled offsets (mirror: negated)
  float w;         // the visibility's weight
  int pad0;
  float vr, vi;    // its value (mirror: conjugate); (1, 0) for the beam grid
  float pad1, pad2;
};

// FFT work item: instance and first line (pass A) or first row (pass B).
struct FftWork { int inst; int first; };

// Arguments of the persistent CLEAN kernel.
struct CleanArgs {
  const InstDesc* inst;
  const int* team_off;     // CSR of images per team
  const int* team_imgs;
  const int2* blk;         // per block: (team, member); team < 0: idle block
  const int* team_G;       // workgroups per team
  const int64_t* team_slot;  // first exchange slot of each team (2 G slots per team)
  const float* dirty;
  const float* beam;
  const int* niter;
  const float* thr;        // may be null (threshold 0)
  const int4* win;         // per instance peak-search box (x0, y0, x1, y1), or null: whole maps
  float gain;
  int posonly;
  const double* cbeam;     // 6 per instance (a, b, c, ...) or null: no restore
  const int* rrad;         // restore radius per instance
  float* resid;
  double* model;           // may be null
  const int64_t* comp_off; // first component slot per instance
  int* comp_idx;           // null only when neither components nor restore are wanted
  double* comp_flux;
  int* ncomp;              // may be null
  float* restored;         // may be null
  int sub_px;              // restore: residual pixels staged in LDS per pass (power of two)
  unsigned long long* slots;  // per team: 2 x G keys
  const int* asym;         // per instance: nonzero unless the beam is exactly point-symmetric
  int* status;             // may be null
  unsigned poll_limit;     // polls per team wait before giving up (0: the default)
  int test_stall;          // failure-path tests: member 0 never publishes, every wait times out
};

// Steer CLEAN: pixels per work item of its elementwise passes (4 per thread, 512 threads).
constexpr int ST_PIX_PER_ITEM = 2048;

// Disk centering: two maps of equal size share one complex transform (map a in the real
// part, map b in the imaginary part; b = -1 for a map left alone).
struct CorrSlot {
  int a, b;          // instances
  int N, log2N;
  int64_t off;       // element offset of the slot's N^2 complex values
};

// Steer CLEAN: per-instance layout of the workspaces (built on the host per plan).
struct SteerInst {
  int64_t x_off;     // blocked row spectra (complex, stored FP32): 2N rows x (N+1) columns
  int64_t s_off;     // spectrum of the beam / clean beam (complex, stored FP32): (N+1) columns x 2N
  int64_t ctl_off;   // u32 control words: [0], [1] peak keys by iteration parity, [2] max |D| key,
                     // [3] unused, [4 + k] pixels selected in iteration k
  int64_t log_off;   // doubles: (peak, alpha, count) per iteration
  int64_t mask_off;  // u32 words: N^2 / 32 per iteration (selection bit masks)
  int32_t ncycle;    // iteration cap
  int32_t rb;        // rows per block of the blocked spectra (power of two)
  float thr;         // host threshold (device thresholds override it)
  int32_t pad;
};

// Arguments of the Steer CLEAN kernels (one struct for all of them; each reads its part).
struct SteerArgs {
  const InstDesc* inst;
  const SteerInst* sti;
  const FftWork* work;     // this launch's work items
  const float* thr_dev;    // device thresholds or null
  float gain, trim;
  int posonly;
  int k;                   // iteration of this launch
  int iter;                // 1: an iteration launch (inactive instances skip it), 0: set-up / restore
  const float* dirty;
  const float* beam;
  const double* cbeam;     // clean-beam Gaussian (a, b, c, ...) per instance
  float* R;                // residual (the caller's output, updated in place)
  double* model;
  float* D;                // convolution of this iteration's components with the beam, N^2
  float2* X;               // spectra between the passes (transforms run in FP64 in LDS)
  float2* S;
  unsigned* ctl;
  double* log;             // or null
  unsigned* mask;          // or null
  int* ncyc_out;           // or null
  float* restored;
  Tables T;
};

// Round half away from zero, written as sign(x) floor(|x| + 1/2) in FP64 (identical
// arithmetic on every side that needs the same cell decisions).
__device__ __forceinline__ double rhaz(double x) {
  double a = floor(fabs(x) + 0.5);
  return x < 0.0 ? -a : a;
}

struct Sample {
  int cu, cv, ou, ov;      // N grid
  int cu2, cv2, ou2, ov2;  // 2N beam grid
  bool keep;
};

// Cell/offset decisions for one visibility.  The keep test is made in FP64 before any
// integer conversion, so non-finite or huge coordinates are simply dropped.
__device__ __forceinline__ Sample prep_sample(float u, float v, float w_in, double scale, int N) {
  Sample s;
  double gu = (double)u * scale, gv = (double)v * scale;
  double cu = rhaz(gu), cv = rhaz(gv);
  double lim = (double)(N / 2 - 1 - HALF_W);
  s.keep = (w_in > 0.0f) && (fabs(cu) <= lim) && (fabs(cv) <= lim);   // false for NaN
  if (!s.keep) {
    s.cu = s.cv = s.ou = s.ov = s.cu2 = s.cv2 = s.ou2 = s.ov2 = 0;
    return s;
  }
  s.cu = (int)cu;
  s.cv = (int)cv;
  s.ou = (int)rhaz((gu - cu) * (double)OS);
  s.ov = (int)rhaz((gv - cv) * (double)OS);
  double gu2 = 2.0 * gu, gv2 = 2.0 * gv;
  double cu2 = rhaz(gu2), cv2 = rhaz(gv2);
  s.cu2 = (int)cu2;
  s.cv2 = (int)cv2;
  s.ou2 = (int)rhaz((gu2 - cu2) * (double)OS);
  s.ov2 = (int)rhaz((gv2 - cv2) * (double)OS);
  return s;
}

}  // namespace mi
