// C ABI of the imaging hot path: contexts, plans, argument validation, launches.
//
// The entry points follow Algorithm 1: dirty_image (gridding with natural/uniform
// weighting, inverse FFT, grid correction) returning the dirty image and dirty beam, and
// the CLEAN loop (Sec. 4.3) with restore; plus the adjoint (FFT then degrid).
//
// A plan is built the first time a batch descriptor is seen (keyed by its contents): it
// holds the per-instance device descriptors, tile/work maps and the workspace, so later
// calls with the same descriptor launch without allocating or synchronising.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/mi.h"
#include "mi_internal.h"
#include "mi_tables.h"
#include "mi_wproj.h"

namespace mi {


// launchers (defined next to their kernels)
hipError_t launch_bin(const InstDesc*, int, const float2*, const float*, const Tables&, float*, double*, int*, int*,
                      float*, int*, int*, int*, int*, int*, int*, int, int, int, int, int, const float2*, GridRec*,
                      GridRec*, size_t, hipStream_t);
hipError_t launch_grid(const InstDesc*, const int*, int, int, const float2*, const float2*, const float*,
                       const float*, const int*, const int*, const int*, const Tables&, double2*, int, int, hipStream_t);
hipError_t launch_grid_f32(const InstDesc*, const int*, int, int, const float2*, const float2*, const float*,
                           const float*, const int*, const int*, const int*, const Tables&, float2*, int, int,
                           hipStream_t);
hipError_t launch_expand_full(const InstDesc*, int, int, const double2*, float2*, const int64_t*, hipStream_t);
hipError_t launch_fill_u32(unsigned*, int64_t, unsigned, hipStream_t);
hipError_t launch_wtables(const WPlane*, int, const int2*, int, int, const Tables&, double2*, double2*, double2*,
                          hipStream_t);
hipError_t launch_bin_w(const InstDesc*, int, size_t, const float2*, const float*, const float*, const WInst*,
                       const WPlane*, int*, int*, int*, hipStream_t);
hipError_t launch_grid_wt(const InstDesc*, const int*, int, const float2*, const float2*, const float*, const float*,
                          const float*, const int*, const int*, const int*, const WInst*, const WPlane*,
                          const double2*, double2*, hipStream_t);
hipError_t launch_grid_real(const InstDesc*, const int*, int, const float2*, const float*, const float*, const int*,
                            const int*, const int*, const Tables&, double*, int, hipStream_t);
hipError_t launch_fft_a(int, int, const InstDesc*, const FftWork*, int, double2*, const Tables&, hipStream_t);
hipError_t launch_grid_fft_a(int, int, const InstDesc*, const FftWork*, int, const GridRec*, const int*, const int*,
                             double2*, const Tables&, hipStream_t);
hipError_t launch_grid_fft_a_real(int, int, const InstDesc*, const FftWork*, int, const GridRec*, const int*,
                                  const int*, double*, const Tables&, hipStream_t);
hipError_t launch_fft_b_c2r(int, int, const InstDesc*, const FftWork*, int, const double2*, const double*,
                            const Tables&, float*, hipStream_t);
hipError_t launch_fft_a_real(int, int, const InstDesc*, const FftWork*, int, double*, const Tables&, hipStream_t);
hipError_t launch_fft_b_c2r_sym(int, int, const InstDesc*, const FftWork*, int, const double*, const double*,
                                const Tables&, float*, hipStream_t);
hipError_t launch_fft_b_r2c(int, int, const InstDesc*, const FftWork*, int, const float*, const Tables&, double2*,
                            hipStream_t);
hipError_t launch_fft_a_fwd(int, int, const InstDesc*, const FftWork*, int, const Tables&, double2*, hipStream_t);
hipError_t launch_fft_c2c_t_f2d(int, const int*, const int64_t*, const FftWork*, int, const float2*, double2*,
                                const Tables&, double, int, int, hipStream_t);
hipError_t launch_fft_c2c_t_d2f(int, const int*, const int64_t*, const FftWork*, int, const double2*, float2*,
                                const Tables&, double, int, int, hipStream_t);
hipError_t clean_max_blocks_per_cu(int ppt, bool local, bool win, size_t lds, int* nb);
hipError_t launch_clean(const CleanArgs&, int ppt, bool local, int n_blocks, size_t lds, hipStream_t);
hipError_t launch_beamfit(const InstDesc*, int, const float*, double*, int*, int*, hipStream_t);
hipError_t launch_gmm(const InstDesc*, int, const float*, int, int, double*, float*, float*, hipStream_t);
hipError_t launch_fft_c2c_t_d2d(int, const int*, const int64_t*, const FftWork*, int, const double2*, double2*,
                                const Tables&, double, int, int, hipStream_t);
hipError_t launch_corr_prep(const InstDesc*, int, int, const float*, const double*, double2*, double2*, hipStream_t);
hipError_t launch_corr_peak(const InstDesc*, int, const double2*, const int64_t*, double*, hipStream_t);
hipError_t launch_corr_prep_pair(const CorrSlot*, int, const InstDesc*, int, const float*, double2*, hipStream_t);
hipError_t launch_corr_mul_pair(const CorrSlot*, int, const InstDesc*, int, const double2*, const double2*, double2*,
                                hipStream_t);
hipError_t launch_phase_shift(const InstDesc*, int, int, float2*, const float2*, const double*, hipStream_t);
hipError_t launch_beam_symcheck(const InstDesc*, int, int, const float*, int*, hipStream_t);
hipError_t launch_degrid(const InstDesc*, int, int, const float2*, const float*, const float*, const double*,
                         const double2*, const Tables&, int, float2*, hipStream_t);
hipError_t launch_st_rows(int mode, int elems, int n_blocks, const SteerArgs& A, hipStream_t st);
hipError_t launch_st_cols(int mode, int elems, int n_blocks, const SteerArgs& A, hipStream_t st);
hipError_t launch_st_rows_inv(int mode, int elems, int n_blocks, const SteerArgs& A, hipStream_t st);
hipError_t launch_st_init(int n_blocks, const SteerArgs& A, hipStream_t st);
hipError_t launch_st_update(int n_blocks, const SteerArgs& A, hipStream_t st);

// LDS block (complex doubles) used by the FFT kernels for a transform of length P, and
// the lines (pass A) / rows (pass B) it holds.
int fft_elems_for(int P) { return P > FFT_ELEMS_SMALL ? FFT_ELEMS_LARGE : FFT_ELEMS_SMALL; }
int fft_lines_per_block_host(int P, int elems) {
  int nl = elems / P;
  return nl > P / 2 ? P / 2 : nl;
}
// Real lines per workgroup of the beam's pass A (two real lines per complex line).
int fft_real_lines_per_block_host(int P, int elems) {
  int nr = 2 * elems / P;
  return nr > P / 2 ? P / 2 : nr;
}
// Image rows per workgroup of the real-valued passes (two rows per complex line).
int fft_rows_per_block_host(int P, int elems) {
  int ny = 2 * elems / P;
  return ny > P ? P : ny;
}

// --------------------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() { if (p) (void)hipFree(p); }
};

struct MiError {
  mi_status code;
  std::string msg;
};

[[noreturn]] void fail(mi_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  throw MiError{code, buf};
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) fail(MI_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

template <class T>
T* dev_alloc(DevBuf& b, size_t count) {
  size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  if (b.bytes >= bytes) return static_cast<T*>(b.p);
  if (b.p) { (void)hipFree(b.p); b.p = nullptr; b.bytes = 0; }
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) { b.p = nullptr; fail(MI_ERR_NOMEM, "hipMalloc(%zu bytes) failed", bytes); }
  b.bytes = bytes;
  return static_cast<T*>(b.p);
}

template <class T>
T* upload(DevBuf& b, const std::vector<T>& h) {
  T* d = dev_alloc<T>(b, h.size());
  if (!h.empty()) HIPCHK(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
  return h;
}

// Cached plans are evicted least-recently-used first.  A plan used while its stream is
// being captured into a graph is pinned: the graph holds raw pointers into its buffers,
// so it stays until the context is destroyed.
struct CacheEntry {
  uint64_t last_use = 0;
  bool pinned = false;
};

struct CleanPlan : CacheEntry {
  std::vector<int32_t> niter;
  std::vector<float> thr;
  bool has_thr = false;
  std::vector<int32_t> win;   // 4 per instance, empty: whole maps
  int T = 0, local = 1, n_blocks = 0, ppt = 0, team_req = 0, sub_px = 0;
  int64_t n_slots = 0;
  size_t lds = 0;        // restore staging: sub_px floats
  int64_t total_comp = 0;
  DevBuf team_off, team_imgs, blk, team_G, team_slot, niter_d, thr_d, win_d, comp_off, slots, asym, comp_idx,
      comp_flux, cbeam, rrad;
};

// Steer CLEAN: per batch, the work lists of its passes and the workspaces; per parameter
// set (iteration caps, host thresholds), the per-instance descriptors and control words.
struct SteerBase {
  DevBuf rows, rows2, cols, inv, pix;    // FftWork lists: N rows, 2N rows, columns, N rows, pixel blocks
  int n_rows = 0, n_rows2 = 0, n_cols = 0, n_inv = 0, n_pix = 0;
  int elems = 4096;                      // complex doubles per workgroup of the transform passes
  std::vector<int64_t> x_off, s_off;
  std::vector<int32_t> rb;
  int64_t total_x = 0, total_s = 0;
  DevBuf X, S, D, model_ws;
};

struct SteerPlan : CacheEntry {
  std::vector<int32_t> ncycle;
  std::vector<float> thr;
  bool has_thr = false;
  int kmax = 0;
  int64_t total_ctl = 0;
  DevBuf sti, ctl, cbeam, rrad;
};

struct Plan : CacheEntry {
  // key (with the context's transform block size, which shapes the work lists)
  int fft_elems_req = 0;
  std::vector<int64_t> off;
  std::vector<int32_t> n;
  std::vector<double> cell;
  std::vector<int8_t> mode;
  int n_inst = 0;
  int64_t total_vis = 0;
  int max_N = 0, max_nvis = 0;
  std::vector<InstDesc> h_inst;
  int64_t total_img = 0, total_beam = 0, total_gd = 0, total_gb = 0, total_ent = 0, total_cnt = 0;
  int tiles_d = 0, tiles_b = 0;
  size_t bin_lds = 0;
  int n_wa_d = 0, n_wb_d = 0, n_wa_b = 0, n_wb_b = 0;
  int elems_d = FFT_ELEMS_SMALL, elems_b = FFT_ELEMS_SMALL;
  DevBuf inst, tile_inst_d, tile_inst_b, wa_d, wb_d, wa_b, wb_b;
  // workspace
  // gd: dirty half grids (FP64 complex); gbr: beam half grids (FP64 real), then the beam's
  // transform slots in place; gb: FP64 complex beam grids for mi_grid's full layout
  DevBuf wts, b0, nkept, cnt, ent_d, ent_b, ts_d, tc_d, ts_b, tc_b, gd, gbr, gb, status_ws;
  // fused gridding + first transform pass (every instance's blocks hold >= 2 lines, so a
  // sample's 7 lines touch at most 4 blocks): per line block entry lists
  bool fused = false;
  DevBuf bs_d, bc_d, bs_b, bc_b, rec_d, rec_b;
  // element offsets of each instance's grid in mi_grid's full layout: dirty grids; beam
  // grids after all dirty grids; beam grids alone (3 n_inst values, uploaded with the plan)
  DevBuf full_off;
  DevBuf b0_two;      // 2.0 per grid: pass B then scales by 1/2 (transpose of the prediction)
  std::map<uint64_t, std::unique_ptr<CleanPlan>> cleans;
  // w-projection: plane plan and kernel tables for one (w_max, tolerance) set
  struct WProj {
    std::vector<double> w_max;
    double tol = 0.0;
    std::vector<int32_t> n_planes;   // per instance
    DevBuf planes, rows, winst, screen, dft, tabs, ent, ts, tc;
  };
  std::unique_ptr<WProj> wproj;
  std::unique_ptr<SteerBase> steer;
  std::map<uint64_t, std::unique_ptr<SteerPlan>> steers;
  // disk centering: radii (host copy for change detection), 2-D transform work list, buffers
  std::vector<double> radius;
  int corr_elems = 0, corr_nwork = 0;
  bool corr_model_ready = false;      // corr_d holds the disk models' transforms for `radius`
  DevBuf radius_d, corr_n, corr_offs, corr_work, corr_x, corr_d, corr_s, offsets_ws;
  // the maps' transforms: two maps of equal N per slot
  int corr_nslots = 0, corr_snwork = 0;
  int64_t corr_slot_total = 0;
  DevBuf corr_slots, corr_sn, corr_soffs, corr_swork, corr_coff;
};

struct IfftPlan : CacheEntry {
  std::vector<int32_t> n;
  std::vector<int64_t> offs;
  int64_t total = 0;
  int n_work1 = 0;
  int elems = FFT_ELEMS_SMALL;
  DevBuf n_d, offs_d, work;
};

}  // namespace mi

struct mi_ctx {
  int device = 0;
  std::string err;
  mi::Tables T{};
  mi::DevBuf tab, tsum, tw, icorr;
  std::map<uint64_t, std::unique_ptr<mi::Plan>> plans;
  std::map<uint64_t, std::unique_ptr<mi::IfftPlan>> ifft_plans;
  mi::DevBuf ifft_scratch;
  unsigned char* noalloc_scratch = nullptr;   // this device's copy of the static CLEAN scratch
  int fail_inst = -1;
  int clean_stall = 0;   // failure-path tests (MI_TEST_CLEAN_STALL): CLEAN team waits give up
  int grid_chunk = 8;    // gridder tiles per workgroup (mi_set_tuning)
  int fft_elems = 0;     // transform points per workgroup, 0 = by size (mi_set_tuning)
  int n_cu = 256;
  uint64_t tick = 0;     // plan-cache clock (least recently used is evicted first)
  // kernel timing: event pairs around launches of the kinds in prof_kinds (MI_PROF_*)
  uint32_t prof_kinds = 0;
  size_t prof_used = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev;
  std::vector<uint32_t> prof_kind;
  ~mi_ctx() {
    for (auto& e : prof_ev) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  }
};

namespace mi {
namespace {

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIPCHK(hipStreamIsCapturing(st, &cs));
  return cs != hipStreamCaptureStatusNone;
}

// Marks a cached plan as used now (pinned for good when the stream is being captured).
void touch(mi_ctx* ctx, CacheEntry* e, hipStream_t st) {
  e->last_use = ++ctx->tick;
  if (capturing(st)) e->pinned = true;
}

// Makes room for one more entry in a plan cache of at most `cap` unpinned entries: evicts
// the least recently used unpinned plan.  A new plan allocates and uploads, which a graph
// capture cannot record, so creating one while capturing is an error.
template <class M>
void make_room(M& cache, size_t cap, hipStream_t st) {
  if (capturing(st))
    fail(MI_ERR_UNSUPPORTED, "a call with new arguments cannot be captured: run it once outside the capture first");
  size_t unpinned = 0;
  for (auto& kv : cache) unpinned += kv.second->pinned ? 0 : 1;
  if (unpinned < cap) return;
  auto victim = cache.end();
  for (auto it = cache.begin(); it != cache.end(); ++it)
    if (!it->second->pinned && (victim == cache.end() || it->second->last_use < victim->second->last_use)) victim = it;
  if (victim != cache.end()) cache.erase(victim);
}

// Kernel timing: when `kind` is being recorded, record the start event of a fresh pair on
// the stream and return the pair's end event (to be recorded after the launch); else null.
hipEvent_t prof_start(mi_ctx* ctx, uint32_t kind, hipStream_t st) {
  if (!(ctx->prof_kinds & kind)) return nullptr;
  if (ctx->prof_used == ctx->prof_ev.size()) {
    std::pair<hipEvent_t, hipEvent_t> e{};
    HIPCHK(hipEventCreate(&e.first));
    HIPCHK(hipEventCreate(&e.second));
    ctx->prof_ev.push_back(e);
    ctx->prof_kind.push_back(0u);
  }
  const size_t i = ctx->prof_used++;
  ctx->prof_kind[i] = kind;
  HIPCHK(hipEventRecord(ctx->prof_ev[i].first, st));
  return ctx->prof_ev[i].second;
}

void prof_stop(hipEvent_t e, hipStream_t st) {
  if (e) HIPCHK(hipEventRecord(e, st));
}
int ilog2i(int v) { int r = 0; while ((1 << r) < v) ++r; return r; }

void check_batch(const mi_batch* b) {
  if (!b) fail(MI_ERR_ARG, "batch is NULL");
  if (b->n_inst < 1) fail(MI_ERR_ARG, "batch->n_inst must be >= 1 (got %d)", b->n_inst);
  if (!b->vis_offset || !b->n_img || !b->cell_rad || !b->weight_mode)
    fail(MI_ERR_ARG, "batch host arrays (vis_offset, n_img, cell_rad, weight_mode) must not be NULL");
  if (b->vis_offset[0] != 0) fail(MI_ERR_SHAPE, "vis_offset[0] must be 0");
  for (int i = 0; i < b->n_inst; ++i) {
    const int N = b->n_img[i];
    if (!is_pow2(N) || N < N_MIN || N > N_MAX)
      fail(MI_ERR_SHAPE, "n_img[%d] = %d is not a power of two in [%d, %d]", i, N, N_MIN, N_MAX);
    if (!(b->cell_rad[i] > 0.0) || !std::isfinite(b->cell_rad[i]))
      fail(MI_ERR_ARG, "cell_rad[%d] must be finite and > 0", i);
    if (b->weight_mode[i] != MI_NATURAL && b->weight_mode[i] != MI_UNIFORM)
      fail(MI_ERR_ARG, "weight_mode[%d] = %d is not MI_NATURAL or MI_UNIFORM", i, (int)b->weight_mode[i]);
    const int64_t cnt = b->vis_offset[i + 1] - b->vis_offset[i];
    if (cnt < 0) fail(MI_ERR_SHAPE, "vis_offset must be non-decreasing (instance %d)", i);
    if (cnt > (1 << 27)) fail(MI_ERR_SHAPE, "instance %d has %lld visibilities (max 2^27)", i, (long long)cnt);
  }
}

Plan* get_plan(mi_ctx* ctx, const mi_batch* b, hipStream_t st) {
  check_batch(b);
  const int n = b->n_inst;
  uint64_t h = fnv1a(&n, sizeof n);
  h = fnv1a(b->vis_offset, sizeof(int64_t) * (n + 1), h);
  h = fnv1a(b->n_img, sizeof(int32_t) * n, h);
  h = fnv1a(b->cell_rad, sizeof(double) * n, h);
  h = fnv1a(b->weight_mode, sizeof(int8_t) * n, h);
  h = fnv1a(&ctx->fft_elems, sizeof ctx->fft_elems, h);
  auto it = ctx->plans.find(h);
  if (it != ctx->plans.end()) {
    Plan* p = it->second.get();
    if (p->n_inst == n && p->fft_elems_req == ctx->fft_elems && std::equal(p->off.begin(), p->off.end(), b->vis_offset) &&
        std::equal(p->n.begin(), p->n.end(), b->n_img) && std::equal(p->cell.begin(), p->cell.end(), b->cell_rad) &&
        std::equal(p->mode.begin(), p->mode.end(), b->weight_mode)) {
      touch(ctx, p, st);
      return p;
    }
    // another descriptor with the same key (a hash collision): replace it
    if (p->pinned) fail(MI_ERR_UNSUPPORTED, "plan cache collision with a plan held by a captured graph");
    ctx->plans.erase(it);
  }
  make_room(ctx->plans, 16, st);
  auto P = std::make_unique<Plan>();
  P->n_inst = n;
  P->off.assign(b->vis_offset, b->vis_offset + n + 1);
  P->n.assign(b->n_img, b->n_img + n);
  P->cell.assign(b->cell_rad, b->cell_rad + n);
  P->mode.assign(b->weight_mode, b->weight_mode + n);
  P->total_vis = P->off[n];
  P->h_inst.resize(n);
  std::vector<int> tile_inst_d, tile_inst_b;
  std::vector<FftWork> wa_d, wb_d, wa_b, wb_b;
  // first-pass work items per instance, dealt out line block by line block over the
  // instances: the blocks around u = 0 hold most of the gridding records, and in instance
  // order they would all fall to the same few persistent workgroups
  std::vector<std::vector<FftWork>> pa_d(n), pa_b(n);
  int32_t blocks_d = 0, blocks_b = 0;
  int max_tiles = 0;
  int maxN = 0;
  for (int i = 0; i < n; ++i) maxN = std::max(maxN, (int)b->n_img[i]);
  P->fft_elems_req = ctx->fft_elems;
  P->elems_d = std::max(ctx->fft_elems, fft_elems_for(maxN));
  P->elems_b = std::max(ctx->fft_elems, fft_elems_for(2 * maxN));
  bool fused = true;
  for (int i = 0; i < n; ++i) {
    InstDesc& d = P->h_inst[i];
    std::memset(&d, 0, sizeof d);
    const int N = P->n[i];
    d.vis_off = P->off[i];
    d.n_vis = (int32_t)(P->off[i + 1] - P->off[i]);
    d.N = N;
    d.log2N = ilog2i(N);
    d.mode = P->mode[i];
    d.scale = (double)N * P->cell[i];
    d.img_off = P->total_img;
    d.beam_off = P->total_beam;
    d.gd_off = P->total_gd;
    d.gb_off = P->total_gb;
    d.ent_off = P->total_ent;
    d.cnt_off = d.mode == MI_UNIFORM ? P->total_cnt : -1;
    d.tile_base_d = P->tiles_d;
    d.tile_base_b = P->tiles_b;
    P->total_img += (int64_t)N * N;
    P->total_beam += 4LL * N * N;
    P->total_gd += (int64_t)N * N / 2;
    P->total_gb += 2LL * N * N;
    P->total_ent += (int64_t)ENT_PER_VIS * d.n_vis;
    if (d.mode == MI_UNIFORM) P->total_cnt += (int64_t)N * N;
    const int ntd = (N / 2 / TK) * (N / TJ), ntb = (N / TK) * (2 * N / TJ);
    P->tiles_d += ntd;
    P->tiles_b += ntb;
    max_tiles = std::max(max_tiles, std::max(ntd, ntb));
    for (int t = 0; t < ntd; ++t) tile_inst_d.push_back(i);
    for (int t = 0; t < ntb; ++t) tile_inst_b.push_back(i);
    const int nld = fft_lines_per_block_host(N, P->elems_d), nrb = fft_real_lines_per_block_host(2 * N, P->elems_b);
    // line blocks are numbered instance by instance (the gridding records' block index)
    d.blk_base_d = blocks_d;
    d.blk_base_b = blocks_b;
    fused = fused && nld >= 2 && nrb >= 2;
    const int nyd = fft_rows_per_block_host(N, P->elems_d), nyb = fft_rows_per_block_host(2 * N, P->elems_b);
    for (int l = 0; l < N / 2; l += nld, ++blocks_d) pa_d[i].push_back({i, l});
    for (int y = 0; y < N; y += nyd) wb_d.push_back({i, y});
    for (int l = 0; l < N; l += nrb, ++blocks_b) pa_b[i].push_back({i, l});   // beam: N real lines
    for (int y = 0; y <= N; y += nyb) wb_b.push_back({i, y});       // beam: rows 0..N
    P->max_N = std::max(P->max_N, N);
    P->max_nvis = std::max(P->max_nvis, d.n_vis);
  }
  for (size_t k = 0;; ++k) {
    bool any = false;
    for (int i = 0; i < n; ++i) {
      if (k < pa_d[i].size()) { wa_d.push_back(pa_d[i][k]); any = true; }
      if (k < pa_b[i].size()) { wa_b.push_back(pa_b[i][k]); any = true; }
    }
    if (!any) break;
  }
  if (P->total_ent >= (1LL << 31)) fail(MI_ERR_SHAPE, "batch too large: %lld gridding entries", (long long)P->total_ent);
  P->bin_lds = (size_t)max_tiles * sizeof(int);
  if (P->bin_lds > 140 * 1024) fail(MI_ERR_UNSUPPORTED, "tile count per instance too large");
  upload(P->inst, P->h_inst);
  upload(P->tile_inst_d, tile_inst_d);
  upload(P->tile_inst_b, tile_inst_b);
  upload(P->wa_d, wa_d);
  upload(P->wb_d, wb_d);
  upload(P->wa_b, wa_b);
  upload(P->wb_b, wb_b);
  P->fused = fused;
  P->n_wa_d = (int)wa_d.size();
  P->n_wb_d = (int)wb_d.size();
  P->n_wa_b = (int)wa_b.size();
  P->n_wb_b = (int)wb_b.size();
  {
    // full-layout grid offsets for mi_grid (which = 0 / 2: dirty then beam; which = 1: beam alone)
    std::vector<int64_t> fo(3 * (size_t)n);
    int64_t sd = 0, sb = 0;
    for (int i = 0; i < n; ++i) { fo[i] = sd; sd += (int64_t)P->n[i] * P->n[i]; }
    for (int i = 0; i < n; ++i) {
      fo[n + i] = sd + sb;
      fo[2 * n + i] = sb;
      sb += 4LL * P->n[i] * P->n[i];
    }
    upload(P->full_off, fo);
  }
  Plan* raw = P.get();
  touch(ctx, raw, st);
  ctx->plans[h] = std::move(P);
  return raw;
}

// Prep + weights + B0 + binning (k_bin).  Returns the status pointer used.
// Prep, weights, B0 and the entry lists: per tile for the tiled gridder, or per line block
// (blocks = true) for the fused gridding + first transform pass.
int* run_bin(mi_ctx* ctx, Plan* P, const mi_batch* b, const float* uv, const float* w_in, bool beam,
             hipStream_t st, bool unit_w = false, bool blocks = false, const mi_c64* vis = nullptr) {
  float* wts = dev_alloc<float>(P->wts, P->total_vis);
  double* b0 = dev_alloc<double>(P->b0, 2 * P->n_inst);
  int* nk = dev_alloc<int>(P->nkept, P->n_inst);
  float* cnt = dev_alloc<float>(P->cnt, P->total_cnt);
  int* ed = dev_alloc<int>(P->ent_d, P->total_ent);
  int* eb = beam ? dev_alloc<int>(P->ent_b, P->total_ent) : nullptr;
  int *tsd, *tcd, *tsb = nullptr, *tcb = nullptr;
  GridRec *rd = nullptr, *rb = nullptr;
  if (blocks) {
    rd = dev_alloc<GridRec>(P->rec_d, P->total_ent);
    if (beam) rb = dev_alloc<GridRec>(P->rec_b, P->total_ent);
    tsd = dev_alloc<int>(P->bs_d, P->n_wa_d);
    tcd = dev_alloc<int>(P->bc_d, P->n_wa_d);
    if (beam) {
      tsb = dev_alloc<int>(P->bs_b, P->n_wa_b);
      tcb = dev_alloc<int>(P->bc_b, P->n_wa_b);
    }
  } else {
    tsd = dev_alloc<int>(P->ts_d, P->tiles_d);
    tcd = dev_alloc<int>(P->tc_d, P->tiles_d);
    if (beam) {
      tsb = dev_alloc<int>(P->ts_b, P->tiles_b);
      tcb = dev_alloc<int>(P->tc_b, P->tiles_b);
    }
  }
  int* status = b->status ? b->status : dev_alloc<int>(P->status_ws, P->n_inst);
  HIPCHK(launch_bin(static_cast<const InstDesc*>(P->inst.p), P->n_inst, reinterpret_cast<const float2*>(uv), w_in,
                    ctx->T, wts, b0, nk, status, cnt, ed, eb, tsd, tcd, tsb, tcb, ctx->fail_inst, beam ? 1 : 0,
                    unit_w ? 1 : 0, blocks ? P->elems_d : 0, blocks ? P->elems_b : 0,
                    reinterpret_cast<const float2*>(vis), rd, rb, P->bin_lds, st));
  return status;
}

template <class OutT>
void run_grid(mi_ctx* ctx, Plan* P, const mi_c64* vis, const float* uv, const float* w_in, bool beam, OutT* out,
              int modulate, hipStream_t st) {
  const InstDesc* inst = static_cast<const InstDesc*>(P->inst.p);
  const int* tmap = static_cast<const int*>(beam ? P->tile_inst_b.p : P->tile_inst_d.p);
  const int nt = beam ? P->tiles_b : P->tiles_d;
  const int* ent = static_cast<const int*>(beam ? P->ent_b.p : P->ent_d.p);
  const int* ts = static_cast<const int*>(beam ? P->ts_b.p : P->ts_d.p);
  const int* tc = static_cast<const int*>(beam ? P->tc_b.p : P->tc_d.p);
  const float2* v = beam ? nullptr : reinterpret_cast<const float2*>(vis);
  const float* wts = static_cast<const float*>(P->wts.p);
  if constexpr (std::is_same<OutT, double2>::value) {
    hipEvent_t pe = prof_start(ctx, MI_PROF_GRID, st);
    HIPCHK(launch_grid(inst, tmap, nt, beam ? 1 : 0, v, reinterpret_cast<const float2*>(uv), w_in, wts, ent, ts, tc,
                       ctx->T, out, modulate, ctx->grid_chunk, st));
    prof_stop(pe, st);
  } else
    HIPCHK(launch_grid_f32(inst, tmap, nt, beam ? 1 : 0, v, reinterpret_cast<const float2*>(uv), w_in, wts, ent, ts,
                           tc, ctx->T, out, modulate, ctx->grid_chunk, st));
}

// Dirty images straight from the visibilities: the fused gridding + first pass (line-block
// lists from run_bin with blocks = true), then pass B.
void run_dirty_fused(mi_ctx* ctx, Plan* P, const mi_c64* vis, const float* uv, const float* w_in, float* out,
                     hipStream_t st, const double* b0 = nullptr) {
  const InstDesc* inst = static_cast<const InstDesc*>(P->inst.p);
  double2* g = dev_alloc<double2>(P->gd, P->total_gd);
  if (!b0) b0 = static_cast<const double*>(P->b0.p);
  hipEvent_t pe = prof_start(ctx, MI_PROF_GRID_FFT, st);
  HIPCHK(launch_grid_fft_a(P->elems_d, ctx->n_cu, inst, static_cast<const FftWork*>(P->wa_d.p), P->n_wa_d,
                           static_cast<const GridRec*>(P->rec_d.p), static_cast<const int*>(P->bs_d.p),
                           static_cast<const int*>(P->bc_d.p), g, ctx->T, st));
  prof_stop(pe, st);
  pe = prof_start(ctx, MI_PROF_IFFT, st);
  HIPCHK(launch_fft_b_c2r(P->elems_d, ctx->n_cu, inst, static_cast<const FftWork*>(P->wb_d.p), P->n_wb_d, g, b0, ctx->T, out,
                          st));
  prof_stop(pe, st);
}

// Dirty images from the dirty half grids in P->gd.
void run_image(mi_ctx* ctx, Plan* P, float* out, hipStream_t st, const double* b0 = nullptr) {
  const InstDesc* inst = static_cast<const InstDesc*>(P->inst.p);
  double2* g = static_cast<double2*>(P->gd.p);
  if (!b0) b0 = static_cast<const double*>(P->b0.p);
  hipEvent_t pe = prof_start(ctx, MI_PROF_IFFT, st);
  HIPCHK(launch_fft_a(P->elems_d, ctx->n_cu, inst, static_cast<const FftWork*>(P->wa_d.p), P->n_wa_d, g, ctx->T, st));
  prof_stop(pe, st);
  pe = prof_start(ctx, MI_PROF_IFFT, st);
  HIPCHK(launch_fft_b_c2r(P->elems_d, ctx->n_cu, inst, static_cast<const FftWork*>(P->wb_d.p), P->n_wb_d, g, b0, ctx->T, out,
                          st));
  prof_stop(pe, st);
}

// Beams: real FP64 beam grid (gridder), then the two symmetric transform passes.
// With P->fused (line-block lists from run_bin), the gridding and the first pass are one kernel.
void run_beam(mi_ctx* ctx, Plan* P, const float* uv, const float* w_in, float* out, hipStream_t st) {
  const InstDesc* inst = static_cast<const InstDesc*>(P->inst.p);
  double* g = dev_alloc<double>(P->gbr, P->total_gb);
  hipEvent_t pe;
  if (P->fused) {
    pe = prof_start(ctx, MI_PROF_GRID_FFT, st);
    HIPCHK(launch_grid_fft_a_real(P->elems_b, ctx->n_cu, inst, static_cast<const FftWork*>(P->wa_b.p), P->n_wa_b,
                                  static_cast<const GridRec*>(P->rec_b.p), static_cast<const int*>(P->bs_b.p),
                                  static_cast<const int*>(P->bc_b.p), g, ctx->T, st));
    prof_stop(pe, st);
  } else {
    pe = prof_start(ctx, MI_PROF_GRID, st);
    HIPCHK(launch_grid_real(inst, static_cast<const int*>(P->tile_inst_b.p), P->tiles_b,
                            reinterpret_cast<const float2*>(uv), w_in, static_cast<const float*>(P->wts.p),
                            static_cast<const int*>(P->ent_b.p), static_cast<const int*>(P->ts_b.p),
                            static_cast<const int*>(P->tc_b.p), ctx->T, g, ctx->grid_chunk, st));
    prof_stop(pe, st);
    pe = prof_start(ctx, MI_PROF_IFFT, st);
    HIPCHK(launch_fft_a_real(P->elems_b, ctx->n_cu, inst, static_cast<const FftWork*>(P->wa_b.p), P->n_wa_b, g, ctx->T,
                             st));
    prof_stop(pe, st);
  }
  pe = prof_start(ctx, MI_PROF_IFFT, st);
  HIPCHK(launch_fft_b_c2r_sym(P->elems_b, ctx->n_cu, inst, static_cast<const FftWork*>(P->wb_b.p), P->n_wb_b, g,
                              static_cast<const double*>(P->b0.p), ctx->T, out, st));
  prof_stop(pe, st);
}

// CLEAN schedule for one batch.  Every image size N gets its own team size G(N), the
// smallest that keeps each member's chunk N^2/G within 64 residual pixels per thread (so
// all members of a mixed batch carry the same load), or the requested team size scaled by
// (N / N_max)^2.  Teams per size class: one at least, one per image at most; the rest of
// the device goes to the class with the most CLEAN iterations per team.  Teams of up to
// 32 workgroups are packed onto XCDs first-fit in decreasing size (exact for power-of-two
// sizes); images go to the least-loaded team of their class in decreasing niter (LPT).
void build_clean_schedule(mi_ctx* ctx, Plan* P, CleanPlan* C, int req) {
  const int n = P->n_inst;
  std::vector<int> sizes(P->n.begin(), P->n.end());
  std::sort(sizes.begin(), sizes.end(), std::greater<int>());
  sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
  const int n_max = sizes[0];
  struct Cls { int N, G, T, cap; std::vector<int> imgs; double work; };
  std::vector<Cls> cls;
  for (int N : sizes) {
    Cls c{};
    c.N = N;
    const int g_min = std::max(1, (N * N) / 65536);
    c.cap = std::min(256, N);                     // a member's chunk must start on a row
    if (g_min > c.cap) fail(MI_ERR_UNSUPPORTED, "CLEAN team too large for N = %d", N);
    int g = g_min;
    if (req) {
      const int64_t scaled = std::max<int64_t>(1, (int64_t)req * N * N / ((int64_t)n_max * n_max));
      g = 1;
      while ((int64_t)g * 2 <= scaled) g *= 2;
      g = std::min(std::max(g, g_min), c.cap);
    }
    c.G = g;
    c.work = 0.0;
    for (int i = 0; i < n; ++i)
      if (P->n[i] == N) {
        c.imgs.push_back(i);
        c.work += (double)C->niter[i] + 1.0;
      }
    cls.push_back(c);
  }
  // a single size without a request: more workgroups per image when there are few images
  if (!req && cls.size() == 1) {
    Cls& c = cls[0];
    while (c.G * 2 <= std::min(32, c.cap) && (int64_t)c.G * 2 * (int64_t)c.imgs.size() <= 256) c.G *= 2;
  }
  bool local = true;
  int ppt = 4;
  int64_t max_chunk = 1;
  for (const Cls& c : cls) {
    local = local && c.G <= 32;
    while ((int64_t)ppt * 1024 * c.G < (int64_t)c.N * c.N) ppt *= 2;
    max_chunk = std::max<int64_t>(max_chunk, (int64_t)c.N * c.N / c.G);
  }
  const int sub_px = (int)std::min<int64_t>(max_chunk, CLEAN_RESTORE_SUB_PX);
  const size_t lds = (size_t)sub_px * sizeof(float);
  int per_cu = 0;
  HIPCHK(clean_max_blocks_per_cu(ppt, local, !C->win.empty(), lds, &per_cu));
  if (per_cu < 1) fail(MI_ERR_UNSUPPORTED, "CLEAN kernel cannot be resident");
  int cap = per_cu * ctx->n_cu;
  if (local) cap -= cap % 8;
  // teams per class
  int used = 0;
  for (Cls& c : cls) { c.T = 1; used += c.G; }
  if (used > cap) fail(MI_ERR_UNSUPPORTED, "CLEAN teams (%d workgroups) exceed the device (%d)", used, cap);
  for (;;) {
    int best = -1;
    double best_load = -1.0;
    for (int k = 0; k < (int)cls.size(); ++k) {
      const Cls& c = cls[k];
      if (c.T >= (int)c.imgs.size() || used + c.G > cap) continue;
      const double load = c.work / c.T;
      if (load > best_load) { best_load = load; best = k; }
    }
    if (best < 0) break;
    cls[best].T += 1;
    used += cls[best].G;
  }
  // teams in decreasing size (classes are in decreasing N, hence non-increasing G)
  std::vector<int> team_G, team_cls;
  for (int k = 0; k < (int)cls.size(); ++k)
    for (int t = 0; t < cls[k].T; ++t) { team_G.push_back(cls[k].G); team_cls.push_back(k); }
  const int T = (int)team_G.size();
  std::vector<int2> blk;
  if (local) {
    const int per_xcd = cap / 8;
    std::vector<int> fill(8, 0), team_x(T), team_r(T);
    for (int t = 0; t < T; ++t) {
      int x = 0;
      while (x < 8 && fill[x] + team_G[t] > per_xcd) ++x;
      if (x == 8) fail(MI_ERR_UNSUPPORTED, "CLEAN teams do not fit the XCDs");
      team_x[t] = x;
      team_r[t] = fill[x];
      fill[x] += team_G[t];
    }
    const int rows = *std::max_element(fill.begin(), fill.end());
    blk.assign((size_t)8 * rows, make_int2(-1, 0));
    for (int t = 0; t < T; ++t)
      for (int m = 0; m < team_G[t]; ++m) blk[(size_t)team_x[t] + 8 * (team_r[t] + m)] = make_int2(t, m);
  } else {
    for (int t = 0; t < T; ++t)
      for (int m = 0; m < team_G[t]; ++m) blk.push_back(make_int2(t, m));
  }
  // LPT within each class
  std::vector<std::vector<int>> lists(T);
  int first = 0;
  for (int k = 0; k < (int)cls.size(); ++k) {
    std::vector<int> order = cls[k].imgs;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return C->niter[a] > C->niter[b]; });
    std::vector<double> load(cls[k].T, 0.0);
    for (int i : order) {
      const int t = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      lists[first + t].push_back(i);
      load[t] += (double)C->niter[i] + 1.0;
    }
    first += cls[k].T;
  }
  std::vector<int> toff(T + 1, 0), timgs;
  std::vector<int64_t> tslot(T, 0);
  int64_t ns = 0;
  for (int t = 0; t < T; ++t) {
    toff[t + 1] = toff[t] + (int)lists[t].size();
    timgs.insert(timgs.end(), lists[t].begin(), lists[t].end());
    tslot[t] = ns;
    ns += 2 * (int64_t)team_G[t];
  }
  std::vector<int64_t> coff(n);
  int64_t sum = 0;
  for (int i = 0; i < n; ++i) { coff[i] = sum; sum += C->niter[i]; }
  C->total_comp = sum;
  C->T = T;
  C->local = local ? 1 : 0;
  C->ppt = ppt;
  C->n_blocks = (int)blk.size();
  C->lds = lds;
  C->sub_px = sub_px;
  C->n_slots = ns;
  upload(C->team_off, toff);
  upload(C->team_imgs, timgs);
  upload(C->blk, blk);
  upload(C->team_G, team_G);
  upload(C->team_slot, tslot);
  upload(C->niter_d, C->niter);
  if (C->has_thr) upload(C->thr_d, C->thr);
  if (!C->win.empty()) upload(C->win_d, C->win);
  upload(C->comp_off, coff);
  dev_alloc<unsigned long long>(C->slots, (size_t)ns);
}

void copy_b0(Plan* P, double* b0_out, hipStream_t st) {
  if (b0_out)
    HIPCHK(hipMemcpyAsync(b0_out, P->b0.p, sizeof(double) * 2 * P->n_inst, hipMemcpyDeviceToDevice, st));
}

template <class F>
mi_status guard(mi_ctx* ctx, F&& f) {
  if (!ctx) return MI_ERR_ARG;
  ctx->err.clear();
  try {
    f();
    return MI_OK;
  } catch (const MiError& e) {
    ctx->err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->err = "host allocation failed";
    return MI_ERR_NOMEM;
  } catch (...) {
    ctx->err = "unexpected internal error";
    return MI_ERR_DEVICE;
  }
}

void need(const void* p, const char* name) {
  if (!p) fail(MI_ERR_ARG, "%s must not be NULL", name);
}

}  // namespace
}  // namespace mi

namespace mi {
namespace {

// ---- CLEAN without allocation (mi_hogbom_clean_noalloc) --------------------------------
// A file-scope device array holds everything the CLEAN kernels need beyond the caller's
// inputs and outputs: instance descriptors, team tables, exchange slots, symmetry flags,
// the clean-beam parameters and, when asked to restore without component outputs, the
// component lists.  Each device holds its own copy; host code reaches it only through the
// address hipGetSymbolAddress returns for the device (kept per device at context creation).
constexpr int NA_MAX_INST = 64;
constexpr size_t NA_SCRATCH_BYTES = 8u << 20;
constexpr int NA_MAX_DEVICES = 64;
__device__ __align__(256) unsigned char scratch[NA_SCRATCH_BYTES];
std::atomic<unsigned char*> g_noalloc_ptr[NA_MAX_DEVICES];

// Everything the set-up kernel writes, passed by value (so the call needs no host-to-device
// copy of its own), with the byte offsets of each table in the scratch array.
struct NaSetup {
  int n, N, log2N, G, T, local, n_blocks, has_thr;
  int32_t niter[NA_MAX_INST];
  float thr[NA_MAX_INST];
  int16_t team_off[NA_MAX_INST + 1];
  int16_t team_imgs[NA_MAX_INST];
  int64_t o_inst, o_team_off, o_team_imgs, o_blk, o_team_G, o_team_slot, o_niter, o_thr, o_comp_off, o_slots,
      o_asym, o_rrad, o_cbeam, o_cidx, o_cflx;
  int n_slots;
  int32_t* status;
};

// Writes the tables and clears what must start at zero (exchange slots, symmetry flags,
// status): the array keeps whatever the previous call on this device left in it.
__global__ void __launch_bounds__(256) k_noalloc_setup(unsigned char* base, NaSetup S) {
  const int tid = threadIdx.x;
  InstDesc* inst = reinterpret_cast<InstDesc*>(base + S.o_inst);
  const int64_t n2 = (int64_t)S.N * S.N;
  for (int i = tid; i < S.n; i += 256) {
    InstDesc d{};
    d.img_off = i * n2;
    d.beam_off = 4 * i * n2;
    d.N = S.N;
    d.log2N = S.log2N;
    inst[i] = d;
    reinterpret_cast<int*>(base + S.o_team_imgs)[i] = S.team_imgs[i];
    reinterpret_cast<int*>(base + S.o_niter)[i] = S.niter[i];
    reinterpret_cast<float*>(base + S.o_thr)[i] = S.has_thr ? S.thr[i] : 0.0f;
    reinterpret_cast<int*>(base + S.o_asym)[i] = 0;
    if (S.status) S.status[i] = 0;
  }
  for (int t = tid; t <= S.T; t += 256) reinterpret_cast<int*>(base + S.o_team_off)[t] = S.team_off[t];
  for (int t = tid; t < S.T; t += 256) {
    reinterpret_cast<int*>(base + S.o_team_G)[t] = S.G;
    reinterpret_cast<int64_t*>(base + S.o_team_slot)[t] = 2LL * S.G * t;
  }
  // block roles: teams of up to 32 dealt round-robin over the 8 XCDs (block b runs on XCD
  // b % 8), members of a team in consecutive rows of its XCD; larger teams in order
  int2* blk = reinterpret_cast<int2*>(base + S.o_blk);
  for (int b = tid; b < S.n_blocks; b += 256) {
    int team, member;
    if (S.local) {
      const int x = b & 7, r = b >> 3;
      team = (r / S.G) * 8 + x;
      member = r % S.G;
    } else {
      team = b / S.G;
      member = b % S.G;
    }
    blk[b] = team < S.T ? make_int2(team, member) : make_int2(-1, 0);
  }
  unsigned long long* slots = reinterpret_cast<unsigned long long*>(base + S.o_slots);
  for (int q = tid; q < S.n_slots; q += 256) slots[q] = 0ull;
  if (tid == 0) {
    int64_t* coff = reinterpret_cast<int64_t*>(base + S.o_comp_off);
    int64_t acc = 0;
    for (int i = 0; i < S.n; ++i) { coff[i] = acc; acc += S.niter[i]; }
  }
}

}  // namespace
}  // namespace mi

using namespace mi;

extern "C" {

const char* mi_version(void) { return "mi 0.1 (gfx950)"; }

const char* mi_last_error(const mi_ctx* ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

mi_status mi_ctx_create(mi_ctx** out, int device) {
  if (!out) return MI_ERR_ARG;
  *out = nullptr;
  mi_ctx* ctx = nullptr;
  try {
    ctx = new mi_ctx();
  } catch (...) {
    return MI_ERR_NOMEM;
  }
  mi_status s = guard(ctx, [&] {
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) fail(MI_ERR_ARG, "device %d out of range (%d devices)", device, ndev);
    HIPCHK(hipSetDevice(device));
    ctx->device = device;
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, device));
    ctx->n_cu = prop.multiProcessorCount;
    if (device < NA_MAX_DEVICES) {
      // the device's copy of the no-allocation CLEAN scratch array (device current)
      unsigned char* sp = g_noalloc_ptr[device].load();
      if (!sp) {
        void* a = nullptr;
        HIPCHK(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
        sp = static_cast<unsigned char*>(a);
        g_noalloc_ptr[device].store(sp);
      }
      ctx->noalloc_scratch = sp;
    }
    const char* fi = std::getenv("MI_TEST_FAIL_INSTANCE");
    ctx->fail_inst = fi ? std::atoi(fi) : -1;
    const char* cs = std::getenv("MI_TEST_CLEAN_STALL");
    ctx->clean_stall = cs && std::atoi(cs) != 0 ? 1 : 0;
    HostTables H = build_host_tables(W, OS, 1.0, 200);
    ctx->T.tab = upload(ctx->tab, H.tab);
    ctx->T.tsum = upload(ctx->tsum, H.tsum);
    ctx->T.twiddle = reinterpret_cast<const double2*>(upload(ctx->tw, H.twiddle));
    ctx->T.inv_corr = upload(ctx->icorr, H.inv_corr);
    ctx->T.inv_corr0_sq = 1.0 / (H.corr0 * H.corr0);
  });
  if (s != MI_OK) {
    std::fprintf(stderr, "mi_ctx_create: %s\n", ctx->err.c_str());
    delete ctx;
    return s;
  }
  *out = ctx;
  return MI_OK;
}

mi_status mi_ctx_destroy(mi_ctx* ctx) {
  if (!ctx) return MI_ERR_ARG;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  delete ctx;
  return MI_OK;
}

mi_status mi_gmm_levels(mi_ctx* ctx, const mi_batch* batch, const float* images, int32_t n_bins, int32_t n_iter,
                        double* levels_out, float* mu_a_out, float* mu_b_out, hipStream_t stream) {
  return guard(ctx, [&] {
    need(images, "images");
    need(levels_out, "levels_out");
    if (n_bins < 2 || n_bins > 4096) fail(MI_ERR_ARG, "n_bins must be in [2, 4096] (got %d)", n_bins);
    if (n_iter < 0 || n_iter > 100000) fail(MI_ERR_ARG, "n_iter must be in [0, 100000] (got %d)", n_iter);
    HIPCHK(hipSetDevice(ctx->device));
    Plan* P = get_plan(ctx, batch, stream);
    HIPCHK(launch_gmm(static_cast<const InstDesc*>(P->inst.p), P->n_inst, images, n_bins, n_iter, levels_out,
                      mu_a_out, mu_b_out, stream));
  });
}

mi_status mi_disk_offsets(mi_ctx* ctx, const mi_batch* batch, const float* images, const double* radius_px,
                          double* offsets_out, hipStream_t stream) {
  return guard(ctx, [&] {
    need(images, "images");
    need(radius_px, "radius_px");
    need(offsets_out, "offsets_out");
    HIPCHK(hipSetDevice(ctx->device));
    Plan* P = get_plan(ctx, batch, stream);
    const int n = P->n_inst;
    for (int i = 0; i < n; ++i)
      if (!(radius_px[i] > 0.0) || !(radius_px[i] < 1e6)) fail(MI_ERR_ARG, "radius_px[%d] must be positive", i);
    if (P->radius.size() != (size_t)n || !std::equal(P->radius.begin(), P->radius.end(), radius_px)) {
      P->radius.assign(radius_px, radius_px + n);
      upload(P->radius_d, P->radius);
      P->corr_model_ready = false;
    }
    if (!P->corr_work.p) {                              // 2-D transform plans
      // the disk models, one per instance
      std::vector<int32_t> nn(P->n.begin(), P->n.end());
      std::vector<int64_t> offs(n);
      std::vector<FftWork> work;
      P->corr_elems = fft_elems_for(P->max_N);
      for (int i = 0; i < n; ++i) {
        offs[i] = P->h_inst[i].img_off;
        int nl = P->corr_elems / nn[i];
        if (nl > nn[i]) nl = nn[i];
        for (int l = 0; l < nn[i]; l += nl) work.push_back({i, l});
      }
      P->corr_nwork = (int)work.size();
      upload(P->corr_n, nn);
      upload(P->corr_offs, offs);
      upload(P->corr_work, work);
      // the maps, paired in instance order among equal sizes (a map without a partner of
      // its size keeps a slot of its own); coff[i] = 2 x (slot offset) + (0: real part,
      // 1: imaginary part)
      std::vector<CorrSlot> slots;
      std::vector<int64_t> coff(n);
      std::map<int, int> waiting;                       // N -> slot still missing its second map
      int64_t so = 0;
      for (int i = 0; i < n; ++i) {
        const int N = nn[i];
        auto it = waiting.find(N);
        if (it != waiting.end()) {
          CorrSlot& sl = slots[it->second];
          sl.b = i;
          coff[i] = 2 * sl.off + 1;
          waiting.erase(it);
        } else {
          waiting[N] = (int)slots.size();
          slots.push_back(CorrSlot{i, -1, N, ilog2i(N), so});
          coff[i] = 2 * so;
          so += (int64_t)N * N;
        }
      }
      std::vector<int32_t> sn;
      std::vector<int64_t> soffs;
      std::vector<FftWork> swork;
      for (int k = 0; k < (int)slots.size(); ++k) {
        const int N = slots[k].N;
        sn.push_back(N);
        soffs.push_back(slots[k].off);
        int nl = P->corr_elems / N;
        if (nl > N) nl = N;
        for (int l = 0; l < N; l += nl) swork.push_back({k, l});
      }
      P->corr_nslots = (int)slots.size();
      P->corr_snwork = (int)swork.size();
      P->corr_slot_total = so;
      upload(P->corr_slots, slots);
      upload(P->corr_sn, sn);
      upload(P->corr_soffs, soffs);
      upload(P->corr_swork, swork);
      upload(P->corr_coff, coff);
    }
    const int64_t total = P->total_img;
    double2* Z = dev_alloc<double2>(P->corr_x, (size_t)P->corr_slot_total);
    double2* D = dev_alloc<double2>(P->corr_d, total);
    double2* S = dev_alloc<double2>(P->corr_s, total);   // >= the slots' total
    const InstDesc* inst = static_cast<const InstDesc*>(P->inst.p);
    const int e = P->corr_elems;
    const CorrSlot* slots = static_cast<const CorrSlot*>(P->corr_slots.p);
    const int ns = P->corr_nslots;
    const int* snd = static_cast<const int*>(P->corr_sn.p);
    const int64_t* sod = static_cast<const int64_t*>(P->corr_soffs.p);
    const FftWork* swk = static_cast<const FftWork*>(P->corr_swork.p);
    const int snw = P->corr_snwork;
    if (!P->corr_model_ready) {                         // the disk models' transforms are kept
      const int* nd = static_cast<const int*>(P->corr_n.p);
      const int64_t* od = static_cast<const int64_t*>(P->corr_offs.p);
      const FftWork* wk = static_cast<const FftWork*>(P->corr_work.p);
      HIPCHK(launch_corr_prep(inst, n, P->max_N, images, static_cast<const double*>(P->radius_d.p), nullptr, D,
                              stream));
      HIPCHK(launch_fft_c2c_t_d2d(e, nd, od, wk, P->corr_nwork, D, S, ctx->T, -1.0, 0, 0, stream));
      HIPCHK(launch_fft_c2c_t_d2d(e, nd, od, wk, P->corr_nwork, S, D, ctx->T, -1.0, 0, 0, stream));
      P->corr_model_ready = true;
    }
    // Z = A + i B per slot; forward 2-D DFTs (two line passes with transposed writes,
    // plain, no centring); W = A^ conj(DA) + i B^ conj(DB); inverse: Re / Im = the two
    // correlations
    HIPCHK(launch_corr_prep_pair(slots, ns, inst, P->max_N, images, Z, stream));
    HIPCHK(launch_fft_c2c_t_d2d(e, snd, sod, swk, snw, Z, S, ctx->T, -1.0, 0, 0, stream));
    HIPCHK(launch_fft_c2c_t_d2d(e, snd, sod, swk, snw, S, Z, ctx->T, -1.0, 0, 0, stream));
    HIPCHK(launch_corr_mul_pair(slots, ns, inst, P->max_N, Z, D, S, stream));
    HIPCHK(launch_fft_c2c_t_d2d(e, snd, sod, swk, snw, S, Z, ctx->T, +1.0, 0, 0, stream));
    HIPCHK(launch_fft_c2c_t_d2d(e, snd, sod, swk, snw, Z, S, ctx->T, +1.0, 0, 0, stream));
    HIPCHK(launch_corr_peak(inst, n, S, static_cast<const int64_t*>(P->corr_coff.p), offsets_out, stream));
  });
}

mi_status mi_phase_shift(mi_ctx* ctx, const mi_batch* batch, mi_c64* vis, const float* uv, const double* offsets,
                         hipStream_t stream) {
  return guard(ctx, [&] {
    need(vis, "vis");
    need(uv, "uv");
    need(offsets, "offsets");
    HIPCHK(hipSetDevice(ctx->device));
    Plan* P = get_plan(ctx, batch, stream);
    HIPCHK(launch_phase_shift(static_cast<const InstDesc*>(P->inst.p), P->n_inst, P->max_nvis,
                              reinterpret_cast<float2*>(vis), reinterpret_cast<const float2*>(uv), offsets, stream));
  });
}

mi_status mi_set_tuning(mi_ctx* ctx, const mi_tuning* t) {
  return guard(ctx, [&] {
    need(t, "tuning");
    if (t->grid_chunk != 0 && (t->grid_chunk < 1 || t->grid_chunk > 32))
      fail(MI_ERR_ARG, "grid_chunk must be 0 or in [1, 32] (got %d)", t->grid_chunk);
    if (t->fft_elems != 0 && t->fft_elems != FFT_ELEMS_SMALL && t->fft_elems != FFT_ELEMS_LARGE)
      fail(MI_ERR_ARG, "fft_elems must be 0, %d or %d (got %d)", FFT_ELEMS_SMALL, FFT_ELEMS_LARGE, t->fft_elems);
    ctx->grid_chunk = t->grid_chunk ? t->grid_chunk : 8;
    ctx->fft_elems = t->fft_elems;
  });
}

mi_status mi_get_tuning(mi_ctx* ctx, mi_tuning* t) {
  return guard(ctx, [&] {
    need(t, "tuning");
    t->grid_chunk = ctx->grid_chunk;
    t->fft_elems = ctx->fft_elems;
  });
}

mi_status mi_profile_begin_kinds(mi_ctx* ctx, uint32_t kinds) {
  return guard(ctx, [&] {
    const uint32_t all = MI_PROF_CLEAN | MI_PROF_GRID | MI_PROF_IFFT | MI_PROF_GRID_FFT;
    if (kinds == 0u || (kinds & ~all)) fail(MI_ERR_ARG, "kinds must be a non-empty mask of MI_PROF_* bits (got %u)", kinds);
    ctx->prof_kinds = kinds;
    ctx->prof_used = 0;
  });
}

mi_status mi_profile_begin(mi_ctx* ctx) { return mi_profile_begin_kinds(ctx, MI_PROF_CLEAN); }

mi_status mi_profile_end_kinds(mi_ctx* ctx, float* ms_out, int32_t* kind_out, int32_t cap, int32_t* n_out) {
  return guard(ctx, [&] {
    need(n_out, "n_out");
    if (cap > 0) need(ms_out, "ms_out");
    HIPCHK(hipSetDevice(ctx->device));
    const size_t n = ctx->prof_used;
    for (size_t i = 0; i < n && (int64_t)i < cap; ++i) {
      HIPCHK(hipEventSynchronize(ctx->prof_ev[i].second));
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, ctx->prof_ev[i].first, ctx->prof_ev[i].second));
      ms_out[i] = ms;
      if (kind_out) kind_out[i] = (int32_t)ctx->prof_kind[i];
    }
    *n_out = (int32_t)n;
    ctx->prof_kinds = 0;
    ctx->prof_used = 0;
  });
}

mi_status mi_profile_end(mi_ctx* ctx, float* ms_out, int32_t cap, int32_t* n_out) {
  return mi_profile_end_kinds(ctx, ms_out, nullptr, cap, n_out);
}

mi_status mi_grid(mi_ctx* ctx, const mi_batch* batch, const mi_c64* vis, const float* uv, const float* w_in,
                  int which, int layout, mi_c64* grid_out, double* b0_out, int32_t* n_kept_out,
                  hipStream_t stream) {
  return guard(ctx, [&] {
    if (which < 0 || which > 2) fail(MI_ERR_ARG, "which must be 0 (dirty), 1 (beam) or 2 (both)");
    if (layout != MI_LAYOUT_FULL && layout != MI_LAYOUT_HALF) fail(MI_ERR_ARG, "bad layout %d", layout);
    need(uv, "uv");
    need(w_in, "w_in");
    need(grid_out, "grid_out");
    if (which != 1) need(vis, "vis");
    if (reinterpret_cast<uintptr_t>(grid_out) % 16) fail(MI_ERR_ARG, "grid_out must be 16-byte aligned");
    HIPCHK(hipSetDevice(ctx->device));
    Plan* P = get_plan(ctx, batch, stream);
    const bool want_d = which != 1, want_b = which != 0;
    run_bin(ctx, P, batch, uv, w_in, want_b, stream);
    float2* out = reinterpret_cast<float2*>(grid_out);
    if (layout == MI_LAYOUT_HALF) {
      if (want_d) run_grid<float2>(ctx, P, vis, uv, w_in, false, out, 0, stream);
      if (want_b) run_grid<float2>(ctx, P, vis, uv, w_in, true, out + (want_d ? P->total_gd : 0), 0, stream);
    } else {
      // offsets uploaded with the plan: dirty grids, beam grids after them, beam grids alone
      const int64_t* offd = static_cast<const int64_t*>(P->full_off.p);
      const InstDesc* inst = static_cast<const InstDesc*>(P->inst.p);
      if (want_d) {
        double2* g = dev_alloc<double2>(P->gd, P->total_gd);
        run_grid<double2>(ctx, P, vis, uv, w_in, false, g, 0, stream);
        HIPCHK(launch_expand_full(inst, P->n_inst, 0, g, out, offd, stream));
      }
      if (want_b) {
        double2* g = dev_alloc<double2>(P->gb, P->total_gb);
        run_grid<double2>(ctx, P, vis, uv, w_in, true, g, 0, stream);
        HIPCHK(launch_expand_full(inst, P->n_inst, 1, g, out, offd + (want_d ? 1 : 2) * P->n_inst, stream));
      }
    }
    copy_b0(P, b0_out, stream);
    if (n_kept_out)
      HIPCHK(hipMemcpyAsync(n_kept_out, P->nkept.p, sizeof(int) * P->n_inst, hipMemcpyDeviceToDevice, stream));
  });
}

mi_status mi_ifft2(mi_ctx* ctx, mi_c64* data, const int32_t* n, const int64_t* offs, int32_t n_inst,
                   hipStream_t stream) {
  return guard(ctx, [&] {
    need(data, "data");
    need(n, "n");
    need(offs, "offs");
    if (n_inst < 1) fail(MI_ERR_ARG, "n_inst must be >= 1");
    for (int i = 0; i < n_inst; ++i) {
      if (!is_pow2(n[i]) || n[i] < 64 || n[i] > 8192)
        fail(MI_ERR_SHAPE, "n[%d] = %d is not a power of two in [64, 8192]", i, n[i]);
      if (offs[i] < 0) fail(MI_ERR_SHAPE, "offs[%d] < 0", i);
    }
    if (reinterpret_cast<uintptr_t>(data) % 8) fail(MI_ERR_ARG, "data must be 8-byte aligned");
    HIPCHK(hipSetDevice(ctx->device));
    uint64_t h = fnv1a(&n_inst, sizeof n_inst);
    h = fnv1a(n, sizeof(int32_t) * n_inst, h);
    h = fnv1a(offs, sizeof(int64_t) * n_inst, h);
    auto it = ctx->ifft_plans.find(h);
    IfftPlan* P;
    if (it != ctx->ifft_plans.end() && std::equal(it->second->n.begin(), it->second->n.end(), n) &&
        std::equal(it->second->offs.begin(), it->second->offs.end(), offs)) {
      P = it->second.get();
      touch(ctx, P, stream);
    } else {
      if (it != ctx->ifft_plans.end()) {            // a hash collision: replace that entry
        if (it->second->pinned) fail(MI_ERR_UNSUPPORTED, "transform plan collision with a plan held by a captured graph");
        ctx->ifft_plans.erase(it);
      }
      make_room(ctx->ifft_plans, 16, stream);
      auto up = std::make_unique<IfftPlan>();
      up->n.assign(n, n + n_inst);
      up->offs.assign(offs, offs + n_inst);
      std::vector<FftWork> work;
      int64_t end = 0;
      int maxn = 0;
      for (int i = 0; i < n_inst; ++i) maxn = std::max(maxn, n[i]);
      up->elems = fft_elems_for(maxn);
      for (int i = 0; i < n_inst; ++i) {
        int nl = up->elems / n[i];
        if (nl > n[i]) nl = n[i];
        for (int l = 0; l < n[i]; l += nl) work.push_back({i, l});
        end = std::max<int64_t>(end, offs[i] + (int64_t)n[i] * n[i]);
      }
      up->total = end;
      up->n_work1 = (int)work.size();
      upload(up->n_d, up->n);
      upload(up->offs_d, up->offs);
      upload(up->work, work);
      P = up.get();
      touch(ctx, P, stream);
      ctx->ifft_plans[h] = std::move(up);
    }
    double2* scratch = dev_alloc<double2>(ctx->ifft_scratch, P->total);
    float2* d = reinterpret_cast<float2*>(data);
    HIPCHK(launch_fft_c2c_t_f2d(P->elems, static_cast<const int*>(P->n_d.p), static_cast<const int64_t*>(P->offs_d.p),
                                static_cast<const FftWork*>(P->work.p), P->n_work1, d, scratch, ctx->T, +1.0, 1, 0,
                                stream));
    HIPCHK(launch_fft_c2c_t_d2f(P->elems, static_cast<const int*>(P->n_d.p), static_cast<const int64_t*>(P->offs_d.p),
                                static_cast<const FftWork*>(P->work.p), P->n_work1, scratch, d, ctx->T, +1.0, 0, 1,
                                stream));
  });
}

mi_status mi_dirty_image(mi_ctx* ctx, const mi_batch* batch, const mi_c64* vis, const float* uv, const float* w_in,
                         float* dirty_out, float* beam_out, double* b0_out, hipStream_t stream) {
  return guard(ctx, [&] {
    need(vis, "vis");
    need(uv, "uv");
    need(w_in, "w_in");
    need(dirty_out, "dirty_out");
    HIPCHK(hipSetDevice(ctx->device));
    Plan* P = get_plan(ctx, batch, stream);
    const bool beam = beam_out != nullptr;
    run_bin(ctx, P, batch, uv, w_in, beam, stream, false, P->fused, vis);
    if (P->fused) {
      run_dirty_fused(ctx, P, vis, uv, w_in, dirty_out, stream);
    } else {
      double2* gd = dev_alloc<double2>(P->gd, P->total_gd);
      run_grid<double2>(ctx, P, vis, uv, w_in, false, gd, 1, stream);
      run_image(ctx, P, dirty_out, stream);
    }
    if (beam) run_beam(ctx, P, uv, w_in, beam_out, stream);
    copy_b0(P, b0_out, stream);
  });
}

// w-projection plan: instances with the same (N, cell) share one set of planes w_j = j dw,
// dw = tol / (pi r2) with r2 = l^2 + m^2 at the field corner; an instance uses planes
// 0 .. floor(w_max / dw + 1/2).  Plane supports widen the W = 7 support by the w-screen's
// largest uv frequency over the field (in cells) on each side.  Tables are built on the
// device, once per plan.
void build_wproj(mi_ctx* ctx, Plan* P, const double* w_max, double tol, hipStream_t st) {
  auto W = std::make_unique<Plan::WProj>();
  const int n = P->n_inst;
  W->w_max.assign(w_max, w_max + n);
  W->tol = tol;
  W->n_planes.resize(n);
  std::vector<WPlane> planes;
  std::vector<int2> rows;
  std::vector<WInst> winst(n);
  std::map<std::pair<int, double>, int> group_plane0;   // (N, cell) -> first plane
  std::map<std::pair<int, double>, int> group_n;
  auto plane_count = [&](int i) {
    const double half = 0.5 * P->n[i] * P->cell[i];
    const double r2 = 2.0 * half * half;
    const double dw = tol / (M_PI * r2);
    return std::make_pair((int)std::floor(w_max[i] / dw + 0.5) + 1, dw);
  };
  for (int i = 0; i < n; ++i) {
    const auto key = std::make_pair((int)P->n[i], P->cell[i]);
    group_n[key] = std::max(group_n[key], plane_count(i).first);
  }
  int64_t off = 0;
  int half_max = 0;
  for (auto& g : group_n) {
    const int N = g.first.first;
    const double cell = g.first.second;
    const double half = 0.5 * N * cell;
    const double r2 = 2.0 * half * half;
    const double dw = tol / (M_PI * r2);
    const double fov = N * cell;
    group_plane0[g.first] = (int)planes.size();
    if (N < WP_M) fail(MI_ERR_UNSUPPORTED, "w-projection needs N >= %d (got %d)", WP_M, N);
    for (int j = 0; j < g.second; ++j) {
      const int S = 2 * (3 + (int)std::ceil(j * dw * std::sqrt(r2) * fov)) + 1;
      if (S > WP_SMAX)
        fail(MI_ERR_UNSUPPORTED, "w-projection support %d > %d cells (w_max too large for N = %d)", S, WP_SMAX, N);
      const int nd = S * WP_OS + 1;
      const int p = (int)planes.size();
      planes.push_back(WPlane{N, S, j * dw, cell, off});
      for (int r = 0; r < nd; ++r) rows.push_back(make_int2(p, r));
      off += (int64_t)nd * nd;
      half_max = std::max(half_max, S * WP_OS / 2);
    }
  }
  if (off * (int64_t)sizeof(double2) > (8LL << 30)) fail(MI_ERR_UNSUPPORTED, "w-projection tables exceed 8 GiB");
  for (int i = 0; i < n; ++i) {
    const auto pc = plane_count(i);
    W->n_planes[i] = pc.first;
    winst[i] = WInst{group_plane0[std::make_pair((int)P->n[i], P->cell[i])], pc.first, pc.second};
  }
  upload(W->planes, planes);
  upload(W->rows, rows);
  upload(W->winst, winst);
  double2* scr = dev_alloc<double2>(W->screen, planes.size() * (size_t)(WP_M - 1) * (WP_M - 1));
  double2* dft = dev_alloc<double2>(W->dft, (size_t)(2 * half_max + 1) * (WP_M - 1));
  double2* tabs = dev_alloc<double2>(W->tabs, (size_t)off);
  HIPCHK(launch_wtables(static_cast<const WPlane*>(W->planes.p), (int)planes.size(),
                        static_cast<const int2*>(W->rows.p), (int)rows.size(), half_max, ctx->T, scr, dft, tabs, st));
  P->wproj = std::move(W);
}

mi_status mi_dirty_image_w(mi_ctx* ctx, const mi_batch* batch, const mi_c64* vis, const float* uv,
                           const float* w_lambda, const float* w_in, const mi_wproj_params* wp, float* dirty_out,
                           double* b0_out, int32_t* n_planes_out, hipStream_t stream) {
  return guard(ctx, [&] {
    need(vis, "vis");
    need(uv, "uv");
    need(w_lambda, "w_lambda");
    need(w_in, "w_in");
    need(wp, "params");
    need(wp->w_max, "params->w_max");
    need(dirty_out, "dirty_out");
    const double tol = wp->phase_tol > 0.0 ? wp->phase_tol : 0.1;
    if (!std::isfinite(tol)) fail(MI_ERR_ARG, "phase_tol must be finite");
    HIPCHK(hipSetDevice(ctx->device));
    Plan* P = get_plan(ctx, batch, stream);
    for (int i = 0; i < P->n_inst; ++i)
      if (!(wp->w_max[i] >= 0.0) || !std::isfinite(wp->w_max[i])) fail(MI_ERR_ARG, "w_max[%d] must be finite and >= 0", i);
    if (!P->wproj || P->wproj->tol != tol ||
        !std::equal(P->wproj->w_max.begin(), P->wproj->w_max.end(), wp->w_max))
      build_wproj(ctx, P, wp->w_max, tol, stream);
    Plan::WProj* W = P->wproj.get();
    run_bin(ctx, P, batch, uv, w_in, false, stream);
    double2* gd = dev_alloc<double2>(P->gd, P->total_gd);
    if ((int64_t)WP_ENT * P->total_vis >= (1LL << 31)) fail(MI_ERR_SHAPE, "batch too large for w-projection binning");
    int* ent = dev_alloc<int>(W->ent, (size_t)WP_ENT * P->total_vis);
    int* ts = dev_alloc<int>(W->ts, P->tiles_d);
    int* tc = dev_alloc<int>(W->tc, P->tiles_d);
    const InstDesc* inst = static_cast<const InstDesc*>(P->inst.p);
    const WInst* winst = static_cast<const WInst*>(W->winst.p);
    const WPlane* planes = static_cast<const WPlane*>(W->planes.p);
    const size_t lds = (size_t)(P->max_N / 2 / TK) * (P->max_N / TJ) * sizeof(int);
    HIPCHK(launch_bin_w(inst, P->n_inst, lds, reinterpret_cast<const float2*>(uv), w_in, w_lambda, winst, planes, ent,
                        ts, tc, stream));
    HIPCHK(launch_grid_wt(inst, static_cast<const int*>(P->tile_inst_d.p), P->tiles_d,
                          reinterpret_cast<const float2*>(vis), reinterpret_cast<const float2*>(uv), w_lambda, w_in,
                          static_cast<const float*>(P->wts.p), ent, ts, tc, winst, planes,
                          static_cast<const double2*>(W->tabs.p), gd, stream));
    run_image(ctx, P, dirty_out, stream);
    copy_b0(P, b0_out, stream);
    if (n_planes_out) std::copy(W->n_planes.begin(), W->n_planes.end(), n_planes_out);
  });
}

mi_status mi_dirty_beam(mi_ctx* ctx, const mi_batch* batch, const float* uv, const float* w_in, float* beam_out,
                        hipStream_t stream) {
  return guard(ctx, [&] {
    need(uv, "uv");
    need(w_in, "w_in");
    need(beam_out, "beam_out");
    HIPCHK(hipSetDevice(ctx->device));
    Plan* P = get_plan(ctx, batch, stream);
    run_bin(ctx, P, batch, uv, w_in, true, stream, false, P->fused);
    run_beam(ctx, P, uv, w_in, beam_out, stream);
  });
}

mi_status mi_hogbom_clean(mi_ctx* ctx, const mi_batch* batch, const float* dirty, const float* beam,
                          const mi_clean_params* prm, float* residual_out, double* model_out, int32_t* comp_idx,
                          double* comp_flux, int32_t* n_comp_out, float* restored_out, double* cbeam_out,
                          hipStream_t stream) {
  return guard(ctx, [&] {
    need(dirty, "dirty");
    need(beam, "beam");
    need(prm, "params");
    need(residual_out, "residual_out");
    need(prm->niter, "params->niter");
    if ((comp_idx == nullptr) != (comp_flux == nullptr)) fail(MI_ERR_ARG, "comp_idx and comp_flux: both or neither");
    if (!(prm->gain > 0.0f && prm->gain <= 1.0f)) fail(MI_ERR_ARG, "gain must be in (0, 1]");
    HIPCHK(hipSetDevice(ctx->device));
    Plan* P = get_plan(ctx, batch, stream);
    const int n = P->n_inst;
    for (int i = 0; i < n; ++i)
      if (prm->niter[i] < 0) fail(MI_ERR_ARG, "niter[%d] < 0", i);
    const int req = prm->team_size;
    if (req != 0 && (!is_pow2(req) || req > 256)) fail(MI_ERR_ARG, "team_size must be 0 or a power of two <= 256");
    // clean plan: team shapes, XCD packing, LPT assignment, device copies of niter / thresholds
    uint64_t h = fnv1a(prm->niter, sizeof(int32_t) * n);
    h = fnv1a(&req, sizeof req, h);
    const bool has_thr = prm->threshold != nullptr && prm->threshold_dev == nullptr;
    if (has_thr) h = fnv1a(prm->threshold, sizeof(float) * n, h ^ 0x9e3779b97f4a7c15ull);
    if (prm->window) {
      for (int i = 0; i < n; ++i) {
        const int32_t* w = prm->window + 4 * i;
        const int N = P->n[i];
        if (!(0 <= w[0] && w[0] < w[2] && w[2] <= N && 0 <= w[1] && w[1] < w[3] && w[3] <= N))
          fail(MI_ERR_ARG, "window[%d] = (%d, %d, %d, %d) is not a non-empty box inside the %d x %d map", i, w[0],
               w[1], w[2], w[3], N, N);
      }
      h = fnv1a(prm->window, sizeof(int32_t) * 4 * n, h ^ 0x7f4a7c159e3779b9ull);
    }
    const size_t n_win = prm->window ? 4 * (size_t)n : 0;
    CleanPlan* C = nullptr;
    auto it = P->cleans.find(h);
    if (it != P->cleans.end() && it->second->team_req == req &&
        std::equal(it->second->niter.begin(), it->second->niter.end(), prm->niter) &&
        it->second->has_thr == has_thr &&
        (!has_thr || std::equal(it->second->thr.begin(), it->second->thr.end(), prm->threshold)) &&
        it->second->win.size() == n_win &&
        std::equal(it->second->win.begin(), it->second->win.end(), prm->window)) {
      C = it->second.get();
      touch(ctx, C, stream);
    } else {
      if (it != P->cleans.end()) {                  // a hash collision: replace that entry
        if (it->second->pinned) fail(MI_ERR_UNSUPPORTED, "CLEAN plan collision with a plan held by a captured graph");
        P->cleans.erase(it);
      }
      make_room(P->cleans, 8, stream);
      auto up = std::make_unique<CleanPlan>();
      C = up.get();
      C->team_req = req;
      C->niter.assign(prm->niter, prm->niter + n);
      C->has_thr = has_thr;
      if (has_thr) C->thr.assign(prm->threshold, prm->threshold + n);
      if (n_win) C->win.assign(prm->window, prm->window + n_win);
      build_clean_schedule(ctx, P, C, req);
      touch(ctx, C, stream);
      P->cleans[h] = std::move(up);
    }
    int* status = batch->status;
    if (status) HIPCHK(launch_fill_u32(reinterpret_cast<unsigned*>(status), n, 0u, stream));
    const bool restore = restored_out != nullptr;
    double* cbeam = cbeam_out;
    int* rrad = dev_alloc<int>(C->rrad, n);
    if (restore || cbeam_out) {
      if (!cbeam) cbeam = dev_alloc<double>(C->cbeam, 6 * (size_t)n);
      HIPCHK(launch_beamfit(static_cast<const InstDesc*>(P->inst.p), n, beam, cbeam, rrad, status, stream));
    }
    int* cidx = comp_idx;
    double* cflx = comp_flux;
    if (!cidx && restore) {
      cidx = dev_alloc<int>(C->comp_idx, (size_t)std::max<int64_t>(C->total_comp, 1));
      cflx = dev_alloc<double>(C->comp_flux, (size_t)std::max<int64_t>(C->total_comp, 1));
    }
    HIPCHK(launch_fill_u32(static_cast<unsigned*>(C->slots.p), C->n_slots * 2, 0u, stream));
    // beams that are exactly point-symmetric let CLEAN read half its window mirrored
    int* asym = dev_alloc<int>(C->asym, n);
    HIPCHK(launch_fill_u32(reinterpret_cast<unsigned*>(asym), n, 0u, stream));
    HIPCHK(launch_beam_symcheck(static_cast<const InstDesc*>(P->inst.p), n, P->max_N, beam, asym, stream));
    CleanArgs A{};
    A.inst = static_cast<const InstDesc*>(P->inst.p);
    A.team_off = static_cast<const int*>(C->team_off.p);
    A.team_imgs = static_cast<const int*>(C->team_imgs.p);
    A.blk = static_cast<const int2*>(C->blk.p);
    A.team_G = static_cast<const int*>(C->team_G.p);
    A.team_slot = static_cast<const int64_t*>(C->team_slot.p);
    A.sub_px = C->sub_px;
    A.dirty = dirty;
    A.beam = beam;
    A.niter = static_cast<const int*>(C->niter_d.p);
    A.thr = prm->threshold_dev ? prm->threshold_dev : (has_thr ? static_cast<const float*>(C->thr_d.p) : nullptr);
    A.win = n_win ? static_cast<const int4*>(C->win_d.p) : nullptr;
    A.gain = prm->gain;
    A.posonly = prm->positive_only ? 1 : 0;
    A.cbeam = restore ? cbeam : nullptr;
    A.rrad = rrad;
    A.resid = residual_out;
    A.model = model_out;
    A.comp_off = static_cast<const int64_t*>(C->comp_off.p);
    A.comp_idx = cidx;
    A.comp_flux = cflx;
    A.ncomp = n_comp_out;
    A.restored = restored_out;
    A.slots = static_cast<unsigned long long*>(C->slots.p);
    A.asym = asym;
    A.status = status;
    A.poll_limit = ctx->clean_stall ? 256u : 0u;
    A.test_stall = ctx->clean_stall;
    hipEvent_t pe = prof_start(ctx, MI_PROF_CLEAN, stream);
    HIPCHK(launch_clean(A, C->ppt, C->local != 0, C->n_blocks, C->lds, stream));
    prof_stop(pe, stream);
  });
}

mi_status mi_hogbom_clean_noalloc(mi_ctx* ctx, const mi_batch* batch, const float* dirty, const float* beam,
                                  const mi_clean_params* prm, float* residual_out, double* model_out,
                                  int32_t* comp_idx, double* comp_flux, int32_t* n_comp_out, float* restored_out,
                                  double* cbeam_out, hipStream_t stream) {
  return guard(ctx, [&] {
    need(dirty, "dirty");
    need(beam, "beam");
    need(prm, "params");
    need(residual_out, "residual_out");
    need(prm->niter, "params->niter");
    if ((comp_idx == nullptr) != (comp_flux == nullptr)) fail(MI_ERR_ARG, "comp_idx and comp_flux: both or neither");
    if (!(prm->gain > 0.0f && prm->gain <= 1.0f)) fail(MI_ERR_ARG, "gain must be in (0, 1]");
    if (prm->window) fail(MI_ERR_UNSUPPORTED, "the no-allocation CLEAN takes no peak-search windows");
    check_batch(batch);
    const int n = batch->n_inst;
    if (n > NA_MAX_INST) fail(MI_ERR_UNSUPPORTED, "the no-allocation CLEAN takes at most %d instances (got %d)",
                              NA_MAX_INST, n);
    const int N = batch->n_img[0];
    for (int i = 0; i < n; ++i) {
      if (batch->n_img[i] != N) fail(MI_ERR_UNSUPPORTED, "the no-allocation CLEAN needs one image size per batch");
      if (prm->niter[i] < 0) fail(MI_ERR_ARG, "niter[%d] < 0", i);
    }
    const int req = prm->team_size;
    if (req != 0 && (!is_pow2(req) || req > 256)) fail(MI_ERR_ARG, "team_size must be 0 or a power of two <= 256");
    if (!ctx->noalloc_scratch) fail(MI_ERR_UNSUPPORTED, "no scratch array for device %d", ctx->device);
    HIPCHK(hipSetDevice(ctx->device));
    // team shape: the allocating entry point's policy for a batch of one image size
    const int g_min = std::max(1, (N * N) / 65536), g_cap = std::min(256, N);
    if (g_min > g_cap) fail(MI_ERR_UNSUPPORTED, "CLEAN team too large for N = %d", N);
    int G = g_min;
    if (req) {
      G = 1;
      while (G * 2 <= req) G *= 2;
      G = std::min(std::max(G, g_min), g_cap);
    } else {
      while (G * 2 <= std::min(32, g_cap) && G * 2 * n <= 256) G *= 2;
    }
    int ppt = 4;
    while ((int64_t)ppt * 1024 * G < (int64_t)N * N) ppt *= 2;
    const bool local = G <= 32;
    const int sub_px = (int)std::min<int64_t>((int64_t)N * N / G, CLEAN_RESTORE_SUB_PX);
    const size_t lds = (size_t)sub_px * sizeof(float);
    int per_cu = 0;
    HIPCHK(clean_max_blocks_per_cu(ppt, local, false, lds, &per_cu));
    int cap = per_cu * ctx->n_cu;
    if (local) cap -= cap % 8;
    // teams of up to 32 are dealt over the 8 XCDs a row of teams at a time
    const int t_max = local ? 8 * ((cap / G) / 8) : cap / G;
    if (t_max < 1) fail(MI_ERR_UNSUPPORTED, "CLEAN teams of %d workgroups do not fit the device", G);
    const int T = std::min(n, t_max);
    // images to teams: longest first, each to the least-loaded team (fixed-size host arrays)
    NaSetup S;
    std::memset(&S, 0, sizeof S);
    S.n = n;
    S.N = N;
    S.log2N = ilog2i(N);
    S.G = G;
    S.T = T;
    S.local = local ? 1 : 0;
    S.n_blocks = local ? 8 * ((T + 7) / 8) * G : T * G;
    S.has_thr = prm->threshold != nullptr && prm->threshold_dev == nullptr;
    S.status = batch->status;
    int order[NA_MAX_INST], team_of[NA_MAX_INST], fill[NA_MAX_INST + 1];
    double load[NA_MAX_INST];
    for (int i = 0; i < n; ++i) {
      order[i] = i;
      S.niter[i] = prm->niter[i];
      S.thr[i] = S.has_thr ? prm->threshold[i] : 0.0f;
    }
    for (int k = 1; k < n; ++k)               // stable insertion sort, longest first
      for (int j = k; j > 0 && prm->niter[order[j - 1]] < prm->niter[order[j]]; --j) std::swap(order[j - 1], order[j]);
    for (int t = 0; t < T; ++t) load[t] = 0.0;
    for (int k = 0; k < n; ++k) {
      int t = 0;
      for (int u = 1; u < T; ++u)
        if (load[u] < load[t]) t = u;
      team_of[order[k]] = t;
      load[t] += (double)prm->niter[order[k]] + 1.0;
    }
    for (int t = 0; t <= T; ++t) fill[t] = 0;
    for (int i = 0; i < n; ++i) ++fill[team_of[i] + 1];
    for (int t = 0; t < T; ++t) fill[t + 1] += fill[t];
    for (int t = 0; t <= T; ++t) S.team_off[t] = (int16_t)fill[t];
    for (int k = 0; k < n; ++k) {             // keep the LPT order within each team
      const int i = order[k];
      S.team_imgs[fill[team_of[i]]++] = (int16_t)i;
    }
    int64_t total_comp = 0;
    for (int i = 0; i < n; ++i) total_comp += prm->niter[i];
    const bool restore = restored_out != nullptr;
    const bool own_comp = restore && comp_idx == nullptr;
    // scratch layout (256-byte aligned pieces)
    int64_t off = 0;
    auto take = [&](int64_t bytes) { const int64_t o = off; off += (bytes + 255) / 256 * 256; return o; };
    S.o_inst = take((int64_t)sizeof(InstDesc) * n);
    S.o_team_off = take(4LL * (T + 1));
    S.o_team_imgs = take(4LL * n);
    S.o_blk = take(8LL * S.n_blocks);
    S.o_team_G = take(4LL * T);
    S.o_team_slot = take(8LL * T);
    S.o_niter = take(4LL * n);
    S.o_thr = take(4LL * n);
    S.o_comp_off = take(8LL * n);
    S.n_slots = 2 * G * T;
    S.o_slots = take(8LL * S.n_slots);
    S.o_asym = take(4LL * n);
    S.o_rrad = take(4LL * n);
    S.o_cbeam = take(48LL * n);
    S.o_cidx = own_comp ? take(4 * std::max<int64_t>(total_comp, 1)) : 0;
    S.o_cflx = own_comp ? take(8 * std::max<int64_t>(total_comp, 1)) : 0;
    if ((size_t)off > NA_SCRATCH_BYTES)
      fail(MI_ERR_UNSUPPORTED, "the call needs %lld bytes of scratch, more than the %zu the no-allocation CLEAN has "
           "(restore with component outputs of your own, or fewer iterations)", (long long)off, NA_SCRATCH_BYTES);
    unsigned char* base = ctx->noalloc_scratch;
    hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(256), 0, stream, base, S);
    HIPCHK(hipGetLastError());
    const InstDesc* inst = reinterpret_cast<const InstDesc*>(base + S.o_inst);
    int* rrad = reinterpret_cast<int*>(base + S.o_rrad);
    double* cbeam = cbeam_out ? cbeam_out : reinterpret_cast<double*>(base + S.o_cbeam);
    if (restore || cbeam_out) HIPCHK(launch_beamfit(inst, n, beam, cbeam, rrad, batch->status, stream));
    int* asym = reinterpret_cast<int*>(base + S.o_asym);
    HIPCHK(launch_beam_symcheck(inst, n, N, beam, asym, stream));
    CleanArgs A{};
    A.inst = inst;
    A.team_off = reinterpret_cast<const int*>(base + S.o_team_off);
    A.team_imgs = reinterpret_cast<const int*>(base + S.o_team_imgs);
    A.blk = reinterpret_cast<const int2*>(base + S.o_blk);
    A.team_G = reinterpret_cast<const int*>(base + S.o_team_G);
    A.team_slot = reinterpret_cast<const int64_t*>(base + S.o_team_slot);
    A.sub_px = sub_px;
    A.dirty = dirty;
    A.beam = beam;
    A.niter = reinterpret_cast<const int*>(base + S.o_niter);
    A.thr = prm->threshold_dev ? prm->threshold_dev : (S.has_thr ? reinterpret_cast<const float*>(base + S.o_thr)
                                                                  : nullptr);
    A.win = nullptr;
    A.gain = prm->gain;
    A.posonly = prm->positive_only ? 1 : 0;
    A.cbeam = restore ? cbeam : nullptr;
    A.rrad = rrad;
    A.resid = residual_out;
    A.model = model_out;
    A.comp_off = reinterpret_cast<const int64_t*>(base + S.o_comp_off);
    A.comp_idx = own_comp ? reinterpret_cast<int*>(base + S.o_cidx) : comp_idx;
    A.comp_flux = own_comp ? reinterpret_cast<double*>(base + S.o_cflx) : comp_flux;
    A.ncomp = n_comp_out;
    A.restored = restored_out;
    A.slots = reinterpret_cast<unsigned long long*>(base + S.o_slots);
    A.asym = asym;
    A.status = batch->status;
    A.poll_limit = ctx->clean_stall ? 256u : 0u;
    A.test_stall = ctx->clean_stall;
    HIPCHK(launch_clean(A, ppt, local, S.n_blocks, lds, stream));
  });
}

mi_status mi_steer_clean(mi_ctx* ctx, const mi_batch* batch, const float* dirty, const float* beam,
                         const mi_steer_params* prm, float* residual_out, double* model_out, int32_t* n_cycle_out,
                         double* log_out, uint32_t* mask_out, float* restored_out, double* cbeam_out,
                         hipStream_t stream) {
  return guard(ctx, [&] {
    need(dirty, "dirty");
    need(beam, "beam");
    need(prm, "params");
    need(residual_out, "residual_out");
    need(prm->ncycle, "params->ncycle");
    if (!(prm->gain > 0.0f && prm->gain <= 1.0f)) fail(MI_ERR_ARG, "gain must be in (0, 1]");
    if (!(prm->trim > 0.0f && prm->trim <= 1.0f)) fail(MI_ERR_ARG, "trim must be in (0, 1]");
    for (const void* q : {static_cast<const void*>(dirty), static_cast<const void*>(residual_out),
                          static_cast<const void*>(restored_out), static_cast<const void*>(model_out)})
      if (reinterpret_cast<uintptr_t>(q) % 16) fail(MI_ERR_ARG, "image pointers must be 16-byte aligned");
    HIPCHK(hipSetDevice(ctx->device));
    Plan* P = get_plan(ctx, batch, stream);
    const int n = P->n_inst;
    for (int i = 0; i < n; ++i)
      if (prm->ncycle[i] < 0) fail(MI_ERR_ARG, "ncycle[%d] < 0", i);
    if (!P->steer) {                                   // work lists and workspaces of the batch
      if (capturing(stream)) fail(MI_ERR_UNSUPPORTED, "the first Steer CLEAN call on a batch cannot be captured");
      auto B = std::make_unique<SteerBase>();
      B->elems = 2 * P->max_N > 4096 ? 8192 : 4096;   // LDS block of the transform passes
      std::vector<FftWork> rows, rows2, cols, pix;
      for (int i = 0; i < n; ++i) {
        const int N = P->n[i], Pn = 2 * N;
        const int rb = std::min(8, 2 * B->elems / Pn), ncol = B->elems / Pn;
        B->rb.push_back(rb);
        B->x_off.push_back(B->total_x);
        B->s_off.push_back(B->total_s);
        B->total_x += 2LL * N * (N + 1);
        B->total_s += (int64_t)(N + 1) * Pn;
        for (int y = 0; y < N; y += rb) rows.push_back({i, y});
        for (int y = 0; y < Pn; y += rb) rows2.push_back({i, y});
        for (int kx = 0; kx <= N; kx += ncol) cols.push_back({i, kx});
        for (int p = 0; p < N * N; p += ST_PIX_PER_ITEM) pix.push_back({i, p});
      }
      upload(B->rows, rows);
      upload(B->rows2, rows2);
      upload(B->cols, cols);
      upload(B->pix, pix);
      B->n_rows = B->n_inv = (int)rows.size();
      B->n_rows2 = (int)rows2.size();
      B->n_cols = (int)cols.size();
      B->n_pix = (int)pix.size();
      dev_alloc<float2>(B->X, (size_t)B->total_x);
      dev_alloc<float2>(B->S, (size_t)B->total_s);
      dev_alloc<float>(B->D, (size_t)P->total_img);
      P->steer = std::move(B);
    }
    SteerBase* B = P->steer.get();
    // per parameter set: descriptors (offsets, caps, host thresholds) and control words
    const bool has_thr = prm->threshold != nullptr && prm->threshold_dev == nullptr;
    uint64_t h = fnv1a(prm->ncycle, sizeof(int32_t) * n);
    if (has_thr) h = fnv1a(prm->threshold, sizeof(float) * n, h ^ 0x9e3779b97f4a7c15ull);
    auto it = P->steers.find(h);
    SteerPlan* S = nullptr;
    if (it != P->steers.end() && it->second->has_thr == has_thr &&
        std::equal(it->second->ncycle.begin(), it->second->ncycle.end(), prm->ncycle) &&
        (!has_thr || std::equal(it->second->thr.begin(), it->second->thr.end(), prm->threshold))) {
      S = it->second.get();
      touch(ctx, S, stream);
    } else {
      if (it != P->steers.end()) {
        if (it->second->pinned) fail(MI_ERR_UNSUPPORTED, "Steer plan collision with a plan held by a captured graph");
        P->steers.erase(it);
      }
      make_room(P->steers, 8, stream);
      auto up = std::make_unique<SteerPlan>();
      S = up.get();
      S->ncycle.assign(prm->ncycle, prm->ncycle + n);
      S->has_thr = has_thr;
      if (has_thr) S->thr.assign(prm->threshold, prm->threshold + n);
      std::vector<SteerInst> si(n);
      int64_t ctl = 0, lg = 0, mk = 0;
      for (int i = 0; i < n; ++i) {
        const int N = P->n[i];
        SteerInst& d = si[i];
        std::memset(&d, 0, sizeof d);
        d.x_off = B->x_off[i];
        d.s_off = B->s_off[i];
        d.ctl_off = ctl;
        d.log_off = lg;
        d.mask_off = mk;
        d.ncycle = prm->ncycle[i];
        d.rb = B->rb[i];
        d.thr = has_thr ? prm->threshold[i] : 0.0f;
        ctl += 4 + d.ncycle;
        lg += 3LL * d.ncycle;
        mk += (int64_t)d.ncycle * N * N / 32;
        S->kmax = std::max(S->kmax, d.ncycle);
      }
      S->total_ctl = ctl;
      upload(S->sti, si);
      dev_alloc<unsigned>(S->ctl, (size_t)ctl);
      dev_alloc<double>(S->cbeam, 6 * (size_t)n);
      dev_alloc<int>(S->rrad, (size_t)n);
      touch(ctx, S, stream);
      P->steers[h] = std::move(up);
    }
    int* status = batch->status;
    if (status) HIPCHK(launch_fill_u32(reinterpret_cast<unsigned*>(status), n, 0u, stream));
    HIPCHK(launch_fill_u32(static_cast<unsigned*>(S->ctl.p), S->total_ctl, 0u, stream));
    SteerArgs A{};
    A.inst = static_cast<const InstDesc*>(P->inst.p);
    A.sti = static_cast<const SteerInst*>(S->sti.p);
    A.thr_dev = prm->threshold_dev;
    A.gain = prm->gain;
    A.trim = prm->trim;
    A.posonly = prm->positive_only ? 1 : 0;
    A.dirty = dirty;
    A.beam = beam;
    A.R = residual_out;
    A.model = model_out ? model_out : dev_alloc<double>(B->model_ws, (size_t)P->total_img);
    A.D = static_cast<float*>(B->D.p);
    A.X = static_cast<float2*>(B->X.p);
    A.S = static_cast<float2*>(B->S.p);
    A.ctl = static_cast<unsigned*>(S->ctl.p);
    A.log = log_out;
    A.mask = mask_out;
    A.ncyc_out = n_cycle_out;
    A.restored = restored_out;
    A.T = ctx->T;
    const FftWork* w_rows = static_cast<const FftWork*>(B->rows.p);
    const FftWork* w_rows2 = static_cast<const FftWork*>(B->rows2.p);
    const FftWork* w_cols = static_cast<const FftWork*>(B->cols.p);
    const FftWork* w_pix = static_cast<const FftWork*>(B->pix.p);
    // the beam's spectrum, then R = dirty and the first peaks
    A.iter = 0;
    A.work = w_rows2;
    HIPCHK(launch_st_rows(2, B->elems, B->n_rows2, A, stream));
    A.work = w_cols;
    HIPCHK(launch_st_cols(0, B->elems, B->n_cols, A, stream));
    A.work = w_pix;
    HIPCHK(launch_st_init(B->n_pix, A, stream));
    A.iter = 1;
    for (int k = 0; k < S->kmax; ++k) {
      A.k = k;
      A.work = w_rows;
      HIPCHK(launch_st_rows(0, B->elems, B->n_rows, A, stream));
      A.work = w_cols;
      HIPCHK(launch_st_cols(1, B->elems, B->n_cols, A, stream));
      A.work = w_rows;
      HIPCHK(launch_st_rows_inv(0, B->elems, B->n_inv, A, stream));
      A.work = w_pix;
      HIPCHK(launch_st_update(B->n_pix, A, stream));
    }
    if (restored_out || cbeam_out) {
      double* cb = cbeam_out ? cbeam_out : static_cast<double*>(S->cbeam.p);
      HIPCHK(launch_beamfit(A.inst, n, beam, cb, static_cast<int*>(S->rrad.p), status, stream));
      if (restored_out) {
        // the clean beam's spectrum replaces the dirty beam's; restored = R + model (*) Gaussian
        A.iter = 0;
        A.cbeam = cb;
        A.work = w_rows2;
        HIPCHK(launch_st_rows(3, B->elems, B->n_rows2, A, stream));
        A.work = w_cols;
        HIPCHK(launch_st_cols(0, B->elems, B->n_cols, A, stream));
        A.work = w_rows;
        HIPCHK(launch_st_rows(1, B->elems, B->n_rows, A, stream));
        A.work = w_cols;
        HIPCHK(launch_st_cols(1, B->elems, B->n_cols, A, stream));
        A.work = w_rows;
        HIPCHK(launch_st_rows_inv(1, B->elems, B->n_inv, A, stream));
      }
    }
  });
}

mi_status mi_degrid(mi_ctx* ctx, const mi_batch* batch, const float* image, const float* uv, const float* w_in,
                    int adjoint, mi_c64* vis_out, hipStream_t stream) {
  return guard(ctx, [&] {
    need(image, "image");
    need(uv, "uv");
    need(w_in, "w_in");
    need(vis_out, "vis_out");
    if (adjoint != 0 && adjoint != 1) fail(MI_ERR_ARG, "adjoint must be 0 or 1");
    HIPCHK(hipSetDevice(ctx->device));
    Plan* P = get_plan(ctx, batch, stream);
    run_bin(ctx, P, batch, uv, w_in, false, stream);
    double2* g = dev_alloc<double2>(P->gd, P->total_gd);
    const InstDesc* inst = static_cast<const InstDesc*>(P->inst.p);
    HIPCHK(launch_fft_b_r2c(P->elems_d, ctx->n_cu, inst, static_cast<const FftWork*>(P->wb_d.p), P->n_wb_d, image, ctx->T, g,
                            stream));
    HIPCHK(launch_fft_a_fwd(P->elems_d, ctx->n_cu, inst, static_cast<const FftWork*>(P->wa_d.p), P->n_wa_d, ctx->T, g, stream));
    HIPCHK(launch_degrid(inst, P->n_inst, P->max_nvis, reinterpret_cast<const float2*>(uv), w_in,
                         static_cast<const float*>(P->wts.p), static_cast<const double*>(P->b0.p), g, ctx->T,
                         adjoint, reinterpret_cast<float2*>(vis_out), stream));
  });
}

mi_status mi_predict_transpose(mi_ctx* ctx, const mi_batch* batch, const mi_c64* vis, const float* uv,
                               const float* w_in, float* image_out, hipStream_t stream) {
  return guard(ctx, [&] {
    need(vis, "vis");
    need(uv, "uv");
    need(w_in, "w_in");
    need(image_out, "image_out");
    HIPCHK(hipSetDevice(ctx->device));
    Plan* P = get_plan(ctx, batch, stream);
    if (!P->b0_two.p) upload(P->b0_two, std::vector<double>(2 * (size_t)P->n_inst, 2.0));
    // unit weights on the kept samples, the dirty-image transform, then 1/(2 corr) per axis
    // pair instead of 1/(corr B0): Re I_raw / (2 corr) = P^T v
    run_bin(ctx, P, batch, uv, w_in, false, stream, true, P->fused, vis);
    if (P->fused) {
      run_dirty_fused(ctx, P, vis, uv, w_in, image_out, stream, static_cast<const double*>(P->b0_two.p));
    } else {
      double2* gd = dev_alloc<double2>(P->gd, P->total_gd);
      run_grid<double2>(ctx, P, vis, uv, w_in, false, gd, 1, stream);
      run_image(ctx, P, image_out, stream, static_cast<const double*>(P->b0_two.p));
    }
  });
}

}  // extern "C"
