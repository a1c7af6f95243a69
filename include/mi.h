/*
 * mi.h -- C ABI of the MI355X (gfx950) imaging hot path for MUSER-style solar
 * radio-interferometric data (Mei et al., "GPU-Based High-Performance Imaging for
 * Mingantu Spectral RadioHeliograph").
 *
 * The calls follow the paper's statement of the imaging problem (Algorithm 1):
 *   dirty_image(visibilities, UVW, weight_mode) -> dirty image, dirty beam, clean beam
 *   CLEAN: find the peak, subtract the beam at the loop gain, repeat until the peak
 *   falls to a threshold (Sec. 4.3), then restore.
 * plus the adjoint of the imaging operator (FFT then degrid).
 *
 * Conventions shared by every entry point
 *  - All data pointers are DEVICE pointers owned by the caller unless marked "host".
 *    The library never allocates or frees caller-visible memory.
 *  - Every call is asynchronous on the given HIP stream (0 = the null stream).  The
 *    first call with a new batch descriptor builds a plan (workspace, device tables) and
 *    may synchronise once; later calls with an identical descriptor do not synchronise.
 *    The same holds for a new set of CLEAN parameters (mi_hogbom_clean, mi_steer_clean:
 *    caps and host thresholds), new w_max / phase_tol (mi_dirty_image_w) and new radii
 *    (mi_disk_offsets): each of those calls uploads its tables synchronously once; repeats
 *    with the same values do not.  No other call synchronises.
 *  - Graph capture: a call whose plan already exists (run it once outside the capture)
 *    can be captured into a HIP graph; its plan is then kept for the context's lifetime.
 *    A call that would build a new plan while its stream is capturing returns
 *    MI_ERR_UNSUPPORTED.  Other plans are evicted least recently used first (at most 16
 *    batch descriptors, 8 CLEAN and 8 Steer CLEAN parameter sets per descriptor, 16
 *    transform layouts).
 *  - Argument errors are detected on the host before any launch; the call then returns
 *    a nonzero mi_status, writes nothing, and mi_last_error() describes the problem.
 *  - Per-instance problems (no kept visibilities, ...) do not abort the batch: they are
 *    reported through batch->status (device int32 per instance, MI_INST_* bits).
 *  - No C++ exception crosses this interface.  A context is not thread-safe: use one
 *    context per host thread/stream.
 *  - Images are row-major [y][x] float32.  Pixel (x, y) is at (l, m) =
 *    ((x - N/2) dl, (y - N/2) dl).  Visibilities follow V = sum I exp(-2 pi i (ul + vm));
 *    the imager uses exp(+2 pi i (ul + vm)).
 *  - uv are (u, v) pairs in wavelengths, float32 [M][2]; w_in are input weights,
 *    float32 [M] (a visibility with w_in <= 0 is flagged and ignored).
 *  - Gridding kernel: truncated prolate spheroidal function (Sec. 3.2.3), support 7
 *    cells, alpha = 1, tabulated at 128 points per cell, with grid correction.
 *  - Image sizes N are powers of two in [64, 4096]; the dirty beam is 2N x 2N ("twice
 *    as large as the image", Sec. 3.2.1) with the same pixel size, peak 1 at (N, N).
 */
#ifndef MI_H
#define MI_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } mi_c64;
typedef int mi_status;
typedef struct mi_ctx mi_ctx;

enum {
  MI_OK = 0,
  MI_ERR_ARG = 1,          /* NULL pointer, bad enum, negative count, ...            */
  MI_ERR_SHAPE = 2,        /* N not a power of two in [64, 4096], bad offsets, ...    */
  MI_ERR_UNSUPPORTED = 3,  /* valid request the library does not implement           */
  MI_ERR_NOMEM = 4,        /* workspace allocation failed                            */
  MI_ERR_DEVICE = 5,       /* a HIP runtime call failed                              */
  MI_ERR_INSTANCE = 6      /* reserved for callers that fold status[] into one code  */
};

/* Per-instance status bits written to batch->status (0 = fine). */
enum {
  MI_INST_EMPTY = 1,          /* no visibility kept (all flagged or off the grid)     */
  MI_INST_LOBE_CLIPPED = 2,   /* clean-beam main lobe reached the fit box edge        */
  MI_INST_RESTORE_CLIPPED = 4,/* restoring Gaussian wider than the restore window     */
  MI_INST_TEST_FAILED = 8,    /* forced by MI_TEST_FAIL_INSTANCE (failure-path tests) */
  MI_INST_ABORTED = 16        /* a CLEAN team barrier timed out; outputs incomplete     */
};

/* Weighting mode, as Algorithm 1's wgtGrid_kernel: mode 1 = uniform, otherwise natural. */
enum { MI_NATURAL = 0, MI_UNIFORM = 1 };

/* Grid layouts returned by mi_grid. */
enum {
  MI_LAYOUT_FULL = 0,  /* full centred P x P complex grid G[j][i], cell (i-P/2, j-P/2) */
  MI_LAYOUT_HALF = 1   /* half plane u <= 0: P/2 lines (u index i = 1..P/2), each P long
                          in v: H[i-1][j] = G[j][i]                                      */
};

/* A batch of independent imaging instances (channel x snapshot x polarisation). */
typedef struct {
  int32_t n_inst;              /* number of instances, >= 1                           */
  const int64_t* vis_offset;   /* host, n_inst+1, CSR offsets into vis/uv/w_in         */
  const int32_t* n_img;        /* host, n_inst, image size N per instance              */
  const double* cell_rad;      /* host, n_inst, pixel size dl in radians (> 0)         */
  const int8_t* weight_mode;   /* host, n_inst, MI_NATURAL or MI_UNIFORM               */
  int32_t* status;             /* device, n_inst, MI_INST_* bits; may be NULL          */
} mi_batch;

/* CLEAN parameters (Sec. 4.3: loop gain gamma = 0.1; stop when the peak reaches the
 * threshold, or after niter components). */
typedef struct {
  float gain;                  /* loop gain in (0, 1]                                  */
  const int32_t* niter;        /* host, n_inst, component cap per instance (>= 0)      */
  const float* threshold;      /* host, n_inst, stop when |peak| <= threshold; or NULL */
  int32_t positive_only;       /* 0: peak of |R| (default); 1: peak of R               */
  int32_t team_size;           /* workgroups per image (power of two); 0 = automatic.
                                  Values up to 32 keep an image on one XCD; larger teams
                                  spread one image over several XCDs (the "plain" path) */
  const float* threshold_dev;  /* device, n_inst, or NULL: thresholds read on the device
                                  (e.g. mu_a from mi_gmm_levels); overrides `threshold` */
  const int32_t* window;       /* host, 4 per instance (x0, y0, x1, y1), or NULL: the peak
                                  is searched only in the half-open box x0 <= x < x1,
                                  y0 <= y < y1 (0 <= x0 < x1 <= N, likewise y); the
                                  subtraction still covers the whole map.  NULL = whole
                                  maps (the paper does not window its CLEAN)           */
} mi_clean_params;

/* Steer CLEAN parameters (the Steer-Dewdney-Ito CLEAN of Sec. 2 and Sec. 4.3; Algorithm 1
 * runs it with gain 0.1 until the peak reaches the sky level). */
typedef struct {
  float gain;                  /* loop gain in (0, 1]: the largest subtracted value is
                                  gain x peak                                          */
  float trim;                  /* (0, 1]: pixels with |R| >= trim x peak are components  */
  const int32_t* ncycle;       /* host, n_inst, iteration cap per instance (>= 0)       */
  const float* threshold;      /* host, n_inst, stop when the peak <= threshold; or NULL */
  const float* threshold_dev;  /* device, n_inst, or NULL; overrides `threshold`         */
  int32_t positive_only;       /* 0: peak and selection on |R|; 1: on R                 */
} mi_steer_params;

/* Create / destroy a context on HIP device `device`.  The context owns plans,
 * workspaces and constant tables. */
mi_status mi_ctx_create(mi_ctx** ctx, int device);
mi_status mi_ctx_destroy(mi_ctx* ctx);
/* Text of the last error on this context ("" if none).  Owned by the context. */
const char* mi_last_error(const mi_ctx* ctx);
/* Library version string (static). */
const char* mi_version(void);

/* Convolutional gridding with natural or uniform weighting (Sec. 3.2.3; Algorithm 1,
 * wgtGrid_kernel).  For every kept visibility (w_in > 0 and its nearest cell c within
 * |c| <= N/2 - 4 in both axes) and its Hermitian mirror, adds w * V * K to the 7 x 7
 * cells around it.  Uniform weights are w_in / (sum of w_in over all samples, mirrors
 * included, whose nearest N-grid cell is the same).
 *   which  = 0: dirty grid (complex, N x N, cell du = 1/(N dl)),
 *            1: beam grid (V = 1, 2N x 2N, cell du/2; imaginary part 0),
 *            2: both, dirty grids of all instances first, then beam grids.
 *   layout = MI_LAYOUT_FULL or MI_LAYOUT_HALF; instances are packed back to back in
 *            grid_out (P*P resp. P*P/2 complex each, P = N or 2N).
 *   b0_out (device, optional): double [n_inst][2] = B0 of the N grid and of the 2N grid
 *            (transform of the weight grid at the centre divided by corr(0)^2).
 *   n_kept_out (device, optional): int32 [n_inst] kept input visibilities.       */
mi_status mi_grid(mi_ctx* ctx, const mi_batch* batch, const mi_c64* vis, const float* uv,
                  const float* w_in, int which, int layout, mi_c64* grid_out,
                  double* b0_out, int32_t* n_kept_out, hipStream_t stream);

/* In-place, unnormalised, centred 2-D inverse DFT of complex P x P arrays (the transform
 * that turns the grid into the dirty image, Sec. 3.2.3):
 *   I[y][x] = sum_{j,i} G[j][i] exp(+2 pi i ((i-P/2)(x-P/2) + (j-P/2)(y-P/2)) / P).
 *   n (host, n_inst): P per array, power of two in [64, 8192];
 *   offs (host, n_inst): element offset of each array in data (complex elements). */
mi_status mi_ifft2(mi_ctx* ctx, mi_c64* data, const int32_t* n, const int64_t* offs,
                   int32_t n_inst, hipStream_t stream);

/* Dirty image (Algorithm 1, dirty_image): grid, inverse FFT, grid correction and
 * normalisation so that a point source of flux S at the phase centre images to S.
 *   dirty_out: float32, N*N per instance, packed back to back.
 *   beam_out (optional): float32, (2N)^2 per instance -- the dirty beam, as from
 *            mi_dirty_beam, computed from the same prep pass.
 *   b0_out (optional): double [n_inst][2], as in mi_grid.
 * An instance with no kept visibility gets an all-zero image and MI_INST_EMPTY.    */
mi_status mi_dirty_image(mi_ctx* ctx, const mi_batch* batch, const mi_c64* vis,
                         const float* uv, const float* w_in, float* dirty_out,
                         float* beam_out, double* b0_out, hipStream_t stream);

/* Dirty beam (Algorithm 1, gpu_dpsf): the image of unit visibilities on the 2N grid
 * (Sec. 3.2.1), normalised to exactly 1 at (N, N).  beam_out: (2N)^2 per instance. */
mi_status mi_dirty_beam(mi_ctx* ctx, const mi_batch* batch, const float* uv,
                        const float* w_in, float* beam_out, hipStream_t stream);

/* w-projection parameters (Sec. 3.2.2, 6.1). */
typedef struct {
  const double* w_max;         /* host, n_inst: bound on |w| (wavelengths) of each
                                  instance's visibilities                              */
  double phase_tol;            /* radians; 0 = 0.1, the phase error the paper tolerates */
} mi_wproj_params;

/* Dirty image with the w-term corrected by w-projection (Sec. 3.2.2, 6.1; Algorithm 1's
 * W-term correction).  w_lambda: float32 [M], the w coordinate of each visibility in
 * wavelengths.  With r2 = l^2 + m^2 at the field corner and dw = phase_tol / (pi r2),
 * instance i uses the planes w_j = j dw, j = 0 .. floor(w_max[i] / dw + 1/2) (one plane,
 * i.e. no correction, when pi w_max r2 <= phase_tol / 2); each visibility is gridded with
 * the kernel of the plane nearest to |w| (halves rounded up; the last plane for |w| beyond
 * it, or not finite), conjugated for w < 0: the field's transform of
 * corr(l) corr(m) exp(+2 pi i w_j (sqrt(1 - l^2 - m^2) - 1)), tabulated at 16 points per
 * cell over a support of 2 (3 + ceil(w_j sqrt(r2) N dl)) + 1 cells and interpolated
 * bilinearly.  Weighting, transform, correction and B0 are those of mi_dirty_image.
 * n_planes_out (host, n_inst, optional) receives the planes used per instance.  Kernel
 * tables are built on the device when w_max or phase_tol change (the call then
 * synchronises once).  MI_ERR_ARG for a negative or non-finite w_max;
 * MI_ERR_UNSUPPORTED for N < 64 or a support above 63 cells.  The dirty beam does not
 * depend on w (use mi_dirty_beam). */
mi_status mi_dirty_image_w(mi_ctx* ctx, const mi_batch* batch, const mi_c64* vis, const float* uv,
                           const float* w_lambda, const float* w_in, const mi_wproj_params* params,
                           float* dirty_out, double* b0_out, int32_t* n_planes_out, hipStream_t stream);

/* Hogbom CLEAN with restore (Algorithm 1, improved_clean; Sec. 4.3).
 *   dirty: float32 N*N per instance; beam: float32 (2N)^2 per instance (peak at (N, N)).
 *   N: every image size of the batch, 64 ... 4096 (each member of a team keeps 64K
 *   residual pixels in registers, so 4096^2 takes all 256 compute units for one image;
 *   MI_ERR_UNSUPPORTED if the teams cannot be resident together).
 *   Per iteration: p = argmax |R| over the window (ties: lowest y*N + x), stop if
 *   |R[p]| <= threshold,
 *   f = gain * R[p] (double), model[p] += f, R -= f * beam[y - p_y + N][x - p_x + N].
 *   residual_out: float32 N*N; model_out: double N*N (optional);
 *   comp_idx (int32) / comp_flux (double): niter[i] slots per instance, packed back to
 *   back in instance order (optional, both or neither); n_comp_out: int32 [n_inst]
 *   components taken (optional);
 *   restored_out (optional): residual + components convolved with the clean beam, a
 *   Gaussian fitted to the beam's main lobe (4-connected, beam > 0.35);
 *   cbeam_out (optional): double [n_inst][6] = a, b, c of exp(-(a dx^2 + b dx dy +
 *   c dy^2)) in pixels, FWHM major and minor axes (pixels), position angle (radians,
 *   major axis from +x towards +y, in [0, pi)).
 * The whole loop runs inside one persistent launch: each image is owned by a team of
 * workgroups that keeps the residual in registers.                                    */
mi_status mi_hogbom_clean(mi_ctx* ctx, const mi_batch* batch, const float* dirty,
                          const float* beam, const mi_clean_params* params,
                          float* residual_out, double* model_out, int32_t* comp_idx,
                          double* comp_flux, int32_t* n_comp_out, float* restored_out,
                          double* cbeam_out, hipStream_t stream);

/* Hogbom CLEAN that allocates nothing, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid it).  Same
 * arguments and results as mi_hogbom_clean; every table it needs (instance descriptors,
 * team schedule, exchange slots, symmetry flags, clean-beam parameters and, when restoring
 * without component outputs, the component lists) lives in one fixed device array of
 * 8 MiB per GPU, held until the process ends and reached through the address the library
 * takes once per device when a context is created.  The schedule is passed to a set-up
 * kernel by value, so the call also makes no host-to-device copy and never synchronises.
 * Limits (MI_ERR_UNSUPPORTED beyond them, before any launch): one image size per batch,
 * at most 64 instances, no peak-search windows, and the tables within 8 MiB (component
 * lists take 12 bytes per iteration cap when restoring without component outputs).
 * Every call on one GPU shares that GPU's array and the array keeps the previous call's
 * contents (the call clears what must start at zero): calls that overlap on one GPU, on
 * different streams or from different threads, race and must be serialised by the caller. */
mi_status mi_hogbom_clean_noalloc(mi_ctx* ctx, const mi_batch* batch, const float* dirty,
                                  const float* beam, const mi_clean_params* params,
                                  float* residual_out, double* model_out, int32_t* comp_idx,
                                  double* comp_flux, int32_t* n_comp_out, float* restored_out,
                                  double* cbeam_out, hipStream_t stream);

/* Steer CLEAN with restore (Sec. 2, Sec. 4.3; Algorithm 1's deconvolver).  Per iteration:
 *   peak = max |R| (max R with positive_only); stop if peak <= threshold;
 *   C = R on the pixels with |R| >= trim peak (R >= trim peak), 0 elsewhere (FP64 test);
 *   D[y][x] = sum_q C[q] beam[y - q_y + N][x - q_x + N]  (linear convolution by FP32 FFTs
 *     with FP64 twiddles: D is within about 1e-7 of max |D|);
 *   alpha = gain peak / max |D| (stop if D = 0);  model += alpha C;  R -= alpha D.
 * So an isolated point is subtracted exactly as a Hogbom step, and a selection covering an
 * extended source never removes more than gain x peak at any pixel.
 *   dirty: float32 N*N per instance; beam: float32 (2N)^2 per instance (peak at (N, N));
 *   N: powers of two in [64, 4096].  Pointers to float images must be 16-byte aligned.
 *   residual_out: float32 N*N; model_out: double N*N (optional);
 *   n_cycle_out (optional): int32 [n_inst], iterations done;
 *   log_out (optional): double [sum ncycle][3] = (peak, alpha, selected pixels) per
 *     iteration, instances back to back;
 *   mask_out (optional): uint32 [sum ncycle_i N_i^2 / 32], the selection of each iteration
 *     as bits (bit b of word w = pixel 32 w + b), instances back to back;
 *   restored_out (optional): R + model convolved with the clean beam (the Gaussian fitted
 *     to the beam's main lobe, as in mi_hogbom_clean, over the whole map);
 *   cbeam_out (optional): double [n_inst][6] as in mi_hogbom_clean.
 * Every image of the batch advances one iteration per launch sequence (four launches per
 * iteration, up to the largest ncycle); workspace per N x N image: about 36 N^2 bytes (44 N^2
 * without model_out).  */
mi_status mi_steer_clean(mi_ctx* ctx, const mi_batch* batch, const float* dirty, const float* beam,
                         const mi_steer_params* params, float* residual_out, double* model_out,
                         int32_t* n_cycle_out, double* log_out, uint32_t* mask_out, float* restored_out,
                         double* cbeam_out, hipStream_t stream);

/* Adjoint of the imaging operator: FFT, then degrid.
 *   image: float32 N*N per instance.  vis_out: complex, one per input visibility.
 *   adjoint = 0: prediction P(y)_k = sum_taps K_k(cell) F[y / (corr_x corr_y)](cell),
 *                F the centred unnormalised forward DFT;
 *   adjoint = 1: (A^T y)_k = (2 w_k / B0_N) P(y)_k, the transpose of mi_dirty_image
 *                under the real inner products <a,b> = sum a b and Re sum conj(v) u.
 *   Visibilities that are not kept get 0.                                            */
mi_status mi_degrid(mi_ctx* ctx, const mi_batch* batch, const float* image, const float* uv,
                    const float* w_in, int adjoint, mi_c64* vis_out, hipStream_t stream);

/* Transpose of the prediction (mi_degrid with adjoint = 0): with unit weights on the kept
 * visibilities (w_in > 0 and on the grid; the weighting mode is ignored),
 *   (P^T v)[x][y] = Re sum_k v_k S_k(x, y) / (corr(x) corr(y)) = Re I_raw / (2 corr corr),
 * i.e. the dirty image of v with unit weights scaled by B0 / 2 instead of 1 / B0.  Under the
 * real inner products <a,b> = sum a b and Re sum conj(v) u, <P y, v> = <y, P^T v>.
 *   vis: complex, one per input visibility; image_out: float32 N*N per instance.   */
mi_status mi_predict_transpose(mi_ctx* ctx, const mi_batch* batch, const mi_c64* vis, const float* uv,
                               const float* w_in, float* image_out, hipStream_t stream);

/* Sky and disk levels of maps (Sec. 4.1): the finite pixel values of each N*N map are put
 * into n_bins equal ranges between their minimum and maximum (bin = floor((x - lo) /
 * (hi - lo) * n_bins), last bin closed) and a two-component Gaussian mixture is fitted
 * to the histogram by n_iter expectation-maximisation steps (FP64; started at the
 * histogram's median and 90th percentile).  The fainter component is the sky (a), the
 * other the disk (b); Algorithm 1 cleans while the peak exceeds mu_a.
 *   images: float32 N*N per instance (e.g. dirty maps from mi_dirty_image).
 *   levels_out (device): double [n_inst][6] = mu_a, sigma_a, weight_a, mu_b, sigma_b,
 *   weight_b; a constant map gives (v, 0, 1, v, 0, 0).
 *   mu_a_out, mu_b_out (device, optional): float [n_inst], ready to pass as
 *   mi_clean_params.threshold_dev.
 *   n_bins in [2, 4096] (the paper uses 2000); n_iter in [0, 100000].                */
mi_status mi_gmm_levels(mi_ctx* ctx, const mi_batch* batch, const float* images, int32_t n_bins,
                        int32_t n_iter, double* levels_out, float* mu_a_out, float* mu_b_out,
                        hipStream_t stream);

/* Disk centering (Sec. 4.2): offset of the solar disk in each map from the field centre.
 * Each N*N map (typically cleaned down to the disk level mu_b of mi_gmm_levels, which
 * removes the active regions) is correlated circularly with a uniform disk of radius
 * radius_px[i] pixels centred on pixel (N/2, N/2) (FP64 DFTs); the largest correlation
 * value (ties: lowest linear index) is refined per axis by a parabola through it and its
 * neighbours.  radius_px: host, n_inst, > 0.  offsets_out (device): double [n_inst][2] =
 * (dl, dm) in radians (+x, +y = increasing pixel index).  The disk models' transforms
 * are kept between calls; a call with new radii uploads them and synchronises once.  */
mi_status mi_disk_offsets(mi_ctx* ctx, const mi_batch* batch, const float* images, const double* radius_px,
                          double* offsets_out, hipStream_t stream);

/* Phase correction (Sec. 4.2, Algorithm 1): vis[k] *= exp(+2 pi i (u_k dl + v_k dm)) in
 * place (FP64 phase), which moves a disk at (dl, dm) to the centre of the next image.
 * offsets (device): double [n_inst][2], e.g. from mi_disk_offsets.                    */
mi_status mi_phase_shift(mi_ctx* ctx, const mi_batch* batch, mi_c64* vis, const float* uv,
                         const double* offsets, hipStream_t stream);

/* ---- tuning (schedules picked by an autotuner; results do not depend on them) -------
 * grid_chunk: gridder tiles (16 x 64 cells) per workgroup, 1..32, 0 = 8 (the default).
 * fft_elems:  complex FP64 points each transform workgroup stages in LDS, which sets the
 *             lines (first pass) and rows (second pass) per workgroup: 0 = by size (4096,
 *             or 8192 for 8192-point lines), 4096 or 8192.  Plans are keyed by it, so a
 *             change builds (and caches) new plans.
 * mi_set_tuning applies to every later call on the context; MI_ERR_ARG for values outside
 * these ranges.  mi_get_tuning reports the values in use.                            */
typedef struct {
  int32_t grid_chunk;
  int32_t fft_elems;
} mi_tuning;
mi_status mi_set_tuning(mi_ctx* ctx, const mi_tuning* tuning);
mi_status mi_get_tuning(mi_ctx* ctx, mi_tuning* tuning);

/* ---- kernel timing (measurement hook, not part of the imaging path) ----------------
 * mi_profile_begin: from now on, every mi_hogbom_clean call records a pair of HIP events
 *   on its stream around its Hogbom kernel launch (the beam fit, symmetry check and fills
 *   before it are outside the pair).  Do not enable it while a stream is being captured
 *   into a graph.  Clears earlier records.
 * mi_profile_end: waits for the recorded events, writes up to `cap` kernel durations in
 *   milliseconds (oldest first) to the host array ms_out, the number recorded to *n_out
 *   (may exceed cap), and stops recording.  MI_ERR_ARG for a NULL ms_out with cap > 0 or a
 *   NULL n_out.                                                                      */
mi_status mi_profile_begin(mi_ctx* ctx);
mi_status mi_profile_end(mi_ctx* ctx, float* ms_out, int32_t cap, int32_t* n_out);

/* Kernel kinds for mi_profile_begin_kinds (bit mask). */
enum {
  MI_PROF_CLEAN = 1,  /* the Hogbom kernel of mi_hogbom_clean (what mi_profile_begin records)  */
  MI_PROF_GRID = 2,   /* each FP64 tiled gridder launch: the dirty half grid (mi_grid with
                         MI_LAYOUT_HALF; mi_dirty_image unfused) and the real beam half grid
                         (mi_dirty_image with beams, mi_dirty_beam, unfused)                  */
  MI_PROF_IFFT = 4,   /* each inverse transform pass: two per dirty-image batch (mi_dirty_image,
                         mi_dirty_image_w), two per beam batch; with fused gridding only the
                         second pass of each                                                  */
  MI_PROF_GRID_FFT = 8 /* each fused gridding + first transform pass (mi_dirty_image,
                         mi_dirty_beam, mi_predict_transpose when every image's transform
                         blocks hold at least two lines, i.e. N <= 2048 at the default
                         block size): one for the dirty images, one for the beams           */
};

/* mi_profile_begin_kinds: as mi_profile_begin, for every launch of the kernel kinds in the
 *   bit mask `kinds` (MI_PROF_*).  MI_ERR_ARG for an empty mask or unknown bits.
 * mi_profile_end_kinds: as mi_profile_end; also writes each record's kind (one MI_PROF_*
 *   bit) to the host array kind_out (up to `cap` entries; kind_out may be NULL).          */
mi_status mi_profile_begin_kinds(mi_ctx* ctx, uint32_t kinds);
mi_status mi_profile_end_kinds(mi_ctx* ctx, float* ms_out, int32_t* kind_out, int32_t cap, int32_t* n_out);

#ifdef __cplusplus
}
#endif
#endif /* MI_H */
