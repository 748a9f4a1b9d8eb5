/*
 * wcal.h -- C ABI of the MI355X (gfx950) Wirtinger-Jacobian gain-calibration library.
 *
 * The library solves the weighted least-squares gain calibration problem of
 * Smirnov & Tasse, "Radio interferometric gain calibration as a complex
 * optimization problem" (MNRAS 2015):
 *
 *   scalar DI   : d_pqs = g_p m_pqs conj(g_q) + n        (Sect. 2.1, 2.3, Eq. cal:DI:tf)
 *   2x2 DI      : D_pqs = G_p M_pqs G_q^H + N            (Sect. 4, Eq. cal:DI:pol)
 *   DD (Nd dirs): d_pqs = sum_d g^d_p m^d_pqs conj(g^d_q) (Sect. 2.5, Eq. cal:dd:unpol)
 *
 * with 0/1 weights given as flags (Sect. 2.4), independently for every
 * time/frequency solution interval (Sect. 2.3).  Algorithms: StefCal, the
 * diagonal approximation of J^H J (Sect. 3.1, Eq. stefcal; polarized form
 * Eq. update:DI:diag:pol), CohJones, the per-antenna Nd x Nd block
 * approximation (Sect. 3.2.2), and AllJones, the fully diagonal DD update in
 * residual form (Sect. 3.2.3, Eq. stefcal:dd:unpol).
 *
 * Conventions (all arrays are C-contiguous):
 *   complex       : wcal_c64, interleaved float32 (re, im) -- the bytes of torch.complex64.
 *   baselines     : ant1[b], ant2[b] for b < n_bl, antenna indices in [0, n_ant), ant1 != ant2.
 *                   Either orientation is accepted; a row stored as (q, p) must hold the
 *                   conjugate (2x2: Hermitian transpose) data and model.
 *   intervals     : ns[k] >= 1 samples per baseline in interval k; interval k owns rows
 *                   [row_off[k], row_off[k+1]) with row_off = n_bl * prefix_sum(ns), ordered
 *                   sample-major: row = row_off[k] + s * n_bl + b.
 *   data          : [rows][n_corr]          (n_corr = 1 scalar, 4 = 2x2 row-major xx,xy,yx,yy)
 *   model         : [rows][n_dir][n_corr]
 *   flags         : [rows] uint8, nonzero = flagged (all correlations), or NULL = none.
 *                   A flagged row is removed from every sum by selection, so NaN/Inf under a
 *                   flag has no effect; its residual is written as exactly 0.
 *   gains         : [n_int][n_dir][n_ant][n_corr]; 2x2 gains are Jones matrices row-major.
 *
 * Memory: every data pointer passed to a compute call is DEVICE memory owned by the
 * caller, which must stay valid until the stream has passed the call.  Host pointers
 * are only taken by wcal_plan_create (tables are copied into plan-owned device memory).
 * The plan owns only those tables; every scratch array a call needs (work counters,
 * per-tile partial sums, statistics, Gram records, the device-side loop's ring) lives in a
 * WORKSPACE the caller allocates -- wcal_plan_workspace gives its size -- and passes to
 * every compute call as (workspace, ws_bytes): device memory, 256-byte aligned, contents
 * irrelevant on entry (each call initialises what it uses).  A workspace smaller than the
 * plan needs is refused with WCAL_ENOMEM before anything is launched.  Calls that share a
 * workspace must not overlap on the device.  The compute calls allocate nothing.
 * Calls are asynchronous on the given stream (a hipStream_t; NULL = default stream).
 * One plan must not be used on two streams at the same time.  data/model/gains/residual
 * pointers must be 8-byte aligned (16-byte for n_corr = 4).
 *
 * Return codes: 0 = success; negative = argument or runtime error detected
 * synchronously (nothing was launched); wcal_last_error() then describes it.
 * Numerical outcomes are never errors: they are written per interval to status[k].
 */
#ifndef WCAL_H
#define WCAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } wcal_c64;

/* return codes */
#define WCAL_OK       0
#define WCAL_EINVAL  (-1)  /* NULL required pointer, non-positive size, unsupported combination */
#define WCAL_EINDEX  (-2)  /* antenna index outside [0, n_ant) or ant1 == ant2 (autocorrelation) */
#define WCAL_ESHAPE  (-3)  /* ns[k] < 1, or a size beyond the library limits */
#define WCAL_EHIP    (-4)  /* a HIP runtime call failed */
#define WCAL_ENOMEM  (-5)  /* a table allocation failed, or the workspace is too small */
#define WCAL_EIO     (-6)  /* a file could not be read or written, or is not a weight file */

/* per-interval status bits */
#define WCAL_CONVERGED    1u  /* ||g_{k+1} - g_k||_F / ||g_{k+1}||_F < tol                      */
#define WCAL_MAXITER      2u  /* max_iter updates applied without meeting tol                     */
#define WCAL_SINGULAR_ANT 4u  /* some antenna's block was not invertible: its gain was kept       */
#define WCAL_NONFINITE    8u  /* a sum over unflagged rows was not finite: the interval stopped   */
                              /* before that update and kept the previous gains                   */
#define WCAL_ABORTED     16u  /* reserved for a device-side iteration loop that gives up a bounded */
                              /* wait; that loop is switched off (plan creation refuses it), so   */
                              /* no solve sets this bit                                            */

/* algorithms */
#define WCAL_STEFCAL   0   /* n_dir == 1; n_corr 1 or 4                     (Sect. 3.1, 4.3)   */
#define WCAL_COHJONES  1   /* per-antenna Nd x Nd blocks (Sect. 3.2.2); n_corr 4: 2Nd x 2Nd     */
                           /* blocks of the polarized case (Sect. 4.4), Nd <= 10, FP32 only     */
#define WCAL_ALLJONES  2   /* fully diagonal, residual form (Sect. 3.2.3; n_corr 4: per-direction*/
                           /* 2x2 blocks, Eq. update:DD:diag:pol), same limits as CohJones      */

/* update schedules: update k = 0, 1, ... from the starting gains either applies the
 * GN value (Eq. stefcal / its block forms) or the lambda = 1 LM average
 * g_{k+1} = (g_k + GN) / 2 (Eq. stefcal-lambda-average). */
#define WCAL_AVG_FIRST 0   /* average on even k, GN on odd k (default) */
#define WCAL_GN_FIRST  1   /* GN on even k, average on odd k           */
#define WCAL_GN_ONLY   2   /* GN on every update                        */

/* solve modes (both give the same updates; Sect. 2.3 sums run over every sample):
 * PASS  -- every update streams all samples of the interval (per-sample J^H J / J^H D pass);
 * STATS -- the gain-independent per-baseline sums over samples are formed in one pass and
 *          every update contracts them with the current gains (cost independent of the
 *          number of samples per interval).  A StefCal plan whose intervals all hold one
 *          sample runs the PASS solve in this mode: one sample's statistics are no smaller
 *          than the sample. */
#define WCAL_MODE_PASS  0
#define WCAL_MODE_STATS 1

/* Precision of the CohJones / AllJones Gram pass (the per-sample products): FP32 MFMA
 * (default), or BF16 MFMA with FP32 accumulation (inputs rounded to BF16; the per-antenna
 * solve stays FP64).  The BF16 Gram also forms the residual in FP32 and the update takes
 * the residual form g + H^-1 J^H r (Eq. ghat:approx), so the fixed point does not carry the
 * rounding of H; it needs PASS mode and Nd <= 13.  StefCal accepts only WCAL_PREC_FP32. */
#define WCAL_PREC_FP32       0
#define WCAL_PREC_BF16_GRAM  1

/* singular-block threshold: a 2x2 block with det Z <= EPS * Z00 * Z11 or an Nd x Nd
 * Cholesky pivot <= EPS * H_jj is treated as not invertible. */
#define WCAL_EPS_PIVOT 1e-5

typedef struct {
    int32_t n_ant;     /* antennas                                   */
    int32_t n_bl;      /* baselines (rows per sample)                */
    int32_t n_dir;     /* directions (1 for StefCal)                 */
    int32_t n_corr;    /* 1 = scalar, 4 = 2x2 Jones                  */
    int32_t n_int;     /* solution intervals                         */
    int32_t algo;      /* WCAL_STEFCAL | WCAL_COHJONES | WCAL_ALLJONES */
    int32_t schedule;  /* WCAL_AVG_FIRST | WCAL_GN_FIRST | WCAL_GN_ONLY */
    int32_t max_iter;  /* maximum number of updates (>= 1)           */
    double  tol;       /* relative parameter-change tolerance (>= 0) */
    int32_t mode;      /* WCAL_MODE_PASS | WCAL_MODE_STATS                 */
    int32_t precision; /* WCAL_PREC_FP32 (0) | WCAL_PREC_BF16_GRAM          */
} wcal_problem;

typedef struct wcal_plan wcal_plan;

/* Message for the last non-zero return on the calling thread ("" if none). */
const char* wcal_last_error(void);

/* Library version string. */
const char* wcal_version(void);

/* Validate a problem and build a plan on HIP device `device`.
 * ant1_h, ant2_h [n_bl] and ns_h [n_int] are HOST arrays, copied into plan-owned device
 * tables.  Fails with WCAL_EINDEX for an antenna outside [0, n_ant) or ant1 == ant2
 * (autocorrelations are excluded from the problem, Sect. 2.1 footnote), WCAL_ESHAPE for
 * ns[k] < 1 or sizes beyond the limits, WCAL_EINVAL for an unsupported combination. */
int wcal_plan_create(const wcal_problem* prob, const int32_t* ant1_h, const int32_t* ant2_h,
                     const int64_t* ns_h, int device, wcal_plan** out);

/* Release a plan and its device tables (NULL is a no-op).  The caller must make sure
 * no call using the plan is still in flight. */
void wcal_plan_destroy(wcal_plan* plan);

/* Bytes of device workspace every compute call on this plan needs (see Memory above).  The
 * size changes only with the plan's tiling (wcal_plan_autotune) and smoothing setting
 * (wcal_plan_smoothing): query it again after either. */
int wcal_plan_workspace(const wcal_plan* plan, size_t* bytes);

/* Total rows (sum over intervals of n_bl * ns[k]) described by the plan. */
int64_t wcal_plan_rows(const wcal_plan* plan);

/* Name of the kernel that streams the visibilities in this plan's solve: the per-update
 * pass (PASS mode) or the one-off statistics pass (STATS mode).  Scalar StefCal whose
 * baselines are every pair p < q in p-major order (the canonical table) runs the triangle
 * pass by default from 64 antennas (environment WCAL_TRI=0 disables it, 1 forces it for any
 * canonical table).  Static string owned by the library; "" for NULL. */
const char* wcal_plan_pass_kernel(const wcal_plan* plan);

/* Autotuner: pick the plan's tiling from measurements on the caller's data.  For StefCal
 * it times, with HIP events on `stream`, n_updates updates (tol 0; or, with n_updates = 0,
 * the plan's own solve to its tolerance; no residual either way) from `gains` for each
 * target of {8192, 16384, 32768, 65536, 131072, 262144} rows per tile and, where
 * the baseline table is canonical (scalar, PASS mode), with and without the triangle pass;
 * it keeps the fastest (best of two timed runs after a warm-up run).  `gains` is only read
 * (a copy in the workspace is iterated).  Its workspace holds that copy and the solves'
 * workspace; wcal_plan_autotune_workspace gives the size that admits every candidate
 * (candidates that do not fit a smaller one are skipped).  CohJones / AllJones stream their
 * rows in the blocked Gram pass, which has no tiling to choose; the call returns at once.
 * Outputs: the chosen rows per tile and 1 if the triangle pass is used (either pointer may
 * be NULL).  The call synchronises the host and rebuilds the plan's tile tables: call it
 * between solves, not under graph capture, and query wcal_plan_workspace afterwards.
 * Errors: WCAL_EINVAL (n_updates outside [0, max_iter], profiling on, no workspace),
 * WCAL_ENOMEM (no candidate fits the workspace), WCAL_EHIP. */
int wcal_plan_autotune_workspace(const wcal_plan* plan, size_t* bytes);
int wcal_plan_autotune(wcal_plan* plan, const wcal_c64* data, const wcal_c64* model,
                       const uint8_t* flags, const wcal_c64* gains, int32_t n_updates,
                       void* workspace, size_t ws_bytes, void* stream, int32_t* tile_rows_out,
                       int32_t* tri_out);

/* Solve every interval: iterate the algorithm's update from the gains held in `gains`
 * until the relative parameter change drops below tol or max_iter updates were applied,
 * then predict the residual R = D - sum_d G_p M G_q^H with the final gains.
 *   gains    in/out [n_int][n_dir][n_ant][n_corr]
 *   residual out    [rows][n_corr], or NULL (flagged rows are written as 0)
 *   n_iter   out    [n_int] updates applied
 *   status   out    [n_int] WCAL_* status bits
 *   chi2     out    [n_int] sum of |R|^2 over unflagged rows (FP64), or NULL
 * The whole batch runs on the device with no host synchronisation.  In PASS mode each
 * update is a pass over the rows of the intervals still iterating (StefCal: the tiles on the
 * device-built active list; CohJones / AllJones: the Gram pass) followed by the update
 * kernels; the launches of all max_iter updates are issued up front and an update with no
 * interval left iterating returns at once (with the plan's host watch on, wcal_plan_watch,
 * the call stops issuing them once every interval has stopped).  In STATS mode one
 * statistics pass is followed by updates on the statistics (StefCal: one launch that
 * iterates every interval; CohJones / AllJones: per-update launches).  Every solve ends with
 * a tiled residual pass.  No call allocates or records a memset node, and none synchronises
 * the host unless the host watch is on, so the call can be captured into a HIP graph. */
int wcal_solve(wcal_plan* plan, const wcal_c64* data, const wcal_c64* model,
               const uint8_t* flags, wcal_c64* gains, wcal_c64* residual,
               int32_t* n_iter, uint32_t* status, double* chi2, void* workspace, size_t ws_bytes,
               void* stream);

/* A wcal_solve captured into an instantiated HIP graph (stream capture of exactly the
 * launches wcal_solve makes; on a NULL stream the capture uses a private stream).  Each
 * wcal_graph_launch re-runs the solve on `stream` with the same pointers, reading the
 * current contents of data, model, flags and gains (gains are updated in place, so reset
 * them for a fresh start).  The plan and the workspace must outlive the graph; launches of
 * graphs or calls that share a workspace must not overlap.  Profiling must be off while
 * capturing.  Errors: WCAL_EINVAL (NULL, profiling on), WCAL_ENOMEM (workspace too small),
 * WCAL_EHIP (capture or instantiation failed). */
typedef struct wcal_graph wcal_graph;
int wcal_solve_graph(wcal_plan* plan, const wcal_c64* data, const wcal_c64* model,
                     const uint8_t* flags, wcal_c64* gains, wcal_c64* residual,
                     int32_t* n_iter, uint32_t* status, double* chi2, void* workspace,
                     size_t ws_bytes, void* stream, wcal_graph** out);
int wcal_graph_launch(wcal_graph* graph, void* stream);
void wcal_graph_destroy(wcal_graph* graph);   /* NULL is a no-op */

/* Host watch of the per-update launches.  A per-update solve (StefCal in PASS mode,
 * CohJones / AllJones in either mode, the smoothed and the predicted-model solves) enqueues
 * one group of launches per update slot, max_iter of them, and the intervals stop at
 * different updates, each at its own convergence test: a slot after the last one has
 * stopped finds nothing to do.  With a watch of depth > 0, wcal_solve, wcal_solve_static,
 * wcal_solve_smooth and wcal_solve_points copy, after every slot, the device count of the
 * work listed for the next update into pinned host memory on a side stream, keep at most
 * `depth` slots enqueued past the last count read, and stop enqueuing once a count reads 0;
 * the residual pass follows as usual.  The results are those of the unwatched call (the
 * omitted slots would do nothing).  The call blocks the calling thread until the solve is
 * within `depth` slots of its last update, so the stream must not wait on work that the
 * caller submits after the call.  Under stream capture (wcal_solve_graph) every slot is
 * recorded, as without the watch.  The watch's events and pinned words belong to the plan:
 * watched calls on one plan must not run concurrently from several host threads.  depth 0
 * (the default) turns the watch off; until then, or
 * wcal_plan_destroy, the plan holds a side stream, 2 depth events and depth pinned host
 * words.  Errors: WCAL_EINVAL (NULL plan, depth outside [0, WCAL_WATCH_MAX]), WCAL_EHIP. */
#define WCAL_WATCH_MAX 64
int wcal_plan_watch(wcal_plan* plan, int32_t depth);

/* wcal_solve for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same solve, arguments as in
 * wcal_solve, with its workspace in a static device array of WCAL_STATIC_WORKSPACE_BYTES
 * that the library holds on every GPU it runs on until the process ends.  The call
 * allocates nothing (the array's device address is looked up once per device, on the first
 * call there).  Every call on one GPU shares that array: calls that overlap on the device
 * (two streams, two threads, two graphs) race; consecutive calls do not (each initialises
 * what it reads).  Errors: as wcal_solve, and WCAL_ENOMEM before any launch when the plan's
 * workspace (wcal_plan_workspace) exceeds the static array, WCAL_EINVAL while profiling is
 * on (its events are created on demand). */
#define WCAL_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int wcal_solve_static(wcal_plan* plan, const wcal_c64* data, const wcal_c64* model,
                      const uint8_t* flags, wcal_c64* gains, wcal_c64* residual,
                      int32_t* n_iter, uint32_t* status, double* chi2, void* stream);

/* One fused pass at fixed gains, no iteration: per interval and antenna the blocks of
 * the approximate J^H J that the algorithm inverts, the top half of J^H D and of J^H r,
 * the number of unflagged stored rows touching the antenna, chi^2 and optionally R.
 *   jhj  [n_int][n_ant][blk]  scalar: blk = 1 (A_p, imaginary part 0; Eq. JHJ:DI:tfw);
 *                             2x2: blk = 4, Z_p = sum Y Y^H (Eq. JHJ:pol diagonal);
 *                             DD:  blk = n_dir * n_dir, H_p[c][d] = sum conj(y^c) y^d
 *                             (Eq. JHJ:DD:unpol diagonal blocks);
 *                             2x2 DD: blk = (2 n_dir)^2, H_p = sum Ys Ys^H with Ys the 2Nd x 2
 *                             stack of Y^d = M^d G^{dH}_q (row 2d + k = row k of Y^d); the
 *                             operator block of Eq. JHJ:DD:pol is I_2 (x) H_p
 *   jhd  [n_int][n_ant][n_dir * n_corr]  J^H D (scalar/DD: sum conj(y) d; 2x2: sum D Y^H;
 *                                        2x2 DD: sum D Y^{dH} per direction, row-major)
 *   jhr  [n_int][n_ant][n_dir * n_corr]  J^H r (same with r in place of d)
 *   count [n_int][n_ant] int32, chi2 [n_int] (FP64), residual [rows][n_corr] or NULL. */
int wcal_accumulate(wcal_plan* plan, const wcal_c64* data, const wcal_c64* model,
                    const uint8_t* flags, const wcal_c64* gains, wcal_c64* jhj, wcal_c64* jhd,
                    wcal_c64* jhr, int32_t* count, double* chi2, wcal_c64* residual,
                    void* workspace, size_t ws_bytes, void* stream);

/* Residual prediction only: R = D - sum_d G_p M G_q^H, flagged rows 0 (Eq. cal:DI,
 * Eq. cal:DI:pol, Eq. cal:dd:unpol); chi2 [n_int] or NULL. */
int wcal_residual(wcal_plan* plan, const wcal_c64* data, const wcal_c64* model,
                  const uint8_t* flags, const wcal_c64* gains, wcal_c64* residual,
                  double* chi2, void* workspace, size_t ws_bytes, void* stream);

/* Point-source models predicted in the Gram and residual passes instead of read from HBM
 * (Sect. 3.2.1: m^d_pq(t, nu) = S_d exp(-2 pi i (u_pq(t) . sigma_d) nu / c), sigma_d =
 * [l_d, m_d, n_d - 1]), for scalar CohJones / AllJones with the FP32 Gram.  The pass then
 * reads 9 bytes per row (data and flag) instead of 8 Nd + 9.  Every interval holds
 * n_time * n_chan samples, sample s = t * n_chan + f, channel f at freq0 + f * dfreq.  The
 * phase is formed in FP64 and reduced by quarter turns; sine and cosine of the remainder are
 * FP32 Taylor series.  That happens at every new time slot and at least every 16 channels
 * (the Gram pass: every 16 steps of 4 channels); in between, the phasor is stepped across
 * channels by one complex multiply (relative model error ~1e-7).  All arrays are device
 * memory. */
typedef struct {
    int32_t n_time;      /* timeslots per interval                                      */
    int32_t n_chan;      /* channels per interval                                       */
    double freq0;        /* Hz, channel 0                                               */
    double dfreq;        /* Hz, channel spacing                                         */
    const double* uvw;   /* [n_int][n_time][n_bl][3] metres, baseline vector ant2 - ant1 */
    const double* lmn;   /* [n_dir][3]: l, m, n - 1                                      */
    const float* flux;   /* [n_dir] Jy                                                   */
} wcal_points;

/* wcal_solve with the model given by `pts` (data, flags, gains, residual, n_iter, status, chi2
 * as in wcal_solve; PASS or STATS mode).  The solve forms a phasor table once (per interval,
 * time slot, baseline and direction: the phasors where the passes start or re-base their
 * channel walk, and the step over four channels) and every pass reads it, so its workspace is
 * the plan's plus the table: wcal_points_workspace gives the size for this grid
 * (n_int * n_time * n_bl * n_dir * (4 * ceil(n_chan / 64) + 1) * 8 bytes, 387 MB for 16
 * intervals of 30 x 64 samples, 2016 baselines and 10 directions).  Errors: WCAL_EINVAL (plan
 * not scalar CohJones / AllJones with the FP32 Gram, NULL or misaligned arrays, n_time or
 * n_chan < 1), WCAL_ESHAPE (an interval that does not hold n_time * n_chan samples),
 * WCAL_ENOMEM (workspace smaller than wcal_points_workspace). */
int wcal_points_workspace(const wcal_plan* plan, const wcal_points* pts, size_t* bytes);
int wcal_solve_points(wcal_plan* plan, const wcal_points* pts, const wcal_c64* data, const uint8_t* flags,
                      wcal_c64* gains, wcal_c64* residual, int32_t* n_iter, uint32_t* status, double* chi2,
                      void* workspace, size_t ws_bytes, void* stream);

/* Time/frequency smoothing of scalar StefCal (Sect. 3.4, Eq. JHJ:diag:smooth).  Every
 * sample of an interval becomes a cell (t, nu) of an n_time x n_chan grid, sample
 * s = t * n_chan + nu, with gains of its own; every update takes
 *     g_p(t, nu) = (w o alpha_p)(t, nu) / (w o beta_p)(t, nu),
 * alpha_p = sum_q conj(y) d and beta_p = sum_q |y|^2 per cell (y formed with the gains of the
 * row's own cell), w(t, nu) = exp(-t^2 / 2 sigma_t^2 - nu^2 / 2 sigma_f^2) truncated at
 * |t| <= ceil(3 sigma_t), |nu| <= ceil(3 sigma_f) (sigma 0: no smoothing along that axis),
 * cells beyond the grid edge absent from both sums; then the plan's schedule.  Convergence
 * per interval: relative change over its cells and antennas after removing, per cell, the
 * best phase between successive iterates (each cell's solution is defined up to its own
 * phase, and the smoothed iterates keep turning along these phases).  A cell whose smoothed
 * beta is not positive keeps its gain (SINGULAR_ANT).
 *
 * wcal_plan_smoothing prepares a scalar StefCal plan in PASS mode whose intervals all hold
 * n_time * n_chan samples: it validates and builds the per-cell tables (synchronous;
 * calling it again replaces the previous setting); the plan's workspace then also holds the
 * smoothing scratch, so query wcal_plan_workspace again.  Errors:
 * WCAL_EINVAL (wrong plan kind, n_time or n_chan < 1, negative or non-finite sigma),
 * WCAL_ESHAPE (an interval of another size, kernel radius above 4096 cells), WCAL_ENOMEM.
 *
 * wcal_solve_smooth then solves every interval with smoothing.  gains in/out
 * [n_int][n_time * n_chan][n_ant] (per cell), residual [rows] or NULL, n_iter, status and
 * chi2 [n_int] per interval (chi2 may be NULL).  No allocation, no host synchronisation. */
int wcal_plan_smoothing(wcal_plan* plan, int32_t n_time, int32_t n_chan, double sigma_t, double sigma_f);
int wcal_solve_smooth(wcal_plan* plan, const wcal_c64* data, const wcal_c64* model, const uint8_t* flags,
                      wcal_c64* gains, wcal_c64* residual, int32_t* n_iter, uint32_t* status, double* chi2,
                      void* workspace, size_t ws_bytes, void* stream);

/* Kernel timing for benchmarks.  While enabled, every kernel launched by wcal_solve and
 * wcal_residual on this plan is bracketed by HIP events on the call's stream.
 * wcal_profile_read waits for those events and returns, per kernel class, the summed
 * duration in milliseconds and the number of launches since the previous read (or since
 * enabling), then clears the record.  ms and launches have WCAL_K_COUNT entries. */
#define WCAL_K_PASS        0   /* per-sample J^H J / J^H D pass (PASS mode)            */
#define WCAL_K_UPDATE      1   /* per-interval solve, schedule and convergence test    */
#define WCAL_K_STATS       2   /* per-baseline statistics pass (STATS mode, DD)         */
#define WCAL_K_SOLVE_STATS 3   /* iterations on the statistics                          */
#define WCAL_K_RESID       4   /* residual and chi^2 pass                               */
#define WCAL_K_OTHER       5   /* initialisation and small reductions                  */
#define WCAL_K_COUNT       6
int wcal_profile_enable(wcal_plan* plan, int enable);
int wcal_profile_read(wcal_plan* plan, double* ms, int32_t* launches);

/* ------------------------------------------------------------------------------------
 * Learned warm start.  Not part of the paper's method: a starting point for the solve,
 * which alone decides the result (its convergence test decides, and intervals that do not
 * converge from the warm start are solved again from unit gains).
 * ---------------------------------------------------------------------------------- */

/* Knots.  Consecutive intervals (one channel each) are grouped in bins of bin_width
 * (the last bin may be shorter); bin B = [lo, hi) has the knot interval lo + (hi - lo - 1) / 2.
 * wcal_bin_knots writes the n_bins = ceil(n_int / bin_width) knot indices to a host array. */
int wcal_bin_knots(int32_t n_int, int32_t bin_width, int32_t* knots);

/* Coarse pass input: copies the rows of every knot interval of the plan (bins in order, rows
 * of each knot in order) into compact device arrays, to be solved by a second plan whose
 * interval sizes are those of the knots.  data_out [rows_k][n_corr], model_out
 * [rows_k][n_dir][n_corr], flags_out [rows_k] (zeros when flags is NULL; not written when
 * flags_out is NULL), rows_k = sum of the knots' rows.  The caller owns every buffer. */
int wcal_gather_knots(const wcal_plan* plan, int32_t bin_width, const wcal_c64* data,
                      const wcal_c64* model, const uint8_t* flags, wcal_c64* data_out,
                      wcal_c64* model_out, uint8_t* flags_out, void* stream);

/* Knot values y [n_ant][2 * n_bins] (real parts, then imaginary parts; device) to gains
 * [n_int][1][n_ant][1] (device): amplitude and phase linear in the interval index between
 * neighbouring knots, the phase step between two knots being the principal argument of
 * z_{B+1} conj(z_B) (so steps must stay below pi); constant beyond the outer knots. */
int wcal_bins_to_gains(int32_t n_int, int32_t n_ant, int32_t bin_width, const float* y,
                       wcal_c64* gains, void* stream);

/* Gains [n_int][1][n_ant][1] referenced to antenna 0 per interval (times conj(g_0)/|g_0|,
 * the phase gauge) and averaged over the intervals within halfwidth of each knot (clipped to
 * [0, n_int)) -> y [n_ant][2 * n_bins].  With bin_width 1 and halfwidth 0 this is the
 * referenced gains of every interval (the coarse-pass features); with the full solve's
 * gains it gives the training targets. */
int wcal_gains_to_bins(int32_t n_int, int32_t n_ant, int32_t bin_width, int32_t halfwidth,
                       const wcal_c64* gains, float* y, void* stream);

/* Fallback: reset the gains of every interval whose status lacks WCAL_CONVERGED to unit
 * gains (identity Jones matrices), ready for another wcal_solve. */
int wcal_reset_unconverged(wcal_plan* plan, const uint32_t* status, wcal_c64* gains, void* stream);

/* Warm-start network: y = tanh(tanh(x W1 + b1) W2 + b2) W3 + b3 (+ x when skip is nonzero,
 * which needs d_in == d_out) row-wise (FP32), trained on
 * the mean squared error with Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
 * Parameters are one flat device array: W1 [d_in][d_hidden], b1, W2 [d_hidden][d_hidden],
 * b2, W3 [d_hidden][d_out], b3, row-major; the caller supplies initial values.  x, y and
 * targets are device arrays [batch][d]. */
typedef struct wcal_mlp wcal_mlp;
int wcal_mlp_create(int32_t d_in, int32_t d_hidden, int32_t d_out, int32_t max_batch, int32_t skip,
                    int device, wcal_mlp** out);
void wcal_mlp_destroy(wcal_mlp* mlp);
int64_t wcal_mlp_num_params(const wcal_mlp* mlp);
int wcal_mlp_set_params(wcal_mlp* mlp, const float* params, void* stream);  /* resets Adam */
int wcal_mlp_get_params(const wcal_mlp* mlp, float* params, void* stream);
int wcal_mlp_forward(wcal_mlp* mlp, const float* x, int32_t batch, float* y, void* stream);
/* forward + backward without an update: gradient [num_params] and loss (FP64), either NULL */
int wcal_mlp_gradients(wcal_mlp* mlp, const float* x, const float* target, int32_t batch,
                       float* grads, double* loss, void* stream);
/* one Adam step on the batch; loss (FP64, device) of the batch before the step, or NULL */
int wcal_mlp_train_step(wcal_mlp* mlp, const float* x, const float* target, int32_t batch,
                        float lr, double* loss, void* stream);

/* Weight files (host calls, synchronous: call them once the work that produced or will read
 * the parameters has completed).  The file is one line of JSON, e.g.
 *   {"format": "wcal-mlp", "version": 1, "d_in": 128, "d_hidden": 256, "d_out": 128, "skip": 1,
 *    "n_params": 131712, "adam_step": 4000, "dtype": "float32", "byteorder": "little",
 *    "sections": ["params", "adam_m", "adam_v"]}
 * then n_params float32 values per section in that order: the flat parameters in the layout
 * of wcal_mlp_set_params, then the two Adam moments, so training resumes where it stopped.
 * wcal_mlp_load checks the header against the network it loads into.  Errors: WCAL_EIO (open,
 * read or write failed, not a weight file, truncated), WCAL_EINVAL (NULL, or a network of
 * another shape), WCAL_EHIP. */
int wcal_mlp_save(const wcal_mlp* mlp, const char* path);
int wcal_mlp_load(wcal_mlp* mlp, const char* path);

#ifdef __cplusplus
}
#endif

#endif /* WCAL_H */
