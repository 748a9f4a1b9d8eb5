// Internal declarations shared by the host API and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "wcal.h"

// A tile of one interval's rows: baselines [b0, b1) x samples [s0, s1) of interval k.
struct Tile {
    int32_t k, b0, b1, s0, s1;
};

// Optional per-kernel-class timing with HIP events (benchmarks).
struct Profiler;
void prof_begin(const wcal_plan* plan, int cls, hipStream_t s);
void prof_end(const wcal_plan* plan, int cls, hipStream_t s);

// Host watch of the per-update launches (wcal_plan_watch).  After every update slot a side
// stream copies the device count of work items listed for the next update into pinned host
// memory; the host keeps at most `depth` slots enqueued past the last count it has read and
// stops enqueuing once a count reads 0: every interval has stopped, and the slots left would
// find nothing listed.  Not under stream capture, where every slot is recorded.
struct SlotWatch {
    int depth = 0;
    hipStream_t side = nullptr;
    std::vector<hipEvent_t> slot_ev, copy_ev;   // [depth] each, reused round robin
    int32_t* host = nullptr;                    // pinned [depth]
    bool live = false;                          // the current call is watched
};
// Call after enqueuing update slot `it` of a per-update solve on stream s, with d_count the
// device counter of the work items listed for update it + 1.  True: no slot after `it`
// has work, so the caller stops enqueuing slots.
bool watch_stop(const wcal_plan* plan, hipStream_t s, const int32_t* d_count, int it);

// A unit of the triangle pass (baselines in the canonical order: all pairs p < q,
// p-major, q increasing): the whole rows p in [p0, p1) of the triangle, at most 64; or, when
// the plan packs rows (possible from TRI_PAIR_MIN antennas on), packed rows r in [p0, p1),
// each row n_ant - 2 - r and row r.
constexpr int TRI_PAIR_MIN = 127;
struct TriUnit {
    int32_t p0, p1, entries, chunks;   // chunks: sum over rows of ceil(length / 64)
};

// ------------------------------------------------------------------ workspace
// Per-call device scratch is carved out of the caller's workspace (wcal_plan_workspace): one
// region per kind of scratch, each starting on a WS_ALIGN boundary.  The plan keeps only the
// tables it builds on the host (baselines, interval offsets, tiles, units, antenna lists).
constexpr size_t WS_ALIGN = 256;
enum WsRegion {
    WS_CTR,       // int32 work counters of the per-update launches
    WS_ACTIVE,    // int32 [n_int] intervals still iterating
    WS_QUEUE,     // int32 [4] queue counters (accumulate pass)
    WS_LISTS,     // int32 [2][tiles] active-tile lists of the per-update launches
    WS_PARTIAL,   // float [tiles][n_ant][nvp] per-tile per-antenna sums
    WS_CHI_PART,  // double [tiles] chi^2 per residual tile
    WS_STATS,     // statistics (STATS mode) or the direction-dependent solve state
    WS_LOOP,      // the device-side iteration loop: control words, tile ring, per-interval counters
    WS_COUNT
};
struct WsLayout {
    size_t off[WS_COUNT + 1] = {};   // off[WS_COUNT]: bytes of the plan's own regions
};
inline size_t ws_round(size_t n) { return (n + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; }

// The device-side iteration loop of the StefCal PASS solve (one persistent launch, the ring
// of loop_ring.h): 64 bytes of control words, LOOP_RING ring slots per tile, one tile
// counter per interval.
constexpr int LOOP_RING = 2;
inline size_t loop_bytes(int64_t ntiles, int64_t n_int) {
    return 64 + ws_round(sizeof(uint64_t) * LOOP_RING * (size_t)ntiles) + sizeof(int32_t) * (size_t)n_int;
}

// ------------------------------------------------------------------ plan
struct wcal_plan {
    wcal_problem prob;
    int device = 0;
    int n_cu = 0;
    int64_t rows = 0;
    int32_t max_ns = 0;
    std::vector<int32_t> h_ns;    // samples per interval (host copy, for re-tiling)
    // device tables (plan-owned)
    int32_t* d_ant1 = nullptr;    // [n_bl]
    int32_t* d_ant2 = nullptr;    // [n_bl]
    int64_t* d_row_off = nullptr; // [n_int + 1]
    int32_t* d_ns = nullptr;      // [n_int]
    int32_t* d_order = nullptr;   // [n_int] intervals by decreasing size (LPT order)
    int32_t* d_queue = nullptr;   // [4] work-queue counters
    // tiles of the per-sample passes (interval k owns tiles [tile_off[k], tile_off[k+1]))
    Tile* d_tiles = nullptr;
    int32_t* d_tile_off = nullptr;
    int32_t ntiles = 0;
    // statistics tiles (every sample of a baseline chunk) for WCAL_MODE_STATS
    Tile* d_stiles = nullptr;
    int32_t nstiles = 0;
    // per-iteration state of the tiled solve
    int32_t* d_lists = nullptr;   // [2][ntiles] active tile lists
    int32_t* d_ctr = nullptr;     // [2][max_iter + 2] pop counters and list lengths
    float* d_partial = nullptr;   // [ntiles][n_ant][nvp] per-tile per-antenna sums
    int32_t* d_active = nullptr;  // [n_int], then (StefCal) [n_int] arrival counters of the triangle pass
    double* d_chi_part = nullptr; // [ntiles]
    float* d_stats = nullptr;     // per-baseline statistics (STATS mode) or DD Gram records
    size_t stats_bytes = 0;
    int32_t* d_ant_ptr = nullptr; // [n_ant + 1] CSR: rows of each antenna (DD)
    int32_t* d_ant_bl = nullptr;  // [2 n_bl]    2 * baseline + side (0: ant1, 1: ant2)
    size_t max_smem = 65536;      // dynamic LDS limit per workgroup
    // launch configuration
    int block = 0;                // threads per workgroup (0 = largest compiled for the kernel)
    int wg_per_cu = 0;            // resident workgroups per CU (0 = occupancy limit)
    int tile_rows = 0;            // target rows per tile
    // triangle pass (scalar StefCal, canonical baseline order): units and tiles whose
    // b0/b1 are unit ranges; the PASS solve uses these tiles for its pass and update
    bool canonical = false;       // baselines are every pair p < q in p-major order
    bool tri = false;
    bool tri_paired = false;      // units are packed row pairs
    bool tri_unfused = false;     // its triangle tiles only feed the unfused pass (cell plans)
    TriUnit* d_units = nullptr;
    int32_t nunits = 0;
    Tile* d_ttiles = nullptr;
    int32_t* d_ttile_off = nullptr;
    int32_t nttiles = 0;
    Profiler* prof = nullptr;     // non-null while timing is enabled
    SlotWatch* watch = nullptr;   // non-null while the host watches the per-update launches
    // time/frequency smoothing (scalar StefCal): the cell plan and its scratch, or null
    struct SmoothPlan* smooth = nullptr;
    // workspace: the plan's own regions, then (with smoothing) the smoothing scratch and the
    // cell plan's workspace
    WsLayout ws;
    size_t ws_bytes = 0;          // total the caller must provide
    bool loop = false;            // StefCal PASS solve as one persistent launch: switched off (its first GPU
                                  // runs did not finish, cause not found)
    int64_t wait_ticks = 1000000000;  // bound of the loop's waits (10 s; WCAL_WAIT_MS)
    int32_t* d_loop = nullptr;    // WS_LOOP region while bound
};

// record the message returned by wcal_last_error() and return `code`
int wcal_error(int code, const std::string& msg);

// Workspace of a plan: lay out its regions (after tiling or smoothing changes) and point its
// scratch fields into a caller's buffer.
void ws_layout(wcal_plan* plan);
void ws_bind(wcal_plan* plan, char* ws);
size_t smooth_ws_bytes(const struct SmoothPlan* sp);
void smooth_ws_bind(struct SmoothPlan* sp, char* ws);
// checks a caller's workspace against the plan (WCAL_EINVAL / WCAL_ENOMEM), binds it
int ws_check_bind(wcal_plan* plan, void* ws, size_t ws_bytes);

// ------------------------------------------------------------------ kernel arguments
struct DiArgs {
    const float2* data;      // [rows][nc]
    const float2* model;     // [rows][nc]
    const uint8_t* flags;    // [rows] or null
    float2* gains;           // [n_int][n_ant][nc]   (n_dir == 1)
    const float2* gains_in;  // accumulate/residual: gains read only
    float2* residual;        // [rows][nc] or null
    int32_t* n_iter;         // [n_int]
    uint32_t* status;        // [n_int]
    double* chi2;            // [n_int] or null
    // accumulate outputs
    float2* jhj;             // [n_int][n_ant][blk]
    float2* jhd;             // [n_int][n_ant][nc]
    float2* jhr;             // [n_int][n_ant][nc]
    int32_t* count;          // [n_int][n_ant]
    // tables
    const int32_t* ant1;
    const int32_t* ant2;
    const int64_t* row_off;
    const int32_t* ns;
    const int32_t* order;
    int32_t* queue;
    // tiled solve
    const Tile* tiles;
    const int32_t* tile_off;
    int32_t ntiles;
    int32_t* lists;
    int32_t* ctr;
    float* partial;
    int32_t* active;
    double* chi_part;
    float* stats;
    int32_t n_ant, n_bl, n_int, max_iter, schedule;
    int32_t tri_paired;      // triangle units are packed row pairs (see TriUnit)
    int32_t* tri_cnt;        // [n_int] fused triangle pass: workgroups of a shared interval done
    double tol;
};

// Point-source models predicted on the device instead of read from model[] (Sect. 3.2.1):
// sample s = t * n_chan + f of every interval, channel frequency freq0 + f * dfreq.
struct PointArgs {
    const double* uvw = nullptr;   // [n_int][n_time][n_bl][3] metres (ant2 - ant1)
    const double* lmn = nullptr;   // [nd][3]: l, m, n - 1
    const float* flux = nullptr;   // [nd]
    double freq0 = 0.0, dfreq = 0.0;
    int32_t n_time = 0, n_chan = 0;
    // phasor table of the solve, in the workspace (formed once per solve, read by every pass):
    // zt [n_int][n_time][n_bl][nseg][4][nd]: S_d exp(-2 pi i phi nu) at channels 64 j + r,
    // r < 4 (the channels where a lane's phasor walk starts or is re-based), and
    // st [n_int][n_time][n_bl][nd]: exp(-2 pi i phi 4 dfreq), the step over four channels
    float2* zt = nullptr;
    float2* st = nullptr;
    int32_t nseg = 0;              // ceil(n_chan / 64)
};

// Bytes of the phasor table for an n_time x n_chan grid (a multiple of WS_ALIGN).
size_t points_table_bytes(const wcal_problem& p, int32_t n_time, int32_t n_chan);

// Rebuild a plan's tiles with its current tiling (wcal_api.hip).
int plan_retile(wcal_plan* plan);

struct DdArgs {
    const float2* data;      // [rows]
    const float2* model;     // [rows][nd], or null with pt.uvw set
    PointArgs pt;
    const uint8_t* flags;
    float2* gains;           // [n_int][nd][n_ant][n_corr]
    const float2* gains_in;
    float2* residual;
    int32_t* n_iter;
    uint32_t* status;
    double* chi2;
    float2* jhj;             // [n_int][n_ant][nd][nd]
    float2* jhd;             // [n_int][n_ant][nd]
    float2* jhr;             // [n_int][n_ant][nd]
    int32_t* count;          // [n_int][n_ant]
    float* stats;            // per-baseline sufficient statistics scratch
    const int32_t* ant1;
    const int32_t* ant2;
    const int64_t* row_off;
    const int32_t* ns;
    const int32_t* order;
    int32_t* queue;
    int32_t n_ant, n_bl, n_int, n_dir, n_corr, max_iter, schedule, algo, precision;
    double tol;
};

// StefCal runs the statistics solve in WCAL_MODE_STATS unless every interval holds one
// sample (the statistics of one sample are no smaller than the sample: the PASS solve runs)
inline bool di_stats_solve(const wcal_plan* plan) {
    return plan->prob.mode == WCAL_MODE_STATS && plan->max_ns > 1;
}

// launchers (return a hipError_t)
hipError_t launch_di_solve(const wcal_plan* plan, const DiArgs& a, hipStream_t s);
hipError_t launch_di_accumulate(const wcal_plan* plan, const DiArgs& a, hipStream_t s);
hipError_t launch_di_residual(const wcal_plan* plan, const DiArgs& a, hipStream_t s);
size_t di_accumulate_smem(int n_ant, int nc, int block);
int di_nvp(int nc);                        // floats per antenna in a tile partial
int di_nstat(int nc);                      // floats per baseline of the statistics

hipError_t launch_dd_solve(const wcal_plan* plan, const DdArgs& a, hipStream_t s);
hipError_t launch_dd_accumulate(const wcal_plan* plan, const DdArgs& a, hipStream_t s);
hipError_t launch_dd_residual(const wcal_plan* plan, const DdArgs& a, hipStream_t s);
size_t dd_stats_bytes(const wcal_problem& p);
// LDS a workgroup of the per-antenna and residual kernels needs at n_ant = na: the largest
// dynamic size they are launched with plus their static LDS (as the runtime reports it)
size_t dd_lds_need(int nd, int na);
int dd_max_dir();

// 2x2 Jones gains (n_corr == 4)
hipError_t launch_ddp_solve(const wcal_plan* plan, const DdArgs& a, hipStream_t s);
hipError_t launch_ddp_accumulate(const wcal_plan* plan, const DdArgs& a, hipStream_t s);
hipError_t launch_ddp_residual(const wcal_plan* plan, const DdArgs& a, hipStream_t s);
size_t ddp_stats_bytes(const wcal_problem& p);
size_t ddp_lds_need(int nd, int na);
int ddp_max_dir();
const char* ddp_pass_kernel_name(int nd);

hipError_t launch_reset_queue(int32_t* q, hipStream_t s);
// static LDS of a kernel in bytes (hipFuncGetAttributes), or 32 KiB if the runtime cannot say
size_t kernel_static_lds(const void* fn);

// pieces of the scalar solve reused by the smoothed solve
void fill_di_args(const wcal_plan* plan, DiArgs& a);
hipError_t launch_di_pass_partials(const wcal_plan* plan, const wcal_plan* prof_plan, const DiArgs& a, int it,
                                   hipStream_t s);
const int32_t* di_pass_tile_off(const wcal_plan* plan);
int32_t di_pass_ntiles(const wcal_plan* plan);
hipError_t launch_di_resid_tiles(const wcal_plan* plan, const wcal_plan* prof_plan, const DiArgs& a, hipStream_t s);
void smooth_free(struct SmoothPlan* sp);
