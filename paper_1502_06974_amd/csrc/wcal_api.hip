// Host side of the C ABI declared in include/wcal.h: validation, plan tables, launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "wcal_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}


int hip_fail(hipError_t e, const char* where) {
    return fail(WCAL_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

template <typename T>
hipError_t upload(T** dst, const T* src, size_t n) {
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), std::max<size_t>(n, 1) * sizeof(T));
    if (e != hipSuccess) return e;
    if (n) e = hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

int check_common(const wcal_plan* plan, const void* data, const void* model, const void* gains) {
    if (!plan) return fail(WCAL_EINVAL, "plan is NULL");
    if (!data || !model || !gains) return fail(WCAL_EINVAL, "data, model and gains are required");
    const size_t al = plan->prob.n_corr == 4 ? 16 : 8;
    if (!aligned(data, al) || !aligned(model, al) || !aligned(gains, 8))
        return fail(WCAL_EINVAL, "data/model must be 8-byte aligned (16-byte for n_corr = 4)");
    if (hipSetDevice(plan->device) != hipSuccess) return fail(WCAL_EHIP, "hipSetDevice failed");
    return WCAL_OK;
}

}  // namespace

int wcal_error(int code, const std::string& msg) { return fail(code, msg); }

struct Profiler {
    struct Rec { int cls; hipEvent_t a, b; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    std::vector<hipEvent_t> open;   // begin events awaiting their end, per class
};

void prof_begin(const wcal_plan* plan, int cls, hipStream_t s) {
    Profiler* p = plan->prof;
    if (!p) return;
    if (p->open.size() < WCAL_K_COUNT) p->open.assign(WCAL_K_COUNT, nullptr);
    hipEvent_t e = p->get();
    (void)hipEventRecord(e, s);
    p->open[cls] = e;
}

void prof_end(const wcal_plan* plan, int cls, hipStream_t s) {
    Profiler* p = plan->prof;
    if (!p || p->open.size() < WCAL_K_COUNT || !p->open[cls]) return;
    hipEvent_t e = p->get();
    (void)hipEventRecord(e, s);
    p->recs.push_back({cls, p->open[cls], e});
    p->open[cls] = nullptr;
}

extern "C" {

extern "C++" bool watch_stop(const wcal_plan* plan, hipStream_t s, const int32_t* d_count, int it) {
    SlotWatch* w = plan->watch;
    if (!w) return false;
    if (it == 0) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        w->live = hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone;
    }
    if (!w->live) return false;
    const int r = it % w->depth;
    if (hipEventRecord(w->slot_ev[r], s) != hipSuccess || hipStreamWaitEvent(w->side, w->slot_ev[r], 0) != hipSuccess ||
        hipMemcpyAsync(w->host + r, d_count, sizeof(int32_t), hipMemcpyDeviceToHost, w->side) != hipSuccess ||
        hipEventRecord(w->copy_ev[r], w->side) != hipSuccess) {
        w->live = false;   // every remaining slot is enqueued, as without the watch
        return false;
    }
    if (it + 1 < w->depth) return false;
    const int r0 = (it + 1) % w->depth;   // the copy of slot it + 1 - depth
    if (hipEventSynchronize(w->copy_ev[r0]) != hipSuccess) {
        w->live = false;
        return false;
    }
    return *static_cast<volatile int32_t*>(w->host + r0) == 0;
}

static void watch_free(wcal_plan* plan) {
    SlotWatch* w = plan->watch;
    if (!w) return;
    if (w->side) (void)hipStreamSynchronize(w->side);
    for (hipEvent_t e : w->slot_ev) if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : w->copy_ev) if (e) (void)hipEventDestroy(e);
    if (w->side) (void)hipStreamDestroy(w->side);
    if (w->host) (void)hipHostFree(w->host);
    delete w;
    plan->watch = nullptr;
}

int wcal_plan_watch(wcal_plan* plan, int32_t depth) {
    g_err.clear();
    if (!plan) return fail(WCAL_EINVAL, "plan is NULL");
    if (depth < 0 || depth > WCAL_WATCH_MAX) return fail(WCAL_EINVAL, "watch depth must be in [0, WCAL_WATCH_MAX]");
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipSetDevice(plan->device);
    watch_free(plan);
    int rc = WCAL_OK;
    if (depth > 0) {
        SlotWatch* w = new SlotWatch;
        plan->watch = w;
        w->depth = depth;
        w->slot_ev.assign(depth, nullptr);
        w->copy_ev.assign(depth, nullptr);
        hipError_t e = hipStreamCreateWithFlags(&w->side, hipStreamNonBlocking);
        for (int i = 0; i < depth && e == hipSuccess; ++i) {
            e = hipEventCreateWithFlags(&w->slot_ev[i], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&w->copy_ev[i], hipEventDisableTiming);
        }
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&w->host), depth * sizeof(int32_t), hipHostMallocDefault);
        if (e != hipSuccess) {
            watch_free(plan);
            rc = hip_fail(e, "wcal_plan_watch");
        }
    }
    (void)hipSetDevice(dev);
    return rc;
}

int wcal_profile_enable(wcal_plan* plan, int enable) {
    g_err.clear();
    if (!plan) return fail(WCAL_EINVAL, "plan is NULL");
    if (enable && !plan->prof) plan->prof = new Profiler();
    if (!enable && plan->prof) {
        for (auto& r : plan->prof->recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        for (auto e : plan->prof->pool) (void)hipEventDestroy(e);
        delete plan->prof;
        plan->prof = nullptr;
    }
    return WCAL_OK;
}

int wcal_profile_read(wcal_plan* plan, double* ms, int32_t* launches) {
    g_err.clear();
    if (!plan || !ms || !launches) return fail(WCAL_EINVAL, "NULL argument");
    for (int i = 0; i < WCAL_K_COUNT; ++i) { ms[i] = 0.0; launches[i] = 0; }
    if (!plan->prof) return WCAL_OK;
    for (auto& r : plan->prof->recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(WCAL_EHIP, "hipEventSynchronize failed");
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return fail(WCAL_EHIP, "hipEventElapsedTime failed");
        ms[r.cls] += t;
        launches[r.cls] += 1;
        plan->prof->pool.push_back(r.a);
        plan->prof->pool.push_back(r.b);
    }
    plan->prof->recs.clear();
    return WCAL_OK;
}


const char* wcal_last_error(void) { return g_err.c_str(); }

const char* wcal_version(void) { return "wcal 0.1 (gfx950)"; }

// The tiling of a plan for a target of `tile_rows` rows per tile, with or without the
// triangle pass (used only where the plan allows it), computed on the host.
struct TilePlan {
    int64_t tile_rows = 0;
    bool tri = false;
    bool paired = false;
    std::vector<Tile> tiles, stiles, ttiles;
    std::vector<int32_t> tile_off, ttile_off;
    std::vector<TriUnit> units;
};

static int plan_tiles(const wcal_plan* plan, int64_t tile_rows, bool want_tri, TilePlan& tp) {
    const wcal_problem& p = plan->prob;
    const std::vector<int32_t>& ns32 = plan->h_ns;
    tp = TilePlan();
    tp.tile_rows = tile_rows;
    tp.tri = want_tri && plan->canonical && p.algo == WCAL_STEFCAL && p.n_corr == 1 && !di_stats_solve(plan);
    // tiles: samples per tile S and baselines per tile (a multiple of the 256-lane
    // workgroup) chosen for about tile_rows rows; interval k owns a contiguous tile range
    const int TBL = 256;
    auto round_up = [](int64_t x, int64_t m) { return (x + m - 1) / m * m; };
    std::vector<Tile>& tiles = tp.tiles;
    std::vector<Tile>& stiles = tp.stiles;
    std::vector<int32_t>& tile_off = tp.tile_off;
    tile_off.assign(p.n_int + 1, 0);
    for (int32_t k = 0; k < p.n_int; ++k) {
        const int64_t tr = tile_rows;
        const int32_t S = (int32_t)std::max<int64_t>(1, std::min<int64_t>(tr / p.n_bl, ns32[k]));
        const int32_t bc = (int32_t)std::min<int64_t>(std::max<int64_t>(round_up((tr + S - 1) / S, TBL), TBL),
                                                       round_up(p.n_bl, TBL));
        for (int32_t s0 = 0; s0 < ns32[k]; s0 += S)
            for (int32_t b0 = 0; b0 < p.n_bl; b0 += bc)
                tiles.push_back(Tile{k, b0, std::min(b0 + bc, p.n_bl), s0, std::min(s0 + S, ns32[k])});
        tile_off[k + 1] = (int32_t)tiles.size();
        if (p.mode == WCAL_MODE_STATS) {
            const int32_t bs = (int32_t)std::min<int64_t>(
                std::max<int64_t>(round_up((tr + ns32[k] - 1) / ns32[k], TBL), TBL), round_up(p.n_bl, TBL));
            for (int32_t b0 = 0; b0 < p.n_bl; b0 += bs)
                stiles.push_back(Tile{k, b0, std::min(b0 + bs, p.n_bl), 0, ns32[k]});
        }
        if (tiles.size() > (size_t)INT32_MAX / 4) return fail(WCAL_ESHAPE, "too many tiles");
    }
    std::vector<TriUnit>& units = tp.units;
    std::vector<Tile>& ttiles = tp.ttiles;
    std::vector<int32_t>& ttile_off = tp.ttile_off;
    ttile_off.assign(p.n_int + 1, 0);
    // units: blocks of whole rows (at most 64) of about 8 chunks of 64 baselines (the cost of
    // a row is its chunk count), then ordered largest first and dealt in snake order, so the
    // round-robin share of each of the four wavefronts of a workgroup is even; rows, or packed
    // rows (row n_ant - 2 - r with row r)
    auto build_units = [&](bool paired) {
        units.clear();
        ttiles.clear();
        ttile_off.assign(p.n_int + 1, 0);
        const int32_t target = 8;
        const int32_t nrows = paired ? p.n_ant / 2 : p.n_ant - 1;
        std::vector<TriUnit> raw;
        for (int32_t r0 = 0; r0 < nrows;) {
            int32_t r1 = r0, ent = 0, chunks = 0;
            while (r1 < nrows && r1 - r0 < 32) {
                const int32_t len = !paired ? p.n_ant - 1 - r1 : (p.n_ant - 2 - r1 > r1 ? p.n_ant : p.n_ant - 1 - r1);
                const int32_t ch = (len + 63) / 64;
                if (r1 > r0 && chunks + ch > target) break;
                ent += len;
                chunks += ch;
                ++r1;
            }
            raw.push_back(TriUnit{r0, r1, ent, chunks});
            r0 = r1;
        }
        std::stable_sort(raw.begin(), raw.end(), [](const TriUnit& x, const TriUnit& y) { return x.chunks > y.chunks; });
        const int nwv = 4;
        std::vector<std::vector<TriUnit>> lanes(nwv);
        for (size_t i = 0; i < raw.size(); ++i) {
            const size_t r = i / nwv, c = i % nwv;
            lanes[(r % 2 == 0) ? c : nwv - 1 - c].push_back(raw[i]);
        }
        for (size_t r = 0; r * nwv < raw.size(); ++r)
            for (int c = 0; c < nwv; ++c)
                if (r < lanes[c].size()) units.push_back(lanes[c][r]);
        const int64_t tr = tile_rows;
        for (int32_t k = 0; k < p.n_int; ++k) {
            const int32_t S = (int32_t)std::max<int64_t>(1, std::min<int64_t>(tr / p.n_bl, ns32[k]));
            for (int32_t s0 = 0; s0 < ns32[k]; s0 += S) {
                const int32_t s1 = std::min(s0 + S, ns32[k]);
                int32_t u0 = 0;
                while (u0 < (int32_t)units.size()) {
                    int64_t ent = 0;
                    int32_t u1 = u0;
                    while (u1 < (int32_t)units.size() && (u1 == u0 || (ent + units[u1].entries) * (s1 - s0) <= tr))
                        ent += units[u1++].entries;
                    ttiles.push_back(Tile{k, u0, u1, s0, s1});
                    u0 = u1;
                }
            }
            ttile_off[k + 1] = (int32_t)ttiles.size();
            if (ttiles.size() > (size_t)INT32_MAX / 4) return false;
        }
        return true;
    };
    if (tp.tri) {
        // Packed rows fill the chunks of short rows (from TRI_PAIR_MIN antennas on), which pays
        // in the unfused pass (9% on the smoothing cell plan) but not in the fused pass, whose
        // per-lane row selection costs more than the fuller chunks save (1% slower on
        // bandpass_na256): pairs are used unless every interval is one tile (the fused pass),
        // or always for plans whose triangle tiles only feed the unfused pass.
        if (!build_units(false)) return fail(WCAL_ESHAPE, "too many tiles");
        const bool fused = (int32_t)ttiles.size() == p.n_int;
        tp.paired = p.n_ant >= TRI_PAIR_MIN && (plan->tri_unfused || !fused);
        if (tp.paired && !build_units(true)) return fail(WCAL_ESHAPE, "too many tiles");
    }
    // statistics tiles in decreasing-size order (longest first)
    std::stable_sort(stiles.begin(), stiles.end(), [](const Tile& x, const Tile& y) {
        return (int64_t)(x.b1 - x.b0) * (x.s1 - x.s0) > (int64_t)(y.b1 - y.b0) * (y.s1 - y.s0);
    });
    return WCAL_OK;
}

// Workspace regions of a plan with the given tile counts (the triangle tiles drive the
// device-side loop when `tri`).  Returns the bytes of the plan's own regions.
static size_t layout_for(const wcal_plan* plan, int32_t ntiles, int32_t nttiles, bool tri, WsLayout& L) {
    const wcal_problem& p = plan->prob;
    const int32_t ntmax = std::max(ntiles, nttiles);
    const bool di = p.algo == WCAL_STEFCAL;
    const size_t nvp = di ? (size_t)di_nvp(p.n_corr) : 0;
    size_t sz[WS_COUNT] = {};
    sz[WS_CTR] = sizeof(int32_t) * (2 * ((size_t)p.max_iter + 2) + 16);
    sz[WS_ACTIVE] = sizeof(int32_t) * (size_t)p.n_int * (di ? 2 : 1);
    sz[WS_QUEUE] = 4 * sizeof(int32_t);
    sz[WS_LISTS] = 2 * sizeof(int32_t) * (size_t)std::max(1, ntmax);
    sz[WS_PARTIAL] = sizeof(float) * std::max<size_t>(1, (size_t)ntmax * p.n_ant * nvp);
    sz[WS_CHI_PART] = sizeof(double) * (size_t)std::max(1, ntiles);
    if (di) {
        if (di_stats_solve(plan)) sz[WS_STATS] = sizeof(float) * (size_t)p.n_int * p.n_bl * di_nstat(p.n_corr);
        else if (plan->loop) sz[WS_LOOP] = loop_bytes(tri ? nttiles : ntiles, p.n_int);
    } else {
        sz[WS_STATS] = p.n_corr == 4 ? ddp_stats_bytes(p) : dd_stats_bytes(p);
    }
    L.off[0] = 0;
    for (int i = 0; i < WS_COUNT; ++i) L.off[i + 1] = L.off[i] + ws_round(sz[i]);
    return L.off[WS_COUNT];
}

extern "C++" void ws_layout(wcal_plan* plan) {
    const size_t own = layout_for(plan, plan->ntiles, plan->nttiles, plan->tri, plan->ws);
    plan->ws_bytes = own + (plan->smooth ? smooth_ws_bytes(plan->smooth) : 0);
}

extern "C++" void ws_bind(wcal_plan* plan, char* ws) {
    const size_t* o = plan->ws.off;
    plan->d_ctr = reinterpret_cast<int32_t*>(ws + o[WS_CTR]);
    plan->d_active = reinterpret_cast<int32_t*>(ws + o[WS_ACTIVE]);
    plan->d_queue = reinterpret_cast<int32_t*>(ws + o[WS_QUEUE]);
    plan->d_lists = reinterpret_cast<int32_t*>(ws + o[WS_LISTS]);
    plan->d_partial = reinterpret_cast<float*>(ws + o[WS_PARTIAL]);
    plan->d_chi_part = reinterpret_cast<double*>(ws + o[WS_CHI_PART]);
    plan->d_stats = reinterpret_cast<float*>(ws + o[WS_STATS]);
    plan->stats_bytes = o[WS_STATS + 1] - o[WS_STATS];
    plan->d_loop = reinterpret_cast<int32_t*>(ws + o[WS_LOOP]);
    if (plan->smooth) smooth_ws_bind(plan->smooth, ws + o[WS_COUNT]);
}

extern "C++" int ws_check_bind(wcal_plan* plan, void* ws, size_t ws_bytes) {
    if (!ws) return fail(WCAL_EINVAL, "workspace is NULL (size it with wcal_plan_workspace)");
    if (reinterpret_cast<uintptr_t>(ws) % WS_ALIGN)
        return fail(WCAL_EINVAL, "workspace must be " + std::to_string(WS_ALIGN) + "-byte aligned");
    if (ws_bytes < plan->ws_bytes)
        return fail(WCAL_ENOMEM, "workspace of " + std::to_string(ws_bytes) + " bytes, the plan needs " +
                                     std::to_string(plan->ws_bytes));
    ws_bind(plan, reinterpret_cast<char*>(ws));
    return WCAL_OK;
}

// Replace the plan's tile tables by those of `tp` and lay out its workspace anew.
static int upload_tiles(wcal_plan* plan, const TilePlan& tp) {
    for (void** q : {(void**)&plan->d_tiles, (void**)&plan->d_tile_off, (void**)&plan->d_stiles,
                     (void**)&plan->d_units, (void**)&plan->d_ttiles, (void**)&plan->d_ttile_off}) {
        if (*q) (void)hipFree(*q);
        *q = nullptr;
    }
    plan->tile_rows = (int)tp.tile_rows;
    plan->tri = tp.tri;
    plan->tri_paired = tp.tri && tp.paired;
    plan->ntiles = (int32_t)tp.tiles.size();
    plan->nstiles = (int32_t)tp.stiles.size();
    plan->nunits = tp.tri ? (int32_t)tp.units.size() : 0;
    plan->nttiles = tp.tri ? (int32_t)tp.ttiles.size() : 0;
    hipError_t e = hipSuccess;
    if (tp.tri && ((e = upload(&plan->d_units, tp.units.data(), tp.units.size())) != hipSuccess ||
                   (e = upload(&plan->d_ttiles, tp.ttiles.data(), tp.ttiles.size())) != hipSuccess ||
                   (e = upload(&plan->d_ttile_off, tp.ttile_off.data(), tp.ttile_off.size())) != hipSuccess))
        return e == hipErrorOutOfMemory ? fail(WCAL_ENOMEM, "device allocation failed") : hip_fail(e, "plan units");
    if ((e = upload(&plan->d_tiles, tp.tiles.data(), tp.tiles.size())) != hipSuccess ||
        (e = upload(&plan->d_tile_off, tp.tile_off.data(), tp.tile_off.size())) != hipSuccess ||
        (e = upload(&plan->d_stiles, tp.stiles.data(), tp.stiles.size())) != hipSuccess)
        return e == hipErrorOutOfMemory ? fail(WCAL_ENOMEM, "device allocation failed") : hip_fail(e, "plan tiles");
    ws_layout(plan);
    return WCAL_OK;
}

static int build_tiles(wcal_plan* plan, int64_t tile_rows, bool want_tri) {
    TilePlan tp;
    if (int rc = plan_tiles(plan, tile_rows, want_tri, tp)) return rc;
    return upload_tiles(plan, tp);
}

// Rebuild the plan's tiles with its current tiling (after a change of tri_unfused).
extern "C++" int plan_retile(wcal_plan* plan) { return build_tiles(plan, plan->tile_rows, plan->tri); }

int wcal_plan_create(const wcal_problem* prob, const int32_t* ant1_h, const int32_t* ant2_h,
                     const int64_t* ns_h, int device, wcal_plan** out) {
    g_err.clear();
    if (!prob || !ant1_h || !ant2_h || !ns_h || !out) return fail(WCAL_EINVAL, "NULL argument");
    *out = nullptr;
    const wcal_problem& p = *prob;
    if (p.n_ant < 2 || p.n_bl < 1 || p.n_dir < 1 || p.n_int < 1 || p.max_iter < 1)
        return fail(WCAL_EINVAL, "n_ant >= 2, n_bl, n_dir, n_int, max_iter >= 1 required");
    if (p.n_corr != 1 && p.n_corr != 4) return fail(WCAL_EINVAL, "n_corr must be 1 or 4");
    if (!(p.tol >= 0.0)) return fail(WCAL_EINVAL, "tol must be >= 0");
    if (p.schedule < WCAL_AVG_FIRST || p.schedule > WCAL_GN_ONLY) return fail(WCAL_EINVAL, "unknown schedule");
    if (p.mode != WCAL_MODE_PASS && p.mode != WCAL_MODE_STATS) return fail(WCAL_EINVAL, "unknown mode");
    if (p.precision != WCAL_PREC_FP32 && p.precision != WCAL_PREC_BF16_GRAM)
        return fail(WCAL_EINVAL, "unknown precision");
    if (p.precision != WCAL_PREC_FP32 && p.algo == WCAL_STEFCAL)
        return fail(WCAL_EINVAL, "the BF16 Gram is for CohJones / AllJones");
    if (p.precision != WCAL_PREC_FP32 && p.mode != WCAL_MODE_PASS)
        return fail(WCAL_EINVAL, "the BF16 Gram needs PASS mode (its residual column follows the gains)");
    if (p.precision != WCAL_PREC_FP32 && p.n_dir > 13)
        return fail(WCAL_ESHAPE, "the BF16 Gram holds at most 13 directions (16 columns: Nd, d, r twice)");
    if (p.max_iter > 100000) return fail(WCAL_ESHAPE, "max_iter > 100000");
    if (p.algo == WCAL_STEFCAL) {
        if (p.n_dir != 1) return fail(WCAL_EINVAL, "StefCal needs n_dir == 1 (use CohJones/AllJones)");
    } else if (p.algo == WCAL_COHJONES || p.algo == WCAL_ALLJONES) {
        if (p.n_corr == 4 && p.precision != WCAL_PREC_FP32)
            return fail(WCAL_EINVAL, "2x2 CohJones/AllJones take the FP32 Gram only");
        if (p.n_dir > (p.n_corr == 4 ? ddp_max_dir() : dd_max_dir()))
            return fail(WCAL_ESHAPE, "n_dir above the supported maximum");
    } else {
        return fail(WCAL_EINVAL, "unknown algorithm");
    }
    for (int32_t b = 0; b < p.n_bl; ++b) {
        const int32_t a1 = ant1_h[b], a2 = ant2_h[b];
        if (a1 < 0 || a1 >= p.n_ant || a2 < 0 || a2 >= p.n_ant)
            return fail(WCAL_EINDEX, "baseline " + std::to_string(b) + ": antenna index out of range");
        if (a1 == a2) return fail(WCAL_EINDEX, "baseline " + std::to_string(b) + ": autocorrelation (ant1 == ant2)");
    }
    std::vector<int64_t> off(p.n_int + 1, 0);
    std::vector<int32_t> ns32(p.n_int);
    int32_t max_ns = 0;
    for (int32_t k = 0; k < p.n_int; ++k) {
        if (ns_h[k] < 1) return fail(WCAL_ESHAPE, "interval " + std::to_string(k) + ": ns < 1");
        if (ns_h[k] > (int64_t)INT32_MAX / 4) return fail(WCAL_ESHAPE, "ns too large");
        ns32[k] = (int32_t)ns_h[k];
        max_ns = std::max(max_ns, ns32[k]);
        off[k + 1] = off[k] + (int64_t)p.n_bl * ns_h[k];
    }
    // longest-processing-time order for the work queue
    std::vector<int32_t> order(p.n_int);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return ns32[x] > ns32[y]; });

    if (hipSetDevice(device) != hipSuccess) return fail(WCAL_EHIP, "hipSetDevice failed");
    auto* plan = new wcal_plan();
    plan->prob = p;
    plan->device = device;
    plan->rows = off[p.n_int];
    plan->max_ns = max_ns;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete plan;
        return fail(WCAL_EHIP, "hipGetDeviceProperties failed");
    }
    plan->n_cu = prop.multiProcessorCount;
    plan->max_smem = prop.sharedMemPerBlock;
    if (p.algo != WCAL_STEFCAL &&
        (p.n_corr == 4 ? ddp_lds_need(p.n_dir, p.n_ant) : dd_lds_need(p.n_dir, p.n_ant)) > plan->max_smem) {
        delete plan;
        return fail(WCAL_ESHAPE, "n_ant * n_dir too large for the per-interval LDS working set");
    }
    if (const char* s = std::getenv("WCAL_BLOCK")) plan->block = std::max(64, std::min(1024, atoi(s)) / 64 * 64);
    if (const char* s = std::getenv("WCAL_WG_PER_CU")) plan->wg_per_cu = atoi(s);
    if (const char* s = std::getenv("WCAL_TILE_ROWS")) plan->tile_rows = atoi(s);
    if (plan->tile_rows <= 0) plan->tile_rows = 65536;
    // LDS budget of the kernels: per-antenna gains and per-wavefront accumulators
    if (p.algo == WCAL_STEFCAL && di_accumulate_smem(p.n_ant, p.n_corr, p.n_corr == 1 ? 1024 : 512) > 96 * 1024) {
        delete plan;
        return fail(WCAL_ESHAPE, "n_ant too large for the per-interval LDS working set");
    }
    plan->h_ns = ns32;
    {
        bool canonical = (int64_t)p.n_bl == (int64_t)p.n_ant * (p.n_ant - 1) / 2;
        for (int32_t a = 0, b = 0; canonical && a < p.n_ant; ++a)
            for (int32_t c = a + 1; canonical && c < p.n_ant; ++c, ++b)
                canonical = ant1_h[b] == a && ant2_h[b] == c;
        plan->canonical = canonical;
    }
    // The device-side loop (one persistent launch per solve) is switched off: its first runs on
    // the GPU did not finish and the cause is not found.  A request for it is refused.
    if (const char* s = std::getenv("WCAL_LOOP")) {
        if (atoi(s) != 0) {
            delete plan;
            return fail(WCAL_EINVAL, "the device-side iteration loop (WCAL_LOOP=1) is switched off");
        }
    }
    {
        // bound of the device-side loop's waits: WCAL_WAIT_MS milliseconds (default 10 s) in
        // ticks of the real-time counter
        // (the counter runs at 100 MHz on this family; a reported rate outside 1-1000 MHz is
        // not trusted)
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || khz < 1000 ||
            khz > 1000000)
            khz = 100000;
        double ms = 10000.0;
        if (const char* s = std::getenv("WCAL_WAIT_MS")) ms = std::max(0.0, atof(s));
        plan->wait_ticks = (int64_t)(ms * khz);
    }
    const char* env_tri = std::getenv("WCAL_TRI");
    const int want_tri = env_tri ? atoi(env_tri) : -1;   // 0: never, 1: whenever allowed, unset: n_ant >= 64
    hipError_t e = hipSuccess;
    if (int rc = build_tiles(plan, plan->tile_rows, want_tri == 1 || (want_tri < 0 && p.n_ant >= 64))) {
        wcal_plan_destroy(plan);
        return rc;
    }
    if ((e = upload(&plan->d_ant1, ant1_h, p.n_bl)) != hipSuccess ||
        (e = upload(&plan->d_ant2, ant2_h, p.n_bl)) != hipSuccess ||
        (e = upload(&plan->d_row_off, off.data(), off.size())) != hipSuccess ||
        (e = upload(&plan->d_ns, ns32.data(), ns32.size())) != hipSuccess ||
        (e = upload(&plan->d_order, order.data(), order.size())) != hipSuccess) {
        wcal_plan_destroy(plan);
        return e == hipErrorOutOfMemory ? fail(WCAL_ENOMEM, "device allocation failed") : hip_fail(e, "plan tables");
    }
    if (p.algo != WCAL_STEFCAL) {
        // rows touching each antenna: (baseline, side) in baseline order
        std::vector<int32_t> ptr(p.n_ant + 1, 0), bl(2 * (size_t)p.n_bl);
        for (int32_t b = 0; b < p.n_bl; ++b) { ++ptr[ant1_h[b] + 1]; ++ptr[ant2_h[b] + 1]; }
        for (int32_t i = 0; i < p.n_ant; ++i) ptr[i + 1] += ptr[i];
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
        for (int32_t b = 0; b < p.n_bl; ++b) {
            bl[fill[ant1_h[b]]++] = 2 * b;
            bl[fill[ant2_h[b]]++] = 2 * b + 1;
        }
        if ((e = upload(&plan->d_ant_ptr, ptr.data(), ptr.size())) != hipSuccess ||
            (e = upload(&plan->d_ant_bl, bl.data(), bl.size())) != hipSuccess) {
            wcal_plan_destroy(plan);
            return fail(WCAL_ENOMEM, "antenna tables allocation failed");
        }
    }
    *out = plan;
    return WCAL_OK;
}

void wcal_plan_destroy(wcal_plan* plan) {
    if (!plan) return;
    wcal_profile_enable(plan, 0);
    (void)hipSetDevice(plan->device);
    watch_free(plan);
    smooth_free(plan->smooth);
    plan->smooth = nullptr;
    // only the host-built tables are plan-owned; scratch lives in the caller's workspace
    for (void* p : {(void*)plan->d_ant1, (void*)plan->d_ant2, (void*)plan->d_row_off, (void*)plan->d_ns,
                    (void*)plan->d_order, (void*)plan->d_tiles, (void*)plan->d_tile_off, (void*)plan->d_stiles,
                    (void*)plan->d_ant_ptr, (void*)plan->d_ant_bl, (void*)plan->d_units, (void*)plan->d_ttiles,
                    (void*)plan->d_ttile_off})
        if (p) (void)hipFree(p);
    delete plan;
}

int64_t wcal_plan_rows(const wcal_plan* plan) { return plan ? plan->rows : -1; }

const char* wcal_plan_pass_kernel(const wcal_plan* plan) {
    if (!plan) return "";
    const wcal_problem& p = plan->prob;
    if (p.algo != WCAL_STEFCAL && p.n_corr == 4) return ddp_pass_kernel_name(p.n_dir);
    if (p.algo != WCAL_STEFCAL) return p.precision == WCAL_PREC_BF16_GRAM ? "dd_gram_dma_kernel" : "dd_gram_dmaf_kernel";
    if (di_stats_solve(plan)) return p.n_corr == 1 ? "di_stats_kernel<1>" : "di_stats_kernel<4>";
    if (plan->loop) return plan->tri ? "di_loop_kernel<1, true>" : p.n_corr == 1 ? "di_loop_kernel<1, false>" : "di_loop_kernel<4, false>";
    if (plan->tri) return "di_tri_pass_kernel";
    return p.n_corr == 1 ? "di_pass_kernel<1>" : "di_pass_kernel<4>";
}

static void fill_tables_di(const wcal_plan* plan, DiArgs& a) {
    a.ant1 = plan->d_ant1;
    a.ant2 = plan->d_ant2;
    a.row_off = plan->d_row_off;
    a.ns = plan->d_ns;
    a.order = plan->d_order;
    a.queue = plan->d_queue;
    a.tiles = plan->d_tiles;
    a.tile_off = plan->d_tile_off;
    a.ntiles = plan->ntiles;
    a.lists = plan->d_lists;
    a.ctr = plan->d_ctr;
    a.partial = plan->d_partial;
    a.active = plan->d_active;
    a.chi_part = plan->d_chi_part;
    a.stats = plan->d_stats;
    a.n_ant = plan->prob.n_ant;
    a.n_bl = plan->prob.n_bl;
    a.n_int = plan->prob.n_int;
    a.max_iter = plan->prob.max_iter;
    a.schedule = plan->prob.schedule;
    a.tri_paired = plan->tri_paired ? 1 : 0;
    a.tri_cnt = plan->d_active + plan->prob.n_int;
    a.tol = plan->prob.tol;
}

extern "C++" void fill_di_args(const wcal_plan* plan, DiArgs& a) { fill_tables_di(plan, a); }

static void fill_tables_dd(const wcal_plan* plan, DdArgs& a) {
    a.ant1 = plan->d_ant1;
    a.ant2 = plan->d_ant2;
    a.row_off = plan->d_row_off;
    a.ns = plan->d_ns;
    a.order = plan->d_order;
    a.queue = plan->d_queue;
    a.stats = plan->d_stats;
    a.n_ant = plan->prob.n_ant;
    a.n_bl = plan->prob.n_bl;
    a.n_int = plan->prob.n_int;
    a.n_dir = plan->prob.n_dir;
    a.n_corr = plan->prob.n_corr;
    a.max_iter = plan->prob.max_iter;
    a.schedule = plan->prob.schedule;
    a.algo = plan->prob.algo;
    a.tol = plan->prob.tol;
    a.precision = plan->prob.precision;
}

int wcal_plan_workspace(const wcal_plan* plan, size_t* bytes) {
    g_err.clear();
    if (!plan || !bytes) return fail(WCAL_EINVAL, "NULL argument");
    *bytes = plan->ws_bytes;
    return WCAL_OK;
}

int wcal_solve(wcal_plan* plan, const wcal_c64* data, const wcal_c64* model, const uint8_t* flags,
               wcal_c64* gains, wcal_c64* residual, int32_t* n_iter, uint32_t* status, double* chi2,
               void* workspace, size_t ws_bytes, void* stream) {
    g_err.clear();
    int rc = check_common(plan, data, model, gains);
    if (rc) return rc;
    if (!n_iter || !status) return fail(WCAL_EINVAL, "n_iter and status are required");
    if (residual && !aligned(residual, plan->prob.n_corr == 4 ? 16 : 8))
        return fail(WCAL_EINVAL, "residual misaligned");
    if ((rc = ws_check_bind(plan, workspace, ws_bytes))) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e;
    if (plan->prob.algo == WCAL_STEFCAL) {
        DiArgs a{};
        fill_tables_di(plan, a);
        a.data = reinterpret_cast<const float2*>(data);
        a.model = reinterpret_cast<const float2*>(model);
        a.flags = flags;
        a.gains = reinterpret_cast<float2*>(gains);
        a.residual = reinterpret_cast<float2*>(residual);
        a.n_iter = n_iter;
        a.status = status;
        a.chi2 = chi2;
        e = launch_di_solve(plan, a, s);
    } else {
        DdArgs a{};
        fill_tables_dd(plan, a);
        a.data = reinterpret_cast<const float2*>(data);
        a.model = reinterpret_cast<const float2*>(model);
        a.flags = flags;
        a.gains = reinterpret_cast<float2*>(gains);
        a.residual = reinterpret_cast<float2*>(residual);
        a.n_iter = n_iter;
        a.status = status;
        a.chi2 = chi2;
        e = plan->prob.n_corr == 4 ? launch_ddp_solve(plan, a, s) : launch_dd_solve(plan, a, s);
    }
    return e == hipSuccess ? WCAL_OK : hip_fail(e, "wcal_solve launch");
}

// The checks of a points plan and grid shared by wcal_points_workspace and wcal_solve_points.
static int points_check(const wcal_plan* plan, const wcal_points* pts) {
    const wcal_problem& p = plan->prob;
    if ((p.algo != WCAL_COHJONES && p.algo != WCAL_ALLJONES) || p.n_corr != 1 || p.precision != WCAL_PREC_FP32)
        return fail(WCAL_EINVAL, "predicted point-source models need scalar CohJones / AllJones with the FP32 Gram");
    if (pts->n_time < 1 || pts->n_chan < 1 || !std::isfinite(pts->freq0) || !std::isfinite(pts->dfreq))
        return fail(WCAL_EINVAL, "n_time, n_chan >= 1 and finite frequencies required");
    for (int32_t k = 0; k < p.n_int; ++k)
        if (plan->h_ns[k] != (int64_t)pts->n_time * pts->n_chan)
            return fail(WCAL_ESHAPE, "every interval must hold n_time * n_chan samples");
    return WCAL_OK;
}

int wcal_points_workspace(const wcal_plan* plan, const wcal_points* pts, size_t* bytes) {
    g_err.clear();
    if (!plan || !pts || !bytes) return fail(WCAL_EINVAL, "NULL argument");
    if (int rc = points_check(plan, pts)) return rc;
    *bytes = ws_round(plan->ws_bytes) + points_table_bytes(plan->prob, pts->n_time, pts->n_chan);
    return WCAL_OK;
}

int wcal_solve_points(wcal_plan* plan, const wcal_points* pts, const wcal_c64* data, const uint8_t* flags,
                      wcal_c64* gains, wcal_c64* residual, int32_t* n_iter, uint32_t* status, double* chi2,
                      void* workspace, size_t ws_bytes, void* stream) {
    g_err.clear();
    if (!plan || !pts || !data || !gains || !n_iter || !status) return fail(WCAL_EINVAL, "NULL argument");
    const wcal_problem& p = plan->prob;
    if (int rc = points_check(plan, pts)) return rc;
    if (!pts->uvw || !pts->lmn || !pts->flux) return fail(WCAL_EINVAL, "uvw, lmn and flux are required");
    if (!aligned(data, 8) || !aligned(gains, 8) || (residual && !aligned(residual, 8)) || !aligned(pts->uvw, 8) ||
        !aligned(pts->lmn, 8) || !aligned(pts->flux, 4))
        return fail(WCAL_EINVAL, "misaligned argument");
    if (hipSetDevice(plan->device) != hipSuccess) return fail(WCAL_EHIP, "hipSetDevice failed");
    // the plan's regions, then the phasor table
    const size_t base = ws_round(plan->ws_bytes);
    const size_t tab = points_table_bytes(p, pts->n_time, pts->n_chan);
    if (workspace && ws_bytes < base + tab)
        return fail(WCAL_ENOMEM, "workspace of " + std::to_string(ws_bytes) + " bytes, the points solve needs " +
                                     std::to_string(base + tab) + " (wcal_points_workspace)");
    if (int rc = ws_check_bind(plan, workspace, ws_bytes)) return rc;
    DdArgs a{};
    fill_tables_dd(plan, a);
    a.data = reinterpret_cast<const float2*>(data);
    a.model = nullptr;
    a.pt.nseg = (pts->n_chan + 63) / 64;
    a.pt.zt = reinterpret_cast<float2*>(static_cast<char*>(workspace) + base);
    a.pt.st = reinterpret_cast<float2*>(static_cast<char*>(workspace) + base +
                                        ws_round((size_t)p.n_int * pts->n_time * p.n_bl * p.n_dir * a.pt.nseg * 4 *
                                                 sizeof(float2)));
    a.pt.uvw = pts->uvw;
    a.pt.lmn = pts->lmn;
    a.pt.flux = pts->flux;
    a.pt.freq0 = pts->freq0;
    a.pt.dfreq = pts->dfreq;
    a.pt.n_time = pts->n_time;
    a.pt.n_chan = pts->n_chan;
    a.flags = flags;
    a.gains = reinterpret_cast<float2*>(gains);
    a.residual = reinterpret_cast<float2*>(residual);
    a.n_iter = n_iter;
    a.status = status;
    a.chi2 = chi2;
    const hipError_t e = launch_dd_solve(plan, a, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? WCAL_OK : hip_fail(e, "wcal_solve_points launch");
}

// Candidate tilings of the autotuner.
static const int64_t kTuneRows[] = {8192, 16384, 32768, 65536, 131072, 262144};

// Bytes of the autotuner's own scratch at the start of its workspace: a copy of the gains, the
// update counts and the status words of the timed solves.
static size_t tune_scratch_bytes(const wcal_problem& p) {
    return ws_round((size_t)p.n_int * p.n_dir * p.n_ant * p.n_corr * sizeof(wcal_c64)) +
           2 * ws_round(sizeof(int32_t) * (size_t)p.n_int);
}

static bool tune_tri_ok(const wcal_plan* plan) {
    return plan->canonical && plan->prob.n_corr == 1 && !di_stats_solve(plan);
}

int wcal_plan_autotune_workspace(const wcal_plan* plan, size_t* bytes) {
    g_err.clear();
    if (!plan || !bytes) return fail(WCAL_EINVAL, "NULL argument");
    const wcal_problem& p = plan->prob;
    if (p.algo != WCAL_STEFCAL) {
        *bytes = plan->ws_bytes;
        return WCAL_OK;
    }
    const size_t extra = plan->smooth ? smooth_ws_bytes(plan->smooth) : 0;
    size_t most = plan->ws_bytes;
    for (int tri = 0; tri <= (tune_tri_ok(plan) ? 1 : 0); ++tri)
        for (int64_t tr : kTuneRows) {
            TilePlan tp;
            if (int rc = plan_tiles(plan, tr, tri != 0, tp)) return rc;
            WsLayout L;
            most = std::max(most, layout_for(plan, (int32_t)tp.tiles.size(), (int32_t)tp.ttiles.size(), tp.tri, L) + extra);
        }
    *bytes = tune_scratch_bytes(p) + most;
    return WCAL_OK;
}

int wcal_plan_autotune(wcal_plan* plan, const wcal_c64* data, const wcal_c64* model, const uint8_t* flags,
                       const wcal_c64* gains, int32_t n_updates, void* workspace, size_t ws_bytes, void* stream,
                       int32_t* tile_rows_out, int32_t* tri_out) {
    g_err.clear();
    int rc = check_common(plan, data, model, gains);
    if (rc) return rc;
    if (n_updates < 0 || n_updates > plan->prob.max_iter)
        return fail(WCAL_EINVAL, "n_updates must be in [0, max_iter]");
    if (plan->prof) return fail(WCAL_EINVAL, "disable profiling before tuning");
    if (!workspace) return fail(WCAL_EINVAL, "workspace is NULL (size it with wcal_plan_autotune_workspace)");
    if (reinterpret_cast<uintptr_t>(workspace) % WS_ALIGN)
        return fail(WCAL_EINVAL, "workspace must be " + std::to_string(WS_ALIGN) + "-byte aligned");
    wcal_problem& p = plan->prob;
    auto report = [&]() {
        if (tile_rows_out) *tile_rows_out = plan->tile_rows;
        if (tri_out) *tri_out = plan->tri ? 1 : 0;
        return WCAL_OK;
    };
    // CohJones / AllJones stream the rows in their own Gram pass: nothing to tune
    if (p.algo != WCAL_STEFCAL) return report();
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // the tuner's scratch first, the solves' workspace after it
    const size_t tune = tune_scratch_bytes(p);
    if (ws_bytes < tune) return fail(WCAL_ENOMEM, "workspace smaller than the autotuner's scratch");
    char* base = reinterpret_cast<char*>(workspace);
    const size_t gbytes = (size_t)p.n_int * p.n_dir * p.n_ant * p.n_corr * sizeof(wcal_c64);
    wcal_c64* g = reinterpret_cast<wcal_c64*>(base);
    int32_t* nit = reinterpret_cast<int32_t*>(base + ws_round(gbytes));
    uint32_t* st = reinterpret_cast<uint32_t*>(base + ws_round(gbytes) + ws_round(sizeof(int32_t) * p.n_int));
    char* solve_ws = base + tune;
    const size_t solve_bytes = ws_bytes - tune;
    const size_t extra = plan->smooth ? smooth_ws_bytes(plan->smooth) : 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(WCAL_EHIP, "autotune events");
    }
    // every candidate applies exactly n_updates updates (tol 0) from the given gains, or with
    // n_updates = 0 runs the plan's own solve (to its tolerance, so the tail of the last
    // intervals still iterating is timed too); candidates whose workspace does not fit are
    // skipped
    const int saved_iter = p.max_iter;
    const double saved_tol = p.tol;
    if (n_updates > 0) {
        p.max_iter = n_updates;
        p.tol = 0.0;
    }
    const int64_t start_rows = plan->tile_rows;
    const bool start_tri = plan->tri;
    int64_t best_rows = start_rows;
    bool best_tri = start_tri;
    float best_ms = 1e30f;
    int err = WCAL_OK, tried = 0;
    for (int tri = 0; tri <= (tune_tri_ok(plan) ? 1 : 0) && err == WCAL_OK; ++tri) {
        for (int64_t tr : kTuneRows) {
            TilePlan tp;
            if ((err = plan_tiles(plan, tr, tri != 0, tp)) != WCAL_OK) break;
            WsLayout L;
            if (layout_for(plan, (int32_t)tp.tiles.size(), (int32_t)tp.ttiles.size(), tp.tri, L) + extra > solve_bytes)
                continue;
            if ((err = upload_tiles(plan, tp)) != WCAL_OK) break;
            ++tried;
            float ms = 1e30f;
            for (int rep = 0; rep < 3 && err == WCAL_OK; ++rep) {
                if (hipMemcpyAsync(g, gains, gbytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                    hipEventRecord(e0, s) != hipSuccess) {
                    err = fail(WCAL_EHIP, "autotune copy failed");
                    break;
                }
                err = wcal_solve(plan, data, model, flags, g, nullptr, nit, st, nullptr, solve_ws, solve_bytes, stream);
                if (err != WCAL_OK) break;
                float t = 0.f;
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
                    err = fail(WCAL_EHIP, "autotune timing failed");
                    break;
                }
                if (rep > 0) ms = std::min(ms, t);      // the first run warms caches and code
            }
            if (err == WCAL_OK && ms < best_ms) {
                best_ms = ms;
                best_rows = tr;
                best_tri = tri != 0;
            }
        }
    }
    p.max_iter = saved_iter;
    p.tol = saved_tol;
    cleanup();
    if (err == WCAL_OK && tried == 0)
        err = fail(WCAL_ENOMEM, "no candidate tiling fits the workspace (size it with wcal_plan_autotune_workspace)");
    if (err != WCAL_OK) {
        (void)build_tiles(plan, start_rows, start_tri);
        return err;
    }
    if ((err = build_tiles(plan, best_rows, best_tri)) != WCAL_OK) return err;
    return report();
}

struct wcal_graph {
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

int wcal_solve_graph(wcal_plan* plan, const wcal_c64* data, const wcal_c64* model, const uint8_t* flags,
                     wcal_c64* gains, wcal_c64* residual, int32_t* n_iter, uint32_t* status, double* chi2,
                     void* workspace, size_t ws_bytes, void* stream, wcal_graph** out) {
    g_err.clear();
    if (!out) return fail(WCAL_EINVAL, "out is NULL");
    *out = nullptr;
    if (!plan) return fail(WCAL_EINVAL, "plan is NULL");
    if (plan->prof) return fail(WCAL_EINVAL, "disable profiling before capturing a solve");
    if (hipSetDevice(plan->device) != hipSuccess) return fail(WCAL_EHIP, "hipSetDevice failed");
    // the legacy null stream cannot be captured: capture on a private stream instead
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipStream_t own = nullptr;
    if (!s) {
        if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess)
            return fail(WCAL_EHIP, "hipStreamCreateWithFlags failed");
        s = own;
    }
    auto done = [&](int rc) {
        if (own) (void)hipStreamDestroy(own);
        return rc;
    };
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return done(fail(WCAL_EHIP, "hipStreamBeginCapture failed"));
    const int rc = wcal_solve(plan, data, model, flags, gains, residual, n_iter, status, chi2, workspace, ws_bytes, s);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &graph);
    if (rc != WCAL_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return done(rc);
    }
    if (ec != hipSuccess || !graph) return done(hip_fail(ec, "hipStreamEndCapture"));
    auto* g = new wcal_graph();
    g->device = plan->device;
    g->graph = graph;
    const hipError_t ei = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        wcal_graph_destroy(g);
        return done(hip_fail(ei, "hipGraphInstantiate"));
    }
    *out = g;
    return done(WCAL_OK);
}

int wcal_graph_launch(wcal_graph* graph, void* stream) {
    g_err.clear();
    if (!graph) return fail(WCAL_EINVAL, "graph is NULL");
    if (hipSetDevice(graph->device) != hipSuccess) return fail(WCAL_EHIP, "hipSetDevice failed");
    const hipError_t e = hipGraphLaunch(graph->exec, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? WCAL_OK : hip_fail(e, "hipGraphLaunch");
}

void wcal_graph_destroy(wcal_graph* graph) {
    if (!graph) return;
    (void)hipSetDevice(graph->device);
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
}

int wcal_accumulate(wcal_plan* plan, const wcal_c64* data, const wcal_c64* model, const uint8_t* flags,
                    const wcal_c64* gains, wcal_c64* jhj, wcal_c64* jhd, wcal_c64* jhr, int32_t* count,
                    double* chi2, wcal_c64* residual, void* workspace, size_t ws_bytes, void* stream) {
    g_err.clear();
    int rc = check_common(plan, data, model, gains);
    if (rc) return rc;
    if (!jhj || !jhd || !jhr) return fail(WCAL_EINVAL, "jhj, jhd and jhr are required");
    if (residual && !aligned(residual, plan->prob.n_corr == 4 ? 16 : 8))
        return fail(WCAL_EINVAL, "residual misaligned");
    if ((rc = ws_check_bind(plan, workspace, ws_bytes))) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e;
    if (plan->prob.algo == WCAL_STEFCAL) {
        DiArgs a{};
        fill_tables_di(plan, a);
        a.data = reinterpret_cast<const float2*>(data);
        a.model = reinterpret_cast<const float2*>(model);
        a.flags = flags;
        a.gains_in = reinterpret_cast<const float2*>(gains);
        a.residual = reinterpret_cast<float2*>(residual);
        a.chi2 = chi2;
        a.jhj = reinterpret_cast<float2*>(jhj);
        a.jhd = reinterpret_cast<float2*>(jhd);
        a.jhr = reinterpret_cast<float2*>(jhr);
        a.count = count;
        e = launch_di_accumulate(plan, a, s);
    } else {
        DdArgs a{};
        fill_tables_dd(plan, a);
        a.data = reinterpret_cast<const float2*>(data);
        a.model = reinterpret_cast<const float2*>(model);
        a.flags = flags;
        a.gains_in = reinterpret_cast<const float2*>(gains);
        a.residual = reinterpret_cast<float2*>(residual);
        a.chi2 = chi2;
        a.jhj = reinterpret_cast<float2*>(jhj);
        a.jhd = reinterpret_cast<float2*>(jhd);
        a.jhr = reinterpret_cast<float2*>(jhr);
        a.count = count;
        e = plan->prob.n_corr == 4 ? launch_ddp_accumulate(plan, a, s) : launch_dd_accumulate(plan, a, s);
    }
    return e == hipSuccess ? WCAL_OK : hip_fail(e, "wcal_accumulate launch");
}

int wcal_residual(wcal_plan* plan, const wcal_c64* data, const wcal_c64* model, const uint8_t* flags,
                  const wcal_c64* gains, wcal_c64* residual, double* chi2, void* workspace, size_t ws_bytes,
                  void* stream) {
    g_err.clear();
    int rc = check_common(plan, data, model, gains);
    if (rc) return rc;
    if (!residual && !chi2) return fail(WCAL_EINVAL, "residual or chi2 is required");
    if (residual && !aligned(residual, plan->prob.n_corr == 4 ? 16 : 8))
        return fail(WCAL_EINVAL, "residual misaligned");
    if ((rc = ws_check_bind(plan, workspace, ws_bytes))) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e;
    if (plan->prob.algo == WCAL_STEFCAL) {
        DiArgs a{};
        fill_tables_di(plan, a);
        a.data = reinterpret_cast<const float2*>(data);
        a.model = reinterpret_cast<const float2*>(model);
        a.flags = flags;
        a.gains_in = reinterpret_cast<const float2*>(gains);
        a.residual = reinterpret_cast<float2*>(residual);
        a.chi2 = chi2;
        e = launch_di_residual(plan, a, s);
    } else {
        DdArgs a{};
        fill_tables_dd(plan, a);
        a.data = reinterpret_cast<const float2*>(data);
        a.model = reinterpret_cast<const float2*>(model);
        a.flags = flags;
        a.gains_in = reinterpret_cast<const float2*>(gains);
        a.residual = reinterpret_cast<float2*>(residual);
        a.chi2 = chi2;
        e = plan->prob.n_corr == 4 ? launch_ddp_residual(plan, a, s) : launch_dd_residual(plan, a, s);
    }
    return e == hipSuccess ? WCAL_OK : hip_fail(e, "wcal_residual launch");
}

}  // extern "C"
