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

// (Re)build the tiles of a plan for a target of `tile_rows` rows per tile, with or without
// the triangle pass (used only where the plan allows it), and (re)allocate what depends on
// the tile count.  Host-side; no kernel runs.
static int build_tiles(wcal_plan* plan, int64_t tile_rows, bool want_tri) {
    const wcal_problem& p = plan->prob;
    const std::vector<int32_t>& ns32 = plan->h_ns;
    for (void** q : {(void**)&plan->d_tiles, (void**)&plan->d_tile_off, (void**)&plan->d_stiles,
                     (void**)&plan->d_lists, (void**)&plan->d_partial, (void**)&plan->d_chi_part,
                     (void**)&plan->d_units, (void**)&plan->d_ttiles, (void**)&plan->d_ttile_off}) {
        if (*q) (void)hipFree(*q);
        *q = nullptr;
    }
    plan->tile_rows = (int)tile_rows;
    plan->nunits = plan->nttiles = 0;
    plan->tri = want_tri && plan->canonical && p.algo == WCAL_STEFCAL && p.n_corr == 1 && !di_stats_solve(plan);
    // tiles: samples per tile S and baselines per tile (a multiple of the 256-lane
    // workgroup) chosen for about tile_rows rows; interval k owns a contiguous tile range
    const int TBL = 256;
    auto round_up = [](int64_t x, int64_t m) { return (x + m - 1) / m * m; };
    std::vector<Tile> tiles, stiles;
    std::vector<int32_t> tile_off(p.n_int + 1, 0);
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
        if (tiles.size() > (size_t)INT32_MAX / 2) return fail(WCAL_ESHAPE, "too many tiles");
    }
    std::vector<TriUnit> units;
    std::vector<Tile> ttiles;
    std::vector<int32_t> ttile_off(p.n_int + 1, 0);
    if (plan->tri) {
        // units: blocks of whole rows (at most 64) of about 8 chunks of 64 baselines (the
        // cost of a row is its chunk count), then ordered largest first and dealt in snake
        // order, so the round-robin share of each of the four wavefronts of a workgroup is
        // even
        const int32_t target = 8;
        // rows, or packed rows (row n_ant - 2 - r with row r) from TRI_PAIR_MIN antennas on
        const bool paired = p.n_ant >= TRI_PAIR_MIN;
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
            if (ttiles.size() > (size_t)INT32_MAX / 2) return fail(WCAL_ESHAPE, "too many tiles");
        }
        plan->nunits = (int32_t)units.size();
        plan->nttiles = (int32_t)ttiles.size();
    }
    // statistics tiles in decreasing-size order (longest first)
    std::stable_sort(stiles.begin(), stiles.end(), [](const Tile& x, const Tile& y) {
        return (int64_t)(x.b1 - x.b0) * (x.s1 - x.s0) > (int64_t)(y.b1 - y.b0) * (y.s1 - y.s0);
    });
    plan->ntiles = (int32_t)tiles.size();
    plan->nstiles = (int32_t)stiles.size();
    const int nvp = p.algo == WCAL_STEFCAL ? di_nvp(p.n_corr) : 0;
    const int32_t ntmax = std::max(plan->ntiles, plan->nttiles);
    hipError_t e = hipSuccess;
    if (plan->tri && ((e = upload(&plan->d_units, units.data(), units.size())) != hipSuccess ||
                      (e = upload(&plan->d_ttiles, ttiles.data(), ttiles.size())) != hipSuccess ||
                      (e = upload(&plan->d_ttile_off, ttile_off.data(), ttile_off.size())) != hipSuccess))
        return e == hipErrorOutOfMemory ? fail(WCAL_ENOMEM, "device allocation failed") : hip_fail(e, "plan units");
    if ((e = upload(&plan->d_tiles, tiles.data(), tiles.size())) != hipSuccess ||
        (e = upload(&plan->d_tile_off, tile_off.data(), tile_off.size())) != hipSuccess ||
        (e = upload(&plan->d_stiles, stiles.data(), stiles.size())) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void**>(&plan->d_lists), 2 * sizeof(int32_t) * std::max(1, ntmax))) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void**>(&plan->d_partial),
                       sizeof(float) * std::max<size_t>(1, (size_t)ntmax * p.n_ant * nvp))) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void**>(&plan->d_chi_part), sizeof(double) * std::max(1, plan->ntiles))) != hipSuccess)
        return e == hipErrorOutOfMemory ? fail(WCAL_ENOMEM, "device allocation failed") : hip_fail(e, "plan tiles");
    return WCAL_OK;
}

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
        (p.n_corr == 4 ? ddp_smem_bytes(p.n_dir, p.n_ant) : dd_smem_bytes(p.n_dir, p.n_ant)) > plan->max_smem) {
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
    const char* env_tri = std::getenv("WCAL_TRI");
    const int want_tri = env_tri ? atoi(env_tri) : -1;   // 0: never, 1: whenever allowed, unset: n_ant >= 64
    hipError_t e = hipSuccess;
    if (int rc = build_tiles(plan, plan->tile_rows, want_tri == 1 || (want_tri < 0 && p.n_ant >= 64))) {
        wcal_plan_destroy(plan);
        return rc;
    }
    if ((e = hipMalloc(reinterpret_cast<void**>(&plan->d_ctr), sizeof(int32_t) * (2 * (p.max_iter + 2) + 16))) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void**>(&plan->d_active), sizeof(int32_t) * p.n_int)) != hipSuccess) {
        wcal_plan_destroy(plan);
        return e == hipErrorOutOfMemory ? fail(WCAL_ENOMEM, "device allocation failed") : hip_fail(e, "plan state");
    }
    if (p.algo == WCAL_STEFCAL && di_stats_solve(plan)) {
        plan->stats_bytes = sizeof(float) * (size_t)p.n_int * p.n_bl * di_nstat(p.n_corr);
        if ((e = hipMalloc(reinterpret_cast<void**>(&plan->d_stats), plan->stats_bytes)) != hipSuccess) {
            wcal_plan_destroy(plan);
            return fail(WCAL_ENOMEM, "statistics allocation failed");
        }
    }
    if ((e = upload(&plan->d_ant1, ant1_h, p.n_bl)) != hipSuccess ||
        (e = upload(&plan->d_ant2, ant2_h, p.n_bl)) != hipSuccess ||
        (e = upload(&plan->d_row_off, off.data(), off.size())) != hipSuccess ||
        (e = upload(&plan->d_ns, ns32.data(), ns32.size())) != hipSuccess ||
        (e = upload(&plan->d_order, order.data(), order.size())) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void**>(&plan->d_queue), 4 * sizeof(int32_t))) != hipSuccess) {
        wcal_plan_destroy(plan);
        return e == hipErrorOutOfMemory ? fail(WCAL_ENOMEM, "device allocation failed") : hip_fail(e, "plan tables");
    }
    if (p.algo != WCAL_STEFCAL) {
        plan->stats_bytes = p.n_corr == 4 ? ddp_stats_bytes(p) : dd_stats_bytes(p);
        if ((e = hipMalloc(reinterpret_cast<void**>(&plan->d_stats), plan->stats_bytes)) != hipSuccess) {
            wcal_plan_destroy(plan);
            return fail(WCAL_ENOMEM, "Gram record allocation failed");
        }
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
    smooth_free(plan->smooth);
    plan->smooth = nullptr;
    for (void* p : {(void*)plan->d_ant1, (void*)plan->d_ant2, (void*)plan->d_row_off, (void*)plan->d_ns,
                    (void*)plan->d_order, (void*)plan->d_queue, (void*)plan->d_stats, (void*)plan->d_tiles,
                    (void*)plan->d_tile_off, (void*)plan->d_stiles, (void*)plan->d_lists, (void*)plan->d_ctr,
                    (void*)plan->d_partial, (void*)plan->d_active, (void*)plan->d_chi_part,
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

int wcal_solve(wcal_plan* plan, const wcal_c64* data, const wcal_c64* model, const uint8_t* flags,
               wcal_c64* gains, wcal_c64* residual, int32_t* n_iter, uint32_t* status, double* chi2,
               void* stream) {
    g_err.clear();
    int rc = check_common(plan, data, model, gains);
    if (rc) return rc;
    if (!n_iter || !status) return fail(WCAL_EINVAL, "n_iter and status are required");
    if (residual && !aligned(residual, plan->prob.n_corr == 4 ? 16 : 8))
        return fail(WCAL_EINVAL, "residual misaligned");
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

int wcal_solve_points(wcal_plan* plan, const wcal_points* pts, const wcal_c64* data, const uint8_t* flags,
                      wcal_c64* gains, wcal_c64* residual, int32_t* n_iter, uint32_t* status, double* chi2,
                      void* stream) {
    g_err.clear();
    if (!plan || !pts || !data || !gains || !n_iter || !status) return fail(WCAL_EINVAL, "NULL argument");
    const wcal_problem& p = plan->prob;
    if ((p.algo != WCAL_COHJONES && p.algo != WCAL_ALLJONES) || p.n_corr != 1 || p.precision != WCAL_PREC_FP32)
        return fail(WCAL_EINVAL, "predicted point-source models need scalar CohJones / AllJones with the FP32 Gram");
    if (!pts->uvw || !pts->lmn || !pts->flux) return fail(WCAL_EINVAL, "uvw, lmn and flux are required");
    if (pts->n_time < 1 || pts->n_chan < 1 || !std::isfinite(pts->freq0) || !std::isfinite(pts->dfreq))
        return fail(WCAL_EINVAL, "n_time, n_chan >= 1 and finite frequencies required");
    for (int32_t k = 0; k < p.n_int; ++k)
        if (plan->h_ns[k] != (int64_t)pts->n_time * pts->n_chan)
            return fail(WCAL_ESHAPE, "every interval must hold n_time * n_chan samples");
    if (!aligned(data, 8) || !aligned(gains, 8) || (residual && !aligned(residual, 8)) || !aligned(pts->uvw, 8) ||
        !aligned(pts->lmn, 8) || !aligned(pts->flux, 4))
        return fail(WCAL_EINVAL, "misaligned argument");
    if (hipSetDevice(plan->device) != hipSuccess) return fail(WCAL_EHIP, "hipSetDevice failed");
    DdArgs a{};
    fill_tables_dd(plan, a);
    a.data = reinterpret_cast<const float2*>(data);
    a.model = nullptr;
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

int wcal_plan_autotune(wcal_plan* plan, const wcal_c64* data, const wcal_c64* model, const uint8_t* flags,
                       const wcal_c64* gains, int32_t n_updates, void* stream, int32_t* tile_rows_out,
                       int32_t* tri_out) {
    g_err.clear();
    int rc = check_common(plan, data, model, gains);
    if (rc) return rc;
    if (n_updates < 0 || n_updates > plan->prob.max_iter)
        return fail(WCAL_EINVAL, "n_updates must be in [0, max_iter]");
    if (plan->prof) return fail(WCAL_EINVAL, "disable profiling before tuning");
    wcal_problem& p = plan->prob;
    auto report = [&]() {
        if (tile_rows_out) *tile_rows_out = plan->tile_rows;
        if (tri_out) *tri_out = plan->tri ? 1 : 0;
        return WCAL_OK;
    };
    // CohJones / AllJones stream the rows in their own Gram pass: nothing to tune
    if (p.algo != WCAL_STEFCAL) return report();
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const size_t gbytes = (size_t)p.n_int * p.n_dir * p.n_ant * p.n_corr * sizeof(wcal_c64);
    wcal_c64* g = nullptr;
    int32_t* nit = nullptr;
    uint32_t* st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (g) (void)hipFree(g);
        if (nit) (void)hipFree(nit);
        if (st) (void)hipFree(st);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (hipMalloc(reinterpret_cast<void**>(&g), gbytes) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&nit), sizeof(int32_t) * p.n_int) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&st), sizeof(uint32_t) * p.n_int) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(WCAL_ENOMEM, "autotune scratch allocation failed");
    }
    // every candidate applies exactly n_updates updates (tol 0) from the given gains, or with
    // n_updates = 0 runs the plan's own solve (to its tolerance, so the tail of the last
    // intervals still iterating is timed too)
    const int saved_iter = p.max_iter;
    const double saved_tol = p.tol;
    if (n_updates > 0) {
        p.max_iter = n_updates;
        p.tol = 0.0;
    }
    const bool tri_ok = plan->canonical && p.n_corr == 1 && !di_stats_solve(plan);
    const int64_t rows_cand[] = {8192, 16384, 32768, 65536, 131072, 262144};
    int64_t best_rows = plan->tile_rows;
    bool best_tri = plan->tri;
    float best_ms = 1e30f;
    int err = WCAL_OK;
    for (int tri = 0; tri <= (tri_ok ? 1 : 0) && err == WCAL_OK; ++tri) {
        for (int64_t tr : rows_cand) {
            if ((err = build_tiles(plan, tr, tri != 0)) != WCAL_OK) break;
            float ms = 1e30f;
            for (int rep = 0; rep < 3 && err == WCAL_OK; ++rep) {
                if (hipMemcpyAsync(g, gains, gbytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                    hipEventRecord(e0, s) != hipSuccess) {
                    err = fail(WCAL_EHIP, "autotune copy failed");
                    break;
                }
                err = wcal_solve(plan, data, model, flags, g, nullptr, nit, st, nullptr, stream);
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
    if (err != WCAL_OK) return err;
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
                     void* stream, wcal_graph** out) {
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
    const int rc = wcal_solve(plan, data, model, flags, gains, residual, n_iter, status, chi2, s);
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
                    double* chi2, wcal_c64* residual, void* stream) {
    g_err.clear();
    int rc = check_common(plan, data, model, gains);
    if (rc) return rc;
    if (!jhj || !jhd || !jhr) return fail(WCAL_EINVAL, "jhj, jhd and jhr are required");
    if (residual && !aligned(residual, plan->prob.n_corr == 4 ? 16 : 8))
        return fail(WCAL_EINVAL, "residual misaligned");
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
                  const wcal_c64* gains, wcal_c64* residual, double* chi2, void* stream) {
    g_err.clear();
    int rc = check_common(plan, data, model, gains);
    if (rc) return rc;
    if (!residual && !chi2) return fail(WCAL_EINVAL, "residual or chi2 is required");
    if (residual && !aligned(residual, plan->prob.n_corr == 4 ? 16 : 8))
        return fail(WCAL_EINVAL, "residual misaligned");
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
