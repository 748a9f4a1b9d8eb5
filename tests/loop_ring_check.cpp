// CPU check of the device-side loop's work ring (csrc/loop_ring.h): host threads play the
// leaders of workgroups and run the protocol on a model solve, with random delays.
//   loop_ring_check <seed> <threads> <intervals> <max_tiles> <max_updates> <cap_extra> <wait_ticks> [limit]
// Each interval k has n_k tiles and keeps iterating for u_k updates.  Checks: every (interval,
// update, tile) is processed exactly once, tiles of update r + 1 only after update r was
// applied, every interval finishes, the ring ends empty, no wait runs out.  With wait_ticks = 0,
// or a position limit below what the intervals need (a runaway interval), it checks instead
// that every thread ends (through ABORT) and reports the live intervals.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#define LOOP_FN inline
#include "loop_ring.h"

struct HostOps {
    std::mt19937_64 rng;
    int64_t add64(int64_t* p, int64_t v) { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }
    int32_t add32_acq_rel(int32_t* p, int32_t v) { return __atomic_fetch_add(p, v, __ATOMIC_ACQ_REL); }
    uint64_t load64(uint64_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
    void acquire() { __atomic_thread_fence(__ATOMIC_ACQUIRE); }
    void store64_release(uint64_t* p, uint64_t v) { __atomic_store_n(p, v, __ATOMIC_RELEASE); }
    void store64_relaxed(uint64_t* p, uint64_t v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }
    int32_t load32(int32_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
    void store32(int32_t* p, int32_t v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }
    int64_t now() {
        return std::chrono::duration_cast<std::chrono::microseconds>(
                   std::chrono::steady_clock::now().time_since_epoch()).count();
    }
    void pause() { std::this_thread::yield(); }
    void jitter() {
        const int r = (int)(rng() % 16);
        if (r < 2) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 50));
        else if (r < 6) std::this_thread::yield();
    }
};

int main(int argc, char** argv) {
    if (argc != 8 && argc != 9) return 2;
    const uint64_t seed = strtoull(argv[1], nullptr, 10);
    const int nthr = atoi(argv[2]), nint = atoi(argv[3]), maxt = atoi(argv[4]), maxu = atoi(argv[5]);
    const int cap_extra = atoi(argv[6]);
    const int64_t wait = atoll(argv[7]);
    std::mt19937_64 g(seed);
    std::vector<int32_t> ntk(nint), upd(nint), toff(nint + 1, 0);
    for (int k = 0; k < nint; ++k) {
        ntk[k] = 1 + (int)(g() % maxt);
        upd[k] = 1 + (int)(g() % maxu);
        toff[k + 1] = toff[k] + ntk[k];
    }
    const int ntiles = toff[nint];
    std::vector<int32_t> tile_k(ntiles);
    for (int k = 0; k < nint; ++k)
        for (int t = toff[k]; t < toff[k + 1]; ++t) tile_k[t] = k;
    // ring state as the initialisation kernel leaves it
    std::vector<int64_t> pos = {0, ntiles};
    std::vector<int32_t> flag = {nint, 0};
    const int64_t cap = ntiles + cap_extra;
    std::vector<uint64_t> ring(cap, 0);
    for (int t = 0; t < ntiles; ++t) ring[t] = ring_word(1, (uint32_t)t);
    std::vector<int32_t> done(nint, 0);
    const int64_t limit = argc == 9 ? atoll(argv[8]) : (int64_t)ntiles * maxu;
    LoopRing q{pos.data(), flag.data(), ring.data(), done.data(), cap, limit, wait};
    // model solve state
    std::vector<int32_t> iter(nint, 0), finished(nint, 0);
    std::vector<std::atomic<int32_t>> seen((size_t)ntiles * maxu);
    for (auto& x : seen) x.store(0);
    std::atomic<int> errors{0};
    auto worker = [&](int id) {
        HostOps o{std::mt19937_64(seed * 1000 + id)};
        for (;;) {
            const int32_t t = ring_pop(q, o);
            if (t < 0) return;
            if (t >= ntiles) { errors++; return; }
            const int k = tile_k[t];
            const int r = __atomic_load_n(&iter[k], __ATOMIC_ACQUIRE);
            if (r >= upd[k] || __atomic_load_n(&finished[k], __ATOMIC_ACQUIRE)) { errors++; continue; }
            if (seen[(size_t)t * maxu + r].fetch_add(1) != 0) errors++;
            o.jitter();
            if (!ring_tile_done(q, o, k, ntk[k])) continue;
            // the last tile of update r: every tile of the update must have been seen once
            for (int u = toff[k]; u < toff[k + 1]; ++u)
                if (seen[(size_t)u * maxu + r].load() != 1) errors++;
            o.jitter();
            __atomic_store_n(&iter[k], r + 1, __ATOMIC_RELEASE);
            if (r + 1 == upd[k]) {
                __atomic_store_n(&finished[k], 1, __ATOMIC_RELEASE);
                ring_retire(q, o);
                continue;
            }
            const int64_t p0 = ring_reserve(q, o, ntk[k]);
            for (int i = 0; i < ntk[k]; ++i)
                if (!ring_put(q, o, p0 + i, toff[k] + i)) return;
        }
    };
    std::vector<std::thread> th;
    for (int i = 0; i < nthr; ++i) th.emplace_back(worker, i);
    for (auto& x : th) x.join();
    int live = 0;
    for (int k = 0; k < nint; ++k) live += !finished[k];
    if (wait == 0 || argc == 9) {
        // forced abort: every thread ended; the live count equals the unfinished intervals
        printf("aborted=%d live_flag=%d unfinished=%d errors=%d\n", flag[LF_ABORT], flag[LF_LIVE], live, errors.load());
        return (flag[LF_LIVE] == live && errors.load() == 0) ? 0 : 1;
    }
    int64_t total = 0;
    for (int k = 0; k < nint; ++k) {
        if (iter[k] != upd[k]) errors++;
        total += (int64_t)ntk[k] * upd[k];
    }
    for (int t = 0; t < ntiles; ++t)
        for (int r = 0; r < maxu; ++r)
            if (seen[(size_t)t * maxu + r].load() != (r < upd[tile_k[t]] ? 1 : 0)) errors++;
    const bool ok = errors.load() == 0 && flag[LF_ABORT] == 0 && flag[LF_LIVE] == 0 && live == 0 &&
                    pos[LW_TAIL] == total;
    printf("tiles=%d processed=%lld head=%lld tail=%lld abort=%d errors=%d %s\n", ntiles, (long long)total,
           (long long)pos[LW_HEAD], (long long)pos[LW_TAIL], flag[LF_ABORT], errors.load(), ok ? "OK" : "FAIL");
    return ok ? 0 : 1;
}
