// The work ring of the device-side iteration loop.  One persistent launch solves every
// interval: workgroups take tiles from the ring; the workgroup that finishes the last tile of
// an interval's update applies the update and, while the interval keeps iterating, puts the
// interval's tiles back.  Solution intervals are independent (Sect. 2.3), so nothing but the
// ring ties them together.
//
// The leader thread of a workgroup calls these functions (ring_put may be called by any
// thread, one position each).  Waits poll with relaxed loads; the acquire fence follows once
// the awaited word is there.  The atomics come from a
// policy class `Ops`, so that the same protocol runs on the device (agent-scope atomics) and,
// in a CPU test, between host threads.  LOOP_FN is defined by the includer (the device code
// marks the functions __device__).
//
// Positions.  HEAD and TAIL are 64-bit position counters.  Position P lives in slot P mod cap
// at lap L = P / cap.  A slot word is (tag << 32) | tile with tag 2L while the slot waits for
// lap L's producer and 2L + 1 once it holds lap L's tile; the consumer of lap L, having read
// the tile, moves the slot to 2(L + 1).  The first round's tiles sit in positions
// [0, ntiles) from the start, so TAIL starts at ntiles.
//
// Why no wait lasts forever (cap >= ntiles):
//  * a tile is in the ring at most once: an interval puts its tiles back only after all of
//    them were finished, so positions reserved and not yet consumed number at most ntiles;
//  * a consumer waits on a position someone reserved or will reserve; the reserving
//    workgroup is running and writes right away (after a wait of its own, below), so the
//    tile arrives, or no live interval is left (LIVE = 0), which ends the wait;
//  * a producer of position P waits for the consumer of P - cap.  Positions P - cap .. P are
//    cap + 1 > ntiles reserved positions, so not all of them are unconsumed: some position
//    after P - cap was taken, hence P - cap was taken too (HEAD hands positions out in
//    order), by a running workgroup that waits for exactly that slot and then frees it.
// Every wait is still bounded (wait_ticks of the 100 MHz real-time counter): a wait that runs
// out sets ABORT, which ends every other wait, and the intervals still live are reported.
// The work is bounded too: no interval puts its tiles back more than max_iter - 1 times, so a
// solve uses at most `limit` = ntiles * max_iter positions; a position beyond it holds no tile
// (ring_pop returns -1 at once) and a put beyond it is a broken invariant (ABORT).  However an
// interval misbehaved, every workgroup leaves after at most `limit` positions in all.
#pragma once

#include <cstdint>

enum LoopWord { LW_HEAD, LW_TAIL };           // int64 position counters
enum LoopFlag { LF_LIVE, LF_ABORT };          // int32 words after them

struct LoopRing {
    int64_t* pos;          // [2] HEAD, TAIL
    int32_t* flag;         // [2] LIVE (intervals still iterating), ABORT
    uint64_t* ring;        // [cap] slot words
    int32_t* done;         // [n_int] tiles of the interval's current update finished
    int64_t cap;           // ring slots (>= ntiles)
    int64_t limit;         // positions a solve can use: ntiles * max_iter (every tile once per update)
    int64_t wait_ticks;    // bound of every wait
};

__attribute__((always_inline)) inline constexpr uint64_t ring_word(int64_t tag, uint32_t tile) {
    return ((uint64_t)tag << 32) | tile;
}

// Take the next position and wait for its tile.  Returns the tile, or -1 when none will come
// (every interval finished, the loop aborted, or this wait ran out, which sets ABORT).  Once
// ABORT is set no tile is handed out any more.
template <class Ops>
LOOP_FN int32_t ring_pop(const LoopRing& q, Ops& o) {
    const int64_t p = o.add64(&q.pos[LW_HEAD], 1);
    if (p >= q.limit) return -1;
    const int64_t lap = p / q.cap;
    uint64_t* slot = q.ring + (p - lap * q.cap);
    const int64_t t0 = o.now();
    for (;;) {
        if (o.load32(&q.flag[LF_ABORT]) != 0) return -1;
        const uint64_t w = o.load64(slot);
        if ((int64_t)(w >> 32) == 2 * lap + 1) {
            o.acquire();   // what the producer wrote before the tile is visible from here on
            // same slot as the load, so the tile was read before the slot is freed
            o.store64_relaxed(slot, ring_word(2 * lap + 2, 0));
            return (int32_t)(uint32_t)w;
        }
        if (o.load32(&q.flag[LF_LIVE]) == 0) return -1;
        if (o.now() - t0 > q.wait_ticks) {
            o.store32(&q.flag[LF_ABORT], 1);
            return -1;
        }
        o.pause();
    }
}

// Reserve n consecutive positions for the tiles of one interval; returns the first.
template <class Ops>
LOOP_FN int64_t ring_reserve(const LoopRing& q, Ops& o, int32_t n) {
    return o.add64(&q.pos[LW_TAIL], n);
}

// Write `tile` at reserved position p once the slot is free for p's lap.  Returns false if
// the loop aborted (or this wait ran out, which sets ABORT).
template <class Ops>
LOOP_FN bool ring_put(const LoopRing& q, Ops& o, int64_t p, int32_t tile) {
    if (p >= q.limit) {
        o.store32(&q.flag[LF_ABORT], 1);
        return false;
    }
    const int64_t lap = p / q.cap;
    uint64_t* slot = q.ring + (p - lap * q.cap);
    const int64_t t0 = o.now();
    for (;;) {
        if (o.load32(&q.flag[LF_ABORT]) != 0) return false;
        const uint64_t w = o.load64(slot);
        if ((int64_t)(w >> 32) == 2 * lap) {
            o.store64_release(slot, ring_word(2 * lap + 1, (uint32_t)tile));
            return true;
        }
        if (o.now() - t0 > q.wait_ticks) {
            o.store32(&q.flag[LF_ABORT], 1);
            return false;
        }
        o.pause();
    }
}

// Count one finished tile of interval k's current update (the tile's sums must be visible
// before the call).  True for the call that finishes the update's last of n tiles, which
// also re-arms the counter for the next update.
template <class Ops>
LOOP_FN bool ring_tile_done(const LoopRing& q, Ops& o, int32_t k, int32_t n) {
    const int32_t old = o.add32_acq_rel(&q.done[k], 1);
    if (old + 1 < n) return false;
    o.store32(&q.done[k], 0);
    return true;
}

// Interval finished for good: one fewer live interval.
template <class Ops>
LOOP_FN void ring_retire(const LoopRing& q, Ops& o) {
    o.add32_acq_rel(&q.flag[LF_LIVE], -1);
}
