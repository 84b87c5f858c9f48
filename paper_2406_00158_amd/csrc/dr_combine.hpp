// dr_combine.hpp — deterministic combine of partial sums into the result(s)
// of a reduction, inside the launch that produced them.
//
// The paper's reduce computes a partial per segment and adds the partials
// once all are complete (section 4.3, "reduce"; Algorithm 3). Here a
// "unit" is what one result covers: one segment's tiles (BATCH), or all the
// tiles of the launch (CONCAT), and its members are those tiles.
// Each member publishes its partial; the last member to arrive in a group of
// 64 consecutive members sums the group's partials, and the last group to
// arrive sums the group sums and adds `init`. Arrivals are counted with
// agent-scope fetch-and-add on counters the launch prologue zeroed; the sums
// always run in member order over a fixed tree, so a result does not depend
// on the order in which workgroups happen to finish. Partials carry the
// launch's epoch tag: a reader spins until the one it needs is visible.
#pragma once

#include <type_traits>

#include "dr_device.hpp"

namespace dr {

// result[unit] = init combined with `sum` (the unit's combined partials).
template <class P, int CMB = kCmbSum>
__device__ __forceinline__ void write_result(const LaunchArgs& a, int64_t unit, P sum) {
    const bool mn = (a.flags & kFlagMin) != 0;
    if constexpr (!std::is_floating_point<P>::value) {
        ((int64_t*)a.result)[unit] = cmb_op<CMB>(a.init_i, (int64_t)sum, mn);
    } else {
        ((double*)a.result)[unit] = cmb_op<CMB>(a.init_f, (double)sum, mn);
    }
}

template <class P>
__device__ __forceinline__ P wait_tagged(const LaunchArgs& a, const uint64_t* w, uint32_t tag) {
    uint64_t bitsv = 0;
    if (!tagged_load(w, tag, bitsv)) {
        Deadline dl(a.spin_ticks);
        while (!tagged_load(w, tag, bitsv)) {
            if (dl.passed()) {
                flag_error(a, DR_DEVFLAG_TIMEOUT);
                bitsv = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return from_bits<P>(bitsv);
}

// Results of the empty BATCH segments that follow segment k (k = -1: the
// leading ones) are `init`: written by the workgroup of the first tile of
// the preceding non-empty segment. Thread 0 only.
template <class P, int CMB = kCmbSum>
__device__ __forceinline__ void fill_empty_after(const LaunchArgs& a, int64_t k) {
    const P id = cmb_id<CMB, P>((a.flags & kFlagMin) != 0);
    for (int64_t kk = k + 1; kk < a.m && a.rows[kk].length == 0; ++kk) write_result<P, CMB>(a, kk, id);
}

// Member `idx` (0-based within its unit of `count` members, whose partial
// words start at member slot `base` of the tile-word array) publishes
// `partial` (held by lane 0) and, if it completes its group or the unit,
// combines. `slot0` is the unit's first group slot. Called by ONE whole wave
// (the other waves of the workgroup need not wait for it).
template <class P, int CMB = kCmbSum>
__device__ __forceinline__ void combine_member(const LaunchArgs& a, uint32_t tag, int64_t unit, int64_t base,
                                               int64_t idx, int64_t count, int64_t slot0, P partial) {
    const bool mn = (a.flags & kFlagMin) != 0;
    const P id = cmb_id<CMB, P>(mn);
    const int64_t gi = idx / kGroupTiles;
    const int64_t g0 = gi * kGroupTiles;
    const int64_t gn = (count - g0) < kGroupTiles ? (count - g0) : kGroupTiles;
    const int64_t ngroups = (count + kGroupTiles - 1) / kGroupTiles;
    uint64_t* tw = (uint64_t*)(a.ws + a.lay.off_tile);
    uint32_t* gcnt = (uint32_t*)(a.ws + a.lay.off_gcnt);
    uint64_t* gpart = (uint64_t*)(a.ws + a.lay.off_gpart);
    uint32_t* ucnt = (uint32_t*)(a.ws + a.lay.off_ucnt);
    const int64_t TW = a.lay.tile_words, PW = a.lay.part_word;
    const int l = lane_id();
    if (count == 1) {   // the unit's only member: nothing to wait for or count
        if (l == 0) write_result<P, CMB>(a, unit, partial);
        return;
    }

    int last_in_group = 0;
    if (l == 0) {
        tagged_store(tw + (base + idx) * TW + PW, tag, to_bits(partial));
        last_in_group = atomic_add32(gcnt + slot0 + gi, 1u) == (uint32_t)(gn - 1);
    }
    if (!readlane(last_in_group, 0)) return;
    // the group is complete: sum its partials in member order
    P v = id;
    if (l < gn) v = wait_tagged<P>(a, tw + (base + g0 + l) * TW + PW, tag);
    const P gsum = wave_reduce_cmb<CMB>(v, mn);
    if (ngroups == 1) {
        if (l == 0) write_result<P, CMB>(a, unit, gsum);
        return;
    }
    int last = 0;
    if (l == 0) {
        tagged_store(gpart + (slot0 + gi) * 2, tag, to_bits(gsum));
        last = atomic_add32(ucnt + unit, 1u) == (uint32_t)(ngroups - 1);
    }
    if (!readlane(last, 0)) return;
    P acc = id;
    for (int64_t g = l; g < ngroups; g += 64)
        acc = cmb_op<CMB>(acc, wait_tagged<P>(a, gpart + (slot0 + g) * 2, tag), mn);
    const P tot = wave_reduce_cmb<CMB>(acc, mn);
    if (l == 0) write_result<P, CMB>(a, unit, tot);
}

// BATCH: tile t of segment si publishes its partial; the segment's last
// group writes result[k]. Group slots of segment k start at first/64 + k.
// One whole wave.
template <class P, int CMB = kCmbSum>
__device__ __forceinline__ void combine_tile_batch(const LaunchArgs& a, uint32_t tag, int64_t t,
                                                   const SegInfo& si, P partial) {
    if (lane_id() == 0 && t == si.first) {
        if (t == 0) fill_empty_after<P, CMB>(a, -1);
        fill_empty_after<P, CMB>(a, si.k);
    }
    combine_member<P, CMB>(a, tag, si.k, si.first, t - si.first, si.ntiles, si.first / kGroupTiles + si.k,
                           partial);
}

// BATCH launch with no tiles at all: every result is `init`.
template <class P, int CMB = kCmbSum>
__device__ __forceinline__ void write_all_init(const LaunchArgs& a) {
    const P id = cmb_id<CMB, P>((a.flags & kFlagMin) != 0);
    for (int64_t k = 0; k < a.m; ++k) write_result<P, CMB>(a, k, id);
}

}  // namespace dr
