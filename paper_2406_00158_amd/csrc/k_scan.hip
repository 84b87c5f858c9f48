// k_scan.hip — inclusive_scan over a zip/transform view of a segmented
// range (section 4.3, "inclusive_scan"; Algorithm 4), and its fusion with a
// transform_reduce over the same rows.
//
// The paper scans each segment locally, scans the segment totals, then adds
// each segment's offset in a second read-write pass over the data (the
// extra pass it blames for the scan's drop from one to two tiles, section
// 5.1). Three forms are built here, and the chained single pass for one
// long range in k_scan_chain.hip; every one writes each output once:
//  - reduce-then-scan (the default, except for the CONCAT sums past 2^22
//    elements that take the chained pass): a read-only pass forms every tile's
//    total, one small kernel scans the per-chunk totals, and the apply pass
//    re-reads the input, scans each tile in registers and adds its carry
//    (the input is read twice; carries are sums in a fixed order);
//  - decoupled look-back (DR_TUNE_TILE_PER_BLOCK; Merrill & Garland,
//    "Single-pass Parallel Prefix Scan with Decoupled Look-back", 2016): one
//    workgroup per tile, in block-index order, publishes its aggregate and
//    looks back over its predecessors' aggregates / inclusive prefixes for
//    its carry;
//  - specialised waves (DR_TUNE_SPECIALIZED): one pass with loader, writer,
//    publisher and carry-fetcher waves per workgroup and one workgroup that
//    scans the published tile totals in a fixed order.
// Carries cross segment boundaries in CONCAT mode (the carry of segment k
// is the total of the segments before it) and restart at every segment's
// first tile in BATCH mode.
//
// Precision: int32 inputs scan in int64 (exact). binary32 / bfloat16
// inputs scan in binary32 inside a tile; the carries between tiles are
// binary64 (or binary32 with DR_SCAN_CARRY_F32), and each output is the
// binary64 sum of the carry and the tile-local prefix rounded once to
// binary32. binary64 inputs scan in binary64.
//
// Reverse mode (suffix sums, the adjoint of the scan) processes tiles in
// reverse physical order and mirrors the element order inside each tile.
#include "k_scan_core.hpp"

namespace dr {

// ---------------------------------------------------------------------------
// Reduce-then-scan form (the default)
// ---------------------------------------------------------------------------
//
// A decoupled look-back makes every tile wait for the slowest of the
// predecessors still loading, and thousands of tiles are loading at once:
// at full bandwidth those waits, not the memory, set the pace. This form
// never waits on another workgroup:
//
//   pass 1  (k_scan_sums)   a resident grid; workgroup g streams the
//           contiguous chunk [g*Q, (g+1)*Q) of processing indices, forms
//           each tile's total exactly as the scan pass will, and writes each
//           tile's carry relative to the chunk start (or to the segment
//           start, BATCH) plus the chunk's (has-head, trailing sum) pair;
//   pass 1b (k_scan_chunks) one workgroup: segmented exclusive scan of the
//           chunk pairs, giving each chunk its incoming carry;
//   pass 2  (k_scan_apply)  one workgroup per tile: local scan in registers
//           plus the tile's carry, written once. The fused reduction's
//           partials and their combine run here.
//
// The input is read twice (12 bytes per binary32 element instead of 8), in
// two streaming passes. The carries are sums in a fixed order, so results
// are identical from run to run (for a given chunk count).
//
// The paper's scan is also a local pass, a scan of partial totals and a
// second pass over the data (section 4.3, Algorithm 4); here the first pass
// only reads, so the data is written once.

// Chunk area: [0] Q (tiles per chunk), [1] chunk count; chunk g at word
// 4 + 4g: [0] has a segment head, [1] carry bits of the sum after the last
// head (or of the whole chunk), [2] incoming carry bits (pass 1b).
constexpr int kChunkHdr = 4;

// Tile record (processing index r), words [0, 1] of the tile words:
// carry bits relative to the chunk start or the last head, and whether a
// head lies in [chunk start, r].
constexpr int kRecCarry = 0;
constexpr int kRecHead = 1;

template <int IDT, int OP, bool C64, int ITEMS, bool REV, int CMB>
__global__ __launch_bounds__(kBlock) void k_scan_sums(LaunchArgs a) {
    constexpr int V = vwidth<IDT>();
    constexpr int SLOTS = ITEMS / V;
    constexpr int WAVES = kBlock / 64;
    constexpr bool ZIP = zip_view<IDT, OP, false, 0>();
    using L = local_t<IDT>;
    using C = carry_t<IDT, C64>;
    __shared__ L s_wtot[2][WAVES];
    TileMap tm;
    tm.init(a);
    if (!tm.ok) return;
    const int64_t T = tm.total_tiles;
    const int64_t G = gridDim.x;
    const int64_t Q = (T + G - 1) / G;
    const int64_t g = blockIdx.x;
    uint64_t* cw = (uint64_t*)(a.ws + a.lay.off_chunk);
    uint64_t* tws = (uint64_t*)(a.ws + a.lay.off_tile);
    const int64_t TW = a.lay.tile_words;
    if (g == 0 && threadIdx.x == 0) {
        cw[0] = (uint64_t)Q;
        cw[1] = (uint64_t)G;
    }
    const int64_t r0 = g * Q < T ? g * Q : T;
    const int64_t r1 = r0 + Q < T ? r0 + Q : T;
    const int w = threadIdx.x >> 6, l = lane_id();
    const L alpha = (L)a.alpha;
    const bool mn = (a.flags & kFlagMin) != 0;

    C run = cmb_id<CMB, C>(mn);    // thread 0: carry of the next tile relative to the chunk / head
    bool seen = false;
    vec<IDT> xa[SLOTS], ya[SLOTS], xb[SLOTS], yb[SLOTS];
    SegInfo sa, sb;
    int64_t r = r0;
    bool ha = false, hb = false;
    auto tile_of = [&](int64_t rr) { return REV ? T - 1 - rr : rr; };
    auto issue = [&](int64_t rr, SegInfo& si, vec<IDT> (&x)[SLOTS], vec<IDT> (&y)[SLOTS]) -> bool {
        const int64_t t = tile_of(rr);
        if (!tm.find(a, t, si)) return false;
        const int64_t u0 = (t - si.first) * a.tile;
        load_slots<IDT, SLOTS>(x, si.in0, si, u0, w, l, REV);
        if constexpr (ZIP) load_slots<IDT, SLOTS>(y, si.in1, si, u0, w, l, REV);
        return true;
    };
    // one tile whose data is in (x, y): tile total, then (thread 0) its
    // record. A malformed row (flagged) counts as a head with total 0.
    auto consume = [&](int64_t rr, int i, bool ok, const SegInfo& si, const vec<IDT> (&x)[SLOTS],
                       const vec<IDT> (&y)[SLOTS]) {
        if (ok) {
            L v[SLOTS][V];
            L base[SLOTS];
            const int64_t u0 = (tile_of(rr) - si.first) * a.tile;
            const L wt = tile_values<IDT, OP, ZIP, SLOTS, REV, CMB>(x, y, alpha, v, base, mn, si, u0,
                                                                    tile_full<V, SLOTS>(si, u0));
            if (l == 0) s_wtot[i & 1][w] = wt;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            L tl = cmb_id<CMB, L>(mn);
            if (ok)
                for (int k = 0; k < WAVES; ++k) tl = cmb_op<CMB>(tl, s_wtot[i & 1][k], mn);
            const bool head = !ok || rr == stop_of<REV>(a, si, T);
            if (head) {
                run = cmb_id<CMB, C>(mn);
                seen = true;
            }
            uint64_t* rec = tws + rr * TW;
            rec[kRecCarry] = to_bits(run);
            rec[kRecHead] = seen ? 1u : 0u;
            run = cmb_op<CMB>(run, (C)tl, mn);
        }
    };
    if (r < r1) ha = issue(r, sa, xa, ya);
    for (int i = 0; r < r1; i += 2) {
        if (r + 1 < r1) hb = issue(r + 1, sb, xb, yb);
        consume(r, i, ha, sa, xa, ya);
        if (++r >= r1) break;
        if (r + 1 < r1) ha = issue(r + 1, sa, xa, ya);
        consume(r, i + 1, hb, sb, xb, yb);
        ++r;
    }
    if (threadIdx.x == 0) {
        uint64_t* c = cw + kChunkHdr + 4 * g;
        c[0] = seen ? 1u : 0u;
        c[1] = to_bits(run);
    }
}

// Segmented exclusive scan of the chunk pairs (has-head, sum) by one
// workgroup of kScanChunkThreads threads. The pair operator is
// (f1, s1) then (f2, s2) = (f1 | f2, f2 ? s2 : s1 + s2).
constexpr int kScanChunkThreads = 1024;

template <class C, int CMB>
__global__ __launch_bounds__(kScanChunkThreads) void k_scan_chunks(LaunchArgs a) {
    constexpr int N = kScanChunkThreads;
    __shared__ C s_v[2][N];
    __shared__ uint8_t s_f[2][N];
    uint64_t* cw = (uint64_t*)(a.ws + a.lay.off_chunk);
    const int64_t G = cw[1] < (uint64_t)kMaxChunks ? (int64_t)cw[1] : kMaxChunks;
    const int tid = threadIdx.x;
    const int64_t K = (G + N - 1) / N;   // chunks per thread (consecutive)
    const bool mn = (a.flags & kFlagMin) != 0;
    const C id = cmb_id<CMB, C>(mn);
    // serial inclusive pair of this thread's chunks
    bool f = false;
    C sv = id;
    for (int64_t j = 0; j < K; ++j) {
        const int64_t c = tid * K + j;
        if (c >= G) break;
        const uint64_t* cr = cw + kChunkHdr + 4 * c;
        const bool fc = cr[0] != 0;
        const C vc = from_bits<C>(cr[1]);
        sv = fc ? vc : cmb_op<CMB>(sv, vc, mn);
        f = f || fc;
    }
    // inclusive scan of the thread pairs (Hillis-Steele, double-buffered)
    int cur = 0;
    s_v[0][tid] = sv;
    s_f[0][tid] = f ? 1 : 0;
    __syncthreads();
    for (int d = 1; d < N; d <<= 1) {
        C v = s_v[cur][tid];
        uint8_t fl = s_f[cur][tid];
        if (tid >= d && !fl) {
            v = cmb_op<CMB>(s_v[cur][tid - d], v, mn);
            fl = s_f[cur][tid - d];
        }
        s_v[cur ^ 1][tid] = v;
        s_f[cur ^ 1][tid] = fl;
        cur ^= 1;
        __syncthreads();
    }
    // exclusive carry into this thread's first chunk, then serially on
    C cin = tid > 0 ? s_v[cur][tid - 1] : id;
    for (int64_t j = 0; j < K; ++j) {
        const int64_t c = tid * K + j;
        if (c >= G) break;
        uint64_t* cr = cw + kChunkHdr + 4 * c;
        cr[2] = to_bits(cin);
        const C vc = from_bits<C>(cr[1]);
        cin = cr[0] != 0 ? vc : cmb_op<CMB>(cin, vc, mn);
    }
}

template <int IDT, int ODT, int OP, bool C64, bool FUSED, int ROP, int RACC, int ITEMS, bool REV, int CMB>
__global__ __launch_bounds__(kBlock) void k_scan_apply(LaunchArgs a) {
    // int32 -> int64: 8-byte input vectors, so that each lane's outputs are
    // one 16-byte store and every store instruction of the wave covers
    // 1 KiB of consecutive memory (4-element vectors would write 32 bytes
    // per lane as two half-dense stores). The tile and its totals are the
    // same (integer sums are exact in any order).
    constexpr int V = (IDT == DR_I32 && ODT == DR_I64) ? 2 : vwidth<IDT>();
    constexpr int SLOTS = ITEMS / V;
    constexpr int WAVES = kBlock / 64;
    constexpr bool ZIP = zip_view<IDT, OP, FUSED, ROP>();
    using L = local_t<IDT>;
    using C = carry_t<IDT, C64>;
    __shared__ L s_wtot[WAVES];
    __shared__ float s_rs[WAVES], s_rc[WAVES];
    __shared__ double s_rd[WAVES];
    const uint32_t tag = FUSED ? begin_launch(a.ws) : 0u;
    TileMap tm;
    tm.init(a);
    if (!tm.ok) return;
    const int64_t T = tm.total_tiles;
    const int64_t r = blockIdx.x;
    if (r >= T) {
        if (FUSED && T == 0 && r == 0 && threadIdx.x == 0) {   // no tiles at all
            if (a.mode == DR_MODE_BATCH) write_all_init<double>(a);
            else write_result<double>(a, 0, 0.0);
        }
        return;
    }
    const int64_t t = REV ? T - 1 - r : r;
    SegInfo si;
    if (!tm.find(a, t, si)) return;   // malformed row (flagged)
    const int w = threadIdx.x >> 6, l = lane_id();
    // the tile's carry: its record plus (before the first head of the
    // chunk) the chunk's incoming carry
    const uint64_t* cw = (const uint64_t*)(a.ws + a.lay.off_chunk);
    const uint64_t* rec = (const uint64_t*)(a.ws + a.lay.off_tile) + r * a.lay.tile_words;
    const int64_t Q = (int64_t)cw[0];
    const uint64_t rc = rec[kRecCarry], rh = rec[kRecHead];
    const uint64_t ci = cw[kChunkHdr + 4 * (r / Q) + 2];

    const int64_t u0 = (t - si.first) * a.tile;
    const bool full = tile_full<V, SLOTS>(si, u0);
    vec<IDT, V> x[SLOTS], y[SLOTS];
    load_pair<ZIP, IDT, SLOTS, V>(x, y, si, u0, w, l, REV);
    float fws = 0.0f, fwc = 0.0f;
    double fwd = 0.0;
    if constexpr (FUSED) fused_wave<IDT, ROP, RACC, SLOTS>(x, y, fws, fwc, fwd);
    const bool mn = (a.flags & kFlagMin) != 0;
    L v[SLOTS][V];
    L base[SLOTS];
    const L run = tile_values<IDT, OP, ZIP, SLOTS, REV, CMB, V>(x, y, (L)a.alpha, v, base, mn, si, u0, full);
    if (l == 0) s_wtot[w] = run;
    if constexpr (FUSED) {
        if (l == 0) {
            s_rs[w] = fws;
            s_rc[w] = fwc;
            s_rd[w] = fwd;
        }
    }
    __syncthreads();
    L woff = cmb_id<CMB, L>(mn);
    for (int i = 0; i < w; ++i) woff = cmb_op<CMB>(woff, s_wtot[i], mn);
    C excl = rh ? from_bits<C>(rc) : cmb_op<CMB>(from_bits<C>(rc), from_bits<C>(ci), mn);
    if (a.flags & kFlagHasInit) excl = cmb_op<CMB>(init_carry<C, IDT>(a), excl, mn);
    tile_write<IDT, ODT, C64, SLOTS, REV, CMB, V>(v, base, excl, woff, si, u0, w, l, full,
                                               (a.flags & DR_SCAN_EXCLUSIVE) != 0, mn);
    if constexpr (FUSED) {
        if (threadIdx.x >= 64) return;   // wave 0 publishes the partial and combines
        double part = 0.0;
        if (l == 0) part = fused_block<IDT, RACC, WAVES>(s_rs, s_rc, s_rd);
        if (a.mode == DR_MODE_BATCH) combine_tile_batch<double>(a, tag, t, si, part);
        else combine_member<double>(a, tag, 0, 0, t, T, 0, part);
    }
}

// ---------------------------------------------------------------------------
// Single-pass form with specialised waves (on request: DR_TUNE_SPECIALIZED)
// ---------------------------------------------------------------------------
//
// One workgroup per CU, all resident (cooperative launch); workgroup 0 is
// the carry agent, workgroup 1 + g owns the processing indices g, g + G,
// g + 2G, ... (G = tile workgroups). Inside a tile workgroup:
//   waves 0-3  load a tile into registers, form its wave totals exactly as
//              the output pass will, and copy the raw tile into a ring of
//              LDS slots (they only ever load: their in-order memory counter
//              never waits behind a store, so two tiles stay in flight);
//   waves 4-7  take a tile from the ring with its carry, scan it in
//              registers and write it (they never wait for a load);
//   wave 8     publishes each tile's total (and, fused, its dot partial and
//              the combine) as soon as the loaders have it;
//   wave 9     fetches the carries of the next ring slots in one round trip.
// The agent's two waves past the scanning ones store the prefixes it
// computes (handed over in LDS), so that its polls never wait behind its
// own stores in the in-order memory counter.
// The agent scans the published tile totals in windows of kWsWindow tiles
// with a fixed shape (a serial pass over each thread's tiles, a wave scan,
// the waves in order, the window's carry in), so every carry is the same
// sum at every run, and publishes each tile's inclusive prefix; lanes past
// the first unpublished total never feed an earlier one, so a window's
// prefix can be published before the window is complete. Reads: the input
// once; writes: the output once.

constexpr int kWsWaves = 10;
constexpr int kWsThreads = 64 * kWsWaves;
constexpr int kWsAgentWaves = 8;
constexpr int kWsPerThread = 4;
constexpr int kWsWindow = kWsPerThread * 64 * kWsAgentWaves;
constexpr int kWsLdsBytes = 128 * 1024;   // ring budget per workgroup

__device__ __forceinline__ int lds_ld(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(int* p, int v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Bounded wait for an LDS counter; false (and the fault flag) on timeout.
__device__ __forceinline__ bool ws_wait(const int* p, int target, const LaunchArgs& a) {
    if (lds_ld(p) >= target) return true;
    Deadline dl(a.spin_ticks);
    while (lds_ld(p) < target) {
        if (dl.passed()) {
            if (lane_id() == 0) flag_error(a, DR_DEVFLAG_TIMEOUT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// A tile's published total: words kAggWord, kAggWord + 1 with the launch tag
// in the upper halves; the tag of the second word has its top bit flipped
// when the tile starts a range (the segmented scan restarts there).
constexpr uint32_t kHeadBit = 0x80000000u;

template <class C>
__device__ __forceinline__ void ws_publish(uint64_t* tw, uint32_t tag, bool head, C total) {
    const uint64_t v = to_bits(total);
    atomic_st(tw + kAggWord, ((uint64_t)tag << 32) | (uint32_t)v);
    atomic_st(tw + kAggWord + 1, ((uint64_t)(head ? tag ^ kHeadBit : tag) << 32) | (uint32_t)(v >> 32));
}

// The agent: inclusive prefixes of the (head, total) pairs in processing
// order, written to words kInclWord, kInclWord + 1 of every tile.
template <class C>
__device__ void ws_agent(const LaunchArgs& a, uint32_t tag, int64_t T) {
    __shared__ uint32_t s_zmin[kWsWaves];
    __shared__ C s_wt[kWsAgentWaves];
    __shared__ int s_wh[kWsAgentWaves];
    __shared__ C s_last;
    __shared__ int s_to;
    __shared__ C s_I[kWsWindow];   // prefixes handed to the storing waves
    constexpr int PT = kWsPerThread;
    uint64_t* tws = (uint64_t*)(a.ws + a.lay.off_tile);
    const int64_t TW = a.lay.tile_words;
    const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), l = lane_id();
    C carry = (C)0;
    for (int64_t base = 0; base < T; base += kWsWindow) {
        const int n = (int)(T - base < kWsWindow ? T - base : kWsWindow);
        bool have[PT], hd[PT];
        C v[PT];
#pragma unroll
        for (int j = 0; j < PT; ++j) {
            have[j] = false;
            hd[j] = false;
            v[j] = (C)0;
        }
        int pub = 0, nap = 1;
        Deadline dl(a.spin_ticks);
        while (true) {
            uint32_t fm = 0xffffffffu;   // first index of this thread not yet published
            if (w < kWsAgentWaves) {
                uint64_t q0[PT], q1[PT];
#pragma unroll
                for (int j = 0; j < PT; ++j) {
                    const int idx = PT * tid + j < n ? PT * tid + j : n - 1;
                    const uint64_t* p = tws + (base + idx) * TW + kAggWord;
                    q0[j] = atomic_ld(p);
                    q1[j] = atomic_ld(p + 1);
                }
#pragma unroll
                for (int j = 0; j < PT; ++j) {
                    const int idx = PT * tid + j;
                    const uint32_t t0 = (uint32_t)(q0[j] >> 32), t1 = (uint32_t)(q1[j] >> 32);
                    if (idx < n && !have[j] && t0 == tag && (t1 == tag || t1 == (tag ^ kHeadBit))) {
                        have[j] = true;
                        hd[j] = t1 != tag;
                        v[j] = from_bits<C>((uint64_t)(uint32_t)q0[j] | ((uint64_t)(uint32_t)q1[j] << 32));
                    }
                }
#pragma unroll
                for (int j = PT - 1; j >= 0; --j)
                    if (PT * tid + j < n && !have[j]) fm = (uint32_t)(PT * tid + j);
            }
            // the first missing index of the wave is that of its first lane
            // with one (lanes hold increasing indices)
            const uint64_t missing = __ballot(fm != 0xffffffffu);
            const uint32_t wm = missing ? (uint32_t)readlane((int)fm, __builtin_ctzll(missing)) : 0xffffffffu;
            if (l == 0) s_zmin[w] = wm;
            // fixed-shape segmented scan of the window; unpublished entries
            // are the identity and only ever feed later ones
            C run = (C)0;
            bool rh = false;
            C loc[PT];
            bool loch[PT];
#pragma unroll
            for (int j = 0; j < PT; ++j) {
                const bool hj = have[j] && hd[j];
                const C vj = have[j] ? v[j] : (C)0;
                run = hj ? vj : run + vj;
                rh = rh || hj;
                loc[j] = run;
                loch[j] = rh;
            }
            // segmented inclusive scan over the wave with DPP row shifts and
            // broadcasts (lanes without a source receive the identity (0, 0))
            C sv = run;
            int sh = rh ? 1 : 0;
            auto seg_step = [&](C pv, int ph) {
                if (!sh) sv = pv + sv;
                sh = sh | ph;
            };
            seg_step(dpp_move<DPP_ROW_SHR1, 0xf>(sv), dpp_move<DPP_ROW_SHR1, 0xf>(sh));
            seg_step(dpp_move<DPP_ROW_SHR2, 0xf>(sv), dpp_move<DPP_ROW_SHR2, 0xf>(sh));
            seg_step(dpp_move<DPP_ROW_SHR4, 0xf>(sv), dpp_move<DPP_ROW_SHR4, 0xf>(sh));
            seg_step(dpp_move<DPP_ROW_SHR8, 0xf>(sv), dpp_move<DPP_ROW_SHR8, 0xf>(sh));
            seg_step(dpp_move<DPP_ROW_BCAST15, 0xa>(sv), dpp_move<DPP_ROW_BCAST15, 0xa>(sh));
            seg_step(dpp_move<DPP_ROW_BCAST31, 0xc>(sv), dpp_move<DPP_ROW_BCAST31, 0xc>(sh));
            if (w < kWsAgentWaves && l == 63) {
                s_wt[w] = sv;
                s_wh[w] = sh;
            }
            C ev = __shfl_up(sv, 1, 64);
            int eh = __shfl_up(sh, 1, 64);
            if (l == 0) {
                ev = (C)0;
                eh = 0;
            }
            __syncthreads();
            uint32_t z = (uint32_t)n;
            for (int i = 0; i < kWsWaves; ++i) z = s_zmin[i] < z ? s_zmin[i] : z;
            C c = carry;
            for (int i = 0; i < w && i < kWsAgentWaves; ++i) c = s_wh[i] ? s_wt[i] : c + s_wt[i];
            c = eh ? ev : c + ev;
            if (w < kWsAgentWaves) {
#pragma unroll
                for (int j = 0; j < PT; ++j) {
                    const int idx = PT * tid + j;
                    const C I = loch[j] ? loc[j] : c + loc[j];
                    if (idx >= pub && idx < (int)z) s_I[idx] = I;
                    if (idx == n - 1 && (int)z == n) s_last = I;
                }
            }
            if (tid == 0) s_to = ((int)z < n && dl.passed()) ? 1 : 0;
            __syncthreads();
            // the waves past the scanning ones store the new prefixes: the
            // scanning waves only load, so no poll waits behind a store
            for (int idx = pub + tid - 64 * kWsAgentWaves; w >= kWsAgentWaves && idx < (int)z;
                 idx += 64 * (kWsWaves - kWsAgentWaves))
                tagged_store(tws + (base + idx) * TW + kInclWord, tag, to_bits(s_I[idx]));
            const bool progress = (int)z > pub;
            pub = (int)z;
            if ((int)z == n) {
                carry = s_last;
                break;
            }
            if (s_to) {
                if (tid == 0) flag_error(a, DR_DEVFLAG_TIMEOUT);
                return;
            }
            if (progress) {
                nap = 1;
                dl = Deadline(a.spin_ticks);
            } else {
                for (int i = 0; i < nap; ++i) __builtin_amdgcn_s_sleep(1);
                nap = nap < 4 ? 2 * nap : 4;
            }
            __syncthreads();   // s_zmin / s_wt are rewritten next round
        }
        __syncthreads();
    }
}

// Tiles of the specialised-wave form: 32 items per thread (binary64 16), so
// that every role of the one kernel fits in the registers of three waves
// per SIMD without spilling; fused, where the loaders hold both inputs, 16. Built for the identity view of each scan
// dtype pair but int32 -> int64.
template <int IDT, bool FUSED>
constexpr int ws_items() {
    return FUSED ? 16 : (IDT == DR_F64 ? 16 : 32);
}

template <int IDT, int ODT, int OP, bool FUSED, int ITEMS>
constexpr bool ws_form() {
    return OP == DR_OP_IDENTITY && ITEMS == ws_items<IDT, FUSED>() && !(IDT == DR_I32 && ODT == DR_I64) &&
           (!FUSED || IDT == DR_F32);
}

int ws_items_for(int in_dt, bool fused) {
    if (fused) return in_dt == DR_F32 ? 16 : 0;
    return in_dt == DR_F64 ? 16 : 32;
}

template <int IDT, int ITEMS>
constexpr int ws_ring() {
    constexpr int bytes = kBlock * ITEMS * esize<IDT>();
    constexpr int r = kWsLdsBytes / bytes;
    return r > 4 ? 4 : r;
}

template <int IDT, int ODT, int OP, bool C64, bool FUSED, int ROP, int RACC, int ITEMS, bool REV>
__global__ __launch_bounds__(kWsThreads) void k_scan_ws(LaunchArgs a) {
    constexpr int V = vwidth<IDT>();
    constexpr int SLOTS = ITEMS / V;
    constexpr int R = ws_ring<IDT, ITEMS>();
    static_assert(R >= 2, "the ring needs two slots");
    using L = local_t<IDT>;
    using C = carry_t<IDT, C64>;
    __shared__ vec<IDT> s_data[R][kBlock * SLOTS];
    __shared__ L s_wt[R][4];
    __shared__ float s_rs[R][4], s_rc[R][4];
    __shared__ double s_rd[R][4];
    __shared__ int s_ready[R], s_done[R], s_cseq[R];
    __shared__ C s_carry[R];

    const uint32_t tag = begin_launch(a.ws);
    TileMap tm;
    tm.init(a);
    if (!tm.ok) return;
    const int64_t T = tm.total_tiles;
    if (blockIdx.x == 0) {
        if (FUSED && T == 0 && threadIdx.x == 0) {   // no tiles at all
            if (a.mode == DR_MODE_BATCH) write_all_init<double>(a);
            else write_result<double>(a, 0, 0.0);
        }
        ws_agent<C>(a, tag, T);
        return;
    }
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int l = lane_id();
    const int64_t G = gridDim.x - 1;
    const int64_t g = blockIdx.x - 1;
    const int64_t K = g < T ? (T - 1 - g) / G + 1 : 0;   // tiles of this workgroup
    if (threadIdx.x < R) {
        s_ready[threadIdx.x] = 0;
        s_done[threadIdx.x] = 0;
        s_cseq[threadIdx.x] = 0;
    }
    __syncthreads();
    if (K == 0) return;
    uint64_t* tws = (uint64_t*)(a.ws + a.lay.off_tile);
    const int64_t TW = a.lay.tile_words;
    auto proc = [&](int64_t k) { return g + k * G; };                 // processing index
    auto phys = [&](int64_t r) { return REV ? T - 1 - r : r; };        // physical tile
    const L alpha = (L)a.alpha;

    if (w < 4) {
        // loaders: two tiles in flight in registers, then into the ring
        vec<IDT> xa[SLOTS], xb[SLOTS], ya[SLOTS], yb[SLOTS];
        SegInfo sa, sb;
        bool oka = false, okb = false;
        auto issue = [&](int64_t k, SegInfo& si, vec<IDT> (&x)[SLOTS], vec<IDT> (&y)[SLOTS]) -> bool {
            const int64_t r = proc(k < K ? k : K - 1);
            const int64_t t = phys(r);
            if (!tm.find(a, t, si)) return false;
            const int64_t u0 = (t - si.first) * a.tile;
            load_slots<IDT, SLOTS>(x, si.in0, si, u0, w, l, REV);
            if constexpr (FUSED) load_slots<IDT, SLOTS>(y, si.in1, si, u0, w, l, REV);
            return true;
        };
        auto stage = [&](int64_t k, bool ok, const SegInfo& si, const vec<IDT> (&x)[SLOTS],
                         const vec<IDT> (&y)[SLOTS]) -> bool {
            const int slot = (int)(k % R);
            const int fill = (int)(k / R);
            L run = (L)0;
            float prs = 0.0f, prc = 0.0f;
            double prd = 0.0;
            if (ok) {
                const int64_t u0 = (phys(proc(k)) - si.first) * a.tile;
                L v[SLOTS][V];
                L base[SLOTS];
                run = tile_values<IDT, OP, false, SLOTS, REV>(x, x, alpha, v, base, false, si, u0,
                                                              tile_full<V, SLOTS>(si, u0));
                if constexpr (FUSED) fused_wave<IDT, ROP, RACC, SLOTS>(x, y, prs, prc, prd);
            }
            if (!ws_wait(&s_done[slot], 5 * fill, a)) return false;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) s_data[slot][(w * SLOTS + s) * 64 + l] = x[s];
            if (l == 0) {
                s_wt[slot][w] = run;
                s_rs[slot][w] = prs;
                s_rc[slot][w] = prc;
                s_rd[slot][w] = prd;
                lds_add(&s_ready[slot], 1);
            }
            return true;
        };
        oka = issue(0, sa, xa, ya);
        okb = issue(1, sb, xb, yb);
        for (int64_t k = 0; k < K; k += 2) {
            if (!stage(k, oka, sa, xa, ya)) return;
            oka = issue(k + 2, sa, xa, ya);
            if (k + 1 >= K) break;
            if (!stage(k + 1, okb, sb, xb, yb)) return;
            okb = issue(k + 3, sb, xb, yb);
        }
        return;
    }
    if (w < 8) {
        // writers
        const int ww = w - 4;
        for (int64_t k = 0; k < K; ++k) {
            const int slot = (int)(k % R);
            const int fill = (int)(k / R) + 1;
            if (!ws_wait(&s_ready[slot], 4 * fill, a)) return;
            if (!ws_wait(&s_cseq[slot], fill, a)) return;
            vec<IDT> x[SLOTS];
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) x[s] = s_data[slot][(ww * SLOTS + s) * 64 + l];
            L woff = (L)0;
            for (int i = 0; i < ww; ++i) woff += s_wt[slot][i];
            const C cin = s_carry[slot];
            const int64_t r = proc(k);
            const int64_t t = phys(r);
            SegInfo si;
            const bool ok = tm.find(a, t, si);
            __builtin_amdgcn_s_waitcnt(0xc07f);   // every LDS read of the slot is done
            if (l == 0) lds_add(&s_done[slot], 1);
            if (!ok) continue;   // malformed row (flagged)
            const int64_t u0 = (t - si.first) * a.tile;
            const bool full = tile_full<V, SLOTS>(si, u0);
            L v[SLOTS][V];
            L base[SLOTS];
            (void)tile_values<IDT, OP, false, SLOTS, REV>(x, x, alpha, v, base, false, si, u0, full);
            C excl = r == stop_of<REV>(a, si, T) ? (C)0 : cin;
            if (a.flags & kFlagHasInit) excl = init_carry<C, IDT>(a) + excl;
            tile_write<IDT, ODT, C64, SLOTS, REV>(v, base, excl, woff, si, u0, ww, l, full,
                                                  (a.flags & DR_SCAN_EXCLUSIVE) != 0);
        }
        return;
    }
    if (w == 8) {
        // publisher: tile totals (and the fused partials) in order
        for (int64_t k = 0; k < K; ++k) {
            const int slot = (int)(k % R);
            const int fill = (int)(k / R) + 1;
            if (!ws_wait(&s_ready[slot], 4 * fill, a)) return;
            L tl = (L)0;
            for (int i = 0; i < 4; ++i) tl += s_wt[slot][i];
            double part = 0.0;
            if (l == 0) part = fused_block<IDT, RACC, 4>(s_rs[slot], s_rc[slot], s_rd[slot]);
            __builtin_amdgcn_s_waitcnt(0xc07f);
            if (l == 0) lds_add(&s_done[slot], 1);
            const int64_t r = proc(k);
            const int64_t t = phys(r);
            SegInfo si;
            const bool ok = tm.find(a, t, si);
            const bool head = !ok || r == stop_of<REV>(a, si, T);
            if (l == 0) ws_publish<C>(tws + r * TW, tag, head, ok ? (C)tl : (C)0);
            if constexpr (FUSED) {
                if (ok) {
                    if (a.mode == DR_MODE_BATCH) combine_tile_batch<double>(a, tag, t, si, part);
                    else combine_member<double>(a, tag, 0, 0, t, T, 0, part);
                }
            }
        }
        return;
    }
    // carry fetcher: lane j looks after entry kn + j (j < 2R). It fetches
    // the entry's carry as soon as the agent has published it (one round
    // trip for every lane) and keeps it in a register until the entry's ring
    // slot is free, so a freed slot gets its carry at once.
    constexpr int LA = 2 * R;
    int64_t kn = 0;
    bool got = false;
    C c = (C)0;
    int nap = 1;
    Deadline dl(a.spin_ticks);
    while (kn < K) {
        const int64_t k = kn + l;
        const bool mine = l < LA && k < K;
        if (mine && !got) {
            const int64_t r = proc(k);
            if (r == 0) {
                got = true;
            } else {
                uint64_t bits = 0;
                if (tagged_load(tws + (r - 1) * TW + kInclWord, tag, bits)) {
                    got = true;
                    c = from_bits<C>(bits);
                }
            }
        }
        const int slot = (int)(k % R);
        const int fill = (int)(k / R) + 1;
        const bool ready = mine && got && lds_ld(&s_done[slot]) >= 5 * (fill - 1);
        const uint64_t okm = __ballot(ready);
        const int m = (int)__builtin_ctzll(~okm);   // entries delivered, in order
        if (l < m) {
            s_carry[slot] = c;
            lds_st(&s_cseq[slot], fill);
        }
        if (m > 0) {
            // lane j takes over the state of lane j + m
            const int g2 = __shfl_down(got ? 1 : 0, m, 64);
            const C c2 = __shfl_down(c, m, 64);
            got = l + m < LA && g2 != 0;
            c = c2;
            kn += m;
            nap = 1;
            dl = Deadline(a.spin_ticks);
        } else {
            if (dl.passed()) {
                if (l == 0) flag_error(a, DR_DEVFLAG_TIMEOUT);
                return;
            }
            for (int i = 0; i < nap; ++i) __builtin_amdgcn_s_sleep(1);
            nap = nap < 4 ? 2 * nap : 4;
        }
    }
}

template <int IDT, int ODT, int OP, bool C64, bool FUSED, int ROP, int RACC, int ITEMS, bool REV>
hipError_t launch_scan_ws(const LaunchArgs& a, hipStream_t stream) {
    const void* fn = (const void*)k_scan_ws<IDT, ODT, OP, C64, FUSED, ROP, RACC, ITEMS, REV>;
    static const int resident = resident_grid(fn, kWsThreads);
    if (resident < 2) return hipErrorCooperativeLaunchTooLarge;
    LaunchArgs arg = a;
    void* args[] = {&arg};
    return hipLaunchCooperativeKernel(fn, dim3((uint32_t)resident), dim3(kWsThreads), args, 0, stream);
}

template <int IDT, int ODT, int OP, bool C64, bool FUSED, int ROP, int RACC, int ITEMS, bool REV, int CMB>
hipError_t launch_scan_dir(const LaunchArgs& a, int64_t grid, hipStream_t stream) {
    if constexpr (CMB == kCmbSum) {
        if (a.flags & kFlagTilePerBlock) {
            hipLaunchKernelGGL((k_scan<IDT, ODT, OP, C64, FUSED, ROP, RACC, ITEMS, REV>), dim3((uint32_t)grid),
                               dim3(kBlock), 0, stream, a);
            return hipGetLastError();
        }
    }
    using C = carry_t<IDT, C64>;
    static const int resident = resident_grid((const void*)k_scan_sums<IDT, OP, C64, ITEMS, REV, CMB>);
    int64_t g1 = resident < kMaxChunks ? resident : kMaxChunks;
    if (g1 > grid) g1 = grid;
    if (g1 < 1) g1 = 1;
    hipLaunchKernelGGL((k_scan_sums<IDT, OP, C64, ITEMS, REV, CMB>), dim3((uint32_t)g1), dim3(kBlock), 0, stream,
                       a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_scan_chunks<C, CMB>), dim3(1), dim3(kScanChunkThreads), 0, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_scan_apply<IDT, ODT, OP, C64, FUSED, ROP, RACC, ITEMS, REV, CMB>),
                       dim3((uint32_t)grid), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

template <int IDT, int ODT, int OP, bool C64, bool FUSED, int ROP, int RACC, int ITEMS, int CMB = kCmbSum>
hipError_t launch_scan(const LaunchArgs& a, int64_t grid, hipStream_t stream) {
    constexpr bool WS = CMB == kCmbSum && ws_form<IDT, ODT, OP, FUSED, ITEMS>();
    const bool ws = WS && (a.flags & kFlagSpecialized) != 0;
    // the prologue (epoch tag, zeroed counters) serves the single-pass forms
    // and the fused reduction's combine
    if (FUSED || ws || (CMB == kCmbSum && (a.flags & kFlagTilePerBlock))) {
        hipError_t e = launch_prologue(a, stream);
        if (e != hipSuccess) return e;
    }
    if constexpr (WS) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (ws && hipStreamIsCapturing(stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
            const hipError_t e = (a.flags & DR_SCAN_REVERSE)
                                     ? launch_scan_ws<IDT, ODT, OP, C64, FUSED, ROP, RACC, ITEMS, true>(a, stream)
                                     : launch_scan_ws<IDT, ODT, OP, C64, FUSED, ROP, RACC, ITEMS, false>(a, stream);
            if (e == hipSuccess) return e;
            (void)hipGetLastError();   // the grid cannot be held at once: the two passes instead
        }
    }
    if (a.flags & DR_SCAN_REVERSE)
        return launch_scan_dir<IDT, ODT, OP, C64, FUSED, ROP, RACC, ITEMS, true, CMB>(a, grid, stream);
    return launch_scan_dir<IDT, ODT, OP, C64, FUSED, ROP, RACC, ITEMS, false, CMB>(a, grid, stream);
}

#define DR_SCAN_OPS(IDT, ODT, C64, ITEMS)                                                           \
    if (in_dt == IDT && out_dt == ODT && carry64 == C64 && items == ITEMS) {                        \
        switch (op) {                                                                               \
        case DR_OP_IDENTITY: return launch_scan<IDT, ODT, DR_OP_IDENTITY, C64, false, 0, 0, ITEMS>; \
        case DR_OP_SQUARE: return launch_scan<IDT, ODT, DR_OP_SQUARE, C64, false, 0, 0, ITEMS>;     \
        case DR_OP_MUL: return launch_scan<IDT, ODT, DR_OP_MUL, C64, false, 0, 0, ITEMS>;           \
        case DR_OP_AXPY: return launch_scan<IDT, ODT, DR_OP_AXPY, C64, false, 0, 0, ITEMS>;         \
        default: return nullptr;                                                                    \
        }                                                                                           \
    }

#define DR_SCAN_ID(IDT, ODT, C64, ITEMS)                                                           \
    if (in_dt == IDT && out_dt == ODT && carry64 == C64 && items == ITEMS && op == DR_OP_IDENTITY) \
        return launch_scan<IDT, ODT, DR_OP_IDENTITY, C64, false, 0, 0, ITEMS>;

// Every op at 16 items per thread; the identity (plain scan) also at larger
// tiles, the shapes the tuner chooses from.
LaunchFn find_scan(int in_dt, int out_dt, int op, bool carry64, int items) {
    if (in_dt == DR_I32 || in_dt == DR_F64) carry64 = true;
    DR_SCAN_OPS(DR_I32, DR_I64, true, 16)
    DR_SCAN_ID(DR_I32, DR_I64, true, 32)
    DR_SCAN_ID(DR_I32, DR_I64, true, 64)
    DR_SCAN_OPS(DR_I32, DR_I32, true, 16)
    DR_SCAN_ID(DR_I32, DR_I32, true, 32)
    DR_SCAN_ID(DR_I32, DR_I32, true, 64)
    DR_SCAN_OPS(DR_F32, DR_F32, true, 16)
    DR_SCAN_ID(DR_F32, DR_F32, true, 32)
    DR_SCAN_ID(DR_F32, DR_F32, true, 64)
    DR_SCAN_OPS(DR_F32, DR_F32, false, 16)
    DR_SCAN_OPS(DR_BF16, DR_F32, true, 16)
    DR_SCAN_ID(DR_BF16, DR_F32, true, 32)
    DR_SCAN_ID(DR_BF16, DR_F32, true, 64)
    DR_SCAN_OPS(DR_F64, DR_F64, true, 16)
    DR_SCAN_ID(DR_F64, DR_F64, true, 32)
    return nullptr;
}

// max / min scans: the identity view, reduce-then-scan form, 16 items.
// binary32 / bfloat16 inputs keep binary32 carries: rounding is monotone, so
// the max (min) of binary32 values and a rounded init equals the rounding of
// the exact max (min) in binary64.
LaunchFn find_scan_minmax(int in_dt, int out_dt) {
    if (in_dt == DR_I32 && out_dt == DR_I64)
        return launch_scan<DR_I32, DR_I64, DR_OP_IDENTITY, true, false, 0, 0, 16, kCmbMinMax>;
    if (in_dt == DR_I32 && out_dt == DR_I32)
        return launch_scan<DR_I32, DR_I32, DR_OP_IDENTITY, true, false, 0, 0, 16, kCmbMinMax>;
    if (in_dt == DR_F32 && out_dt == DR_F32)
        return launch_scan<DR_F32, DR_F32, DR_OP_IDENTITY, false, false, 0, 0, 16, kCmbMinMax>;
    if (in_dt == DR_BF16 && out_dt == DR_F32)
        return launch_scan<DR_BF16, DR_F32, DR_OP_IDENTITY, false, false, 0, 0, 16, kCmbMinMax>;
    if (in_dt == DR_F64 && out_dt == DR_F64)
        return launch_scan<DR_F64, DR_F64, DR_OP_IDENTITY, true, false, 0, 0, 16, kCmbMinMax>;
    return nullptr;
}

#define DR_FUSED(ITEMS)                                                                                  \
    if (items == ITEMS) {                                                                                \
        if (acc == DR_ACC_COMPENSATED)                                                                   \
            return launch_scan<DR_F32, DR_F32, DR_OP_IDENTITY, true, true, DR_OP_MUL, DR_ACC_COMPENSATED, \
                               ITEMS>;                                                                   \
        return launch_scan<DR_F32, DR_F32, DR_OP_IDENTITY, true, true, DR_OP_MUL, DR_ACC_PLAIN, ITEMS>;   \
    }

LaunchFn find_scan_reduce(int in_dt, int reduce_op, int acc, int items) {
    if (reduce_op != DR_OP_MUL) return nullptr;
    if (in_dt == DR_F64)
        return items == 16 ? launch_scan<DR_F64, DR_F64, DR_OP_IDENTITY, true, true, DR_OP_MUL, DR_ACC_PLAIN, 16>
                           : nullptr;
    if (in_dt != DR_F32) return nullptr;
    DR_FUSED(16)
    DR_FUSED(32)
    DR_FUSED(64)
    return nullptr;
}

}  // namespace dr
