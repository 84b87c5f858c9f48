// k_scan_chain.hip — the chained single pass (DR_TUNE_CHAINED): the sum
// scan of one long range (CONCAT) that reads the input from HBM once
// (section 4.3, "inclusive_scan"; the carries are the segmented scan's
// offsets, here chained across the whole range).
//
// The two-pass form reads the input twice because a tile's carry is not
// known when the tile is read: its second pass starts when the first has
// ended. Here a workgroup reads each chunk the second time one chunk after
// the first, when the carries before it are known: it takes chunks of P
// consecutive tiles (processing order) from a counter and runs each chunk
// in two phases, one chunk apart:
//   phase A  reads the chunk with plain loads (so that the lines may stay in
//            the caches for the re-read), forms each tile's total
//            (chain_tile_sum) and publishes the chunk's
//            total; the last chunk of a superblock of kChainSB chunks to
//            arrive (an arrival counter) sums the superblock's totals and
//            publishes the running carry at its end,
//            E(sb) = E(sb - 1) + that sum;
//   phase B  runs after the workgroup's next chunk has been through phase
//            A: the chunk's carry is E(sb - 1) plus the sum of the totals
//            of the chunks before it in its superblock; the chunk is read
//            again (non-temporal: the last use), each tile scanned in
//            registers, its carry added, and written once.
// (At 2 workgroups per CU the re-read mostly misses the XCD's 4 MiB L2:
// the counters see the input fetched twice. Holding the chunk in LDS
// between the phases instead, which removes that traffic, measured no
// faster: the pass is bound by what each workgroup keeps in flight.)
// Every sum of published totals runs over a fixed shape (one total per
// thread, absent ones 0, a DPP wave sum, the waves in order), so results
// repeat exactly and do not depend on timing or on the grid. A workgroup
// waits only for chunks claimed before its own: their workgroups were
// running when they claimed them and publish a chunk's total before they
// wait for anything, so every wait ends without co-residency; every wait
// is also bounded (fault bit 2).
//
// Every index the kernel forms is checked against the table, the tiles and
// the workspace before it is used: an inconsistency sets a fault bit and
// skips the work instead of touching memory out of range.
//
// Built for sums of the identity view: binary32 -> binary32 (binary64 or
// binary32 carries) and int32 -> int64 / int32, 16 items per thread, chunks
// of 4 tiles (64 KiB of input), forward and reverse, with the initial value
// and the exclusive form of dr_scan.
#include "k_scan_core.hpp"

namespace dr {

namespace {

constexpr int kChainP = 4;            // tiles per chunk
constexpr int kChainItems = 16;       // items per thread
constexpr int kChainWaves = kBlock / 64;

// Bounded wait for a tagged 64-bit word (thread-local); false and the fault
// flag on timeout.
__device__ __forceinline__ bool chain_wait(const LaunchArgs& a, const uint64_t* w, uint32_t tag, uint64_t& bits) {
    if (tagged_load(w, tag, bits)) return true;
    Deadline dl(a.spin_ticks);
    while (!tagged_load(w, tag, bits)) {
        if (dl.passed()) {
            flag_error(a, DR_DEVFLAG_TIMEOUT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// Sum of the published chunk totals j0 .. lim - 1 (lim - j0 <= kChainSB)
// and of the running carry `*e` (when e is not null) over a fixed shape:
// total j0 + i in thread i, the carry in thread kChainSB (0 in every other
// thread), a DPP wave sum, the waves in order. Every thread waits for its
// own term, so all the round trips overlap. Whole workgroup; the result is
// in every thread. A term not published in time counts as 0 (fault bit 2).
template <class C>
__device__ __forceinline__ C chain_sum(const LaunchArgs& a, uint32_t tag, const uint64_t* tws, int64_t TW,
                                       int64_t j0, int64_t lim, const uint64_t* e, C* s_w) {
    const int tid = threadIdx.x, w = tid >> 6, l = lane_id();
    const int64_t j = j0 + tid;
    C mine = (C)0;
    const uint64_t* src = tid < kChainSB    ? (j < lim ? tws + j * TW + kAggWord : nullptr)
                          : tid == kChainSB ? e
                                            : nullptr;
    if (src) {
        uint64_t bits = 0;
        if (chain_wait(a, src, tag, bits)) mine = from_bits<C>(bits);
    }
    const C ws = wave_sum(mine);
    if (l == 0) s_w[w] = ws;
    __syncthreads();
    C f = s_w[0];
    for (int i = 1; i < kChainWaves; ++i) f = f + s_w[i];
    __syncthreads();   // s_w is rewritten by the next sum
    return f;
}

// Segment of physical tile t, checked: the tile must lie in the segment the
// lookup returns (a table or plan inconsistency sets fault bit 1 and the
// tile is skipped).
__device__ __forceinline__ bool chain_find(const LaunchArgs& a, const TileMap& tm, int64_t t, SegInfo& si) {
    if (!tm.find(a, t, si)) return false;
    if (t < si.first || t >= si.first + si.ntiles || si.ntiles <= 0) {
        if (threadIdx.x == 0) flag_error(a, DR_DEVFLAG_BAD_TABLE);
        return false;
    }
    return true;
}

// The segment of a whole chunk: when the P tiles from processing index r0
// (or the tiles up to the last one) all lie in one segment, one lookup
// serves them (`one`); otherwise each tile is looked up on its own.
__device__ __forceinline__ bool chain_segment(const LaunchArgs& a, const TileMap& tm, int64_t T, int64_t r0,
                                              int P, bool rev, SegInfo& si) {
    const int64_t rl = (r0 + P < T ? r0 + P : T) - 1;
    const int64_t t0 = rev ? T - 1 - r0 : r0, tl = rev ? T - 1 - rl : rl;
    if (!chain_find(a, tm, t0, si)) return false;
    return tl >= si.first && tl < si.first + si.ntiles;
}

// The loads of a chunk whose P tiles lie in the segment `si` and are all
// full (whole inside it, rows aligned): unchecked, back to back; plain loads
// in phase A (the lines may stay cached for the re-read), non-temporal ones
// (NT) for phase B's re-read. Returns false, loading nothing, when a tile is not full (the
// caller then takes the tiles one by one, checked).
template <int IDT, int V, int SLOTS, bool REV, bool NT = false, int P>
__device__ __forceinline__ bool chain_load_full(const LaunchArgs& a, const SegInfo& si, int64_t T, int64_t r0,
                                                vec<IDT, V> (&x)[P][SLOTS], int w, int l) {
    using R = typename vbits<V * esize<IDT>()>::T;
    constexpr int64_t NV = (int64_t)kBlock * SLOTS;
    if (r0 + P > T) return false;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int64_t t = REV ? T - 1 - (r0 + p) : r0 + p;
        if (!tile_full<V, SLOTS>(si, (t - si.first) * a.tile)) return false;
    }
    const int64_t p0 = (int64_t)(w * SLOTS) * 64 + l;
    const int64_t q0 = REV ? (NV - 1 - p0) : p0;
    const int64_t step = REV ? -64 * (int64_t)sizeof(R) : 64 * (int64_t)sizeof(R);
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int64_t t = REV ? T - 1 - (r0 + p) : r0 + p;
        const char* b = (const char*)si.in0 + ((t - si.first) * a.tile - si.shift + q0 * V) * esize<IDT>();
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const R wv = NT ? __builtin_nontemporal_load((const R*)(b + s * step)) : *(const R*)(b + s * step);
            __builtin_memcpy(&x[p][s], &wv, sizeof(R));
        }
    }
    return true;
}

// Whether the P tiles of the chunk from processing index r0 all exist and
// are full tiles of the segment `si` (which the caller found holds them).
template <int V, int SLOTS, bool REV, int P>
__device__ __forceinline__ bool chain_chunk_full(const LaunchArgs& a, const SegInfo& si, int64_t T, int64_t r0) {
    if (r0 + P > T) return false;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int64_t t = REV ? T - 1 - (r0 + p) : r0 + p;
        if (!tile_full<V, SLOTS>(si, (t - si.first) * a.tile)) return false;
    }
    return true;
}

// Phase B's re-read of one full tile (processing index r) of segment `si`:
// unchecked non-temporal loads (the last use of the lines).
template <int IDT, int V, int SLOTS, bool REV>
__device__ __forceinline__ void chain_load_tile(const LaunchArgs& a, const SegInfo& si, int64_t T, int64_t r,
                                                vec<IDT, V> (&x)[SLOTS], int w, int l) {
    using R = typename vbits<V * esize<IDT>()>::T;
    constexpr int64_t NV = (int64_t)kBlock * SLOTS;
    const int64_t p0 = (int64_t)(w * SLOTS) * 64 + l;
    const int64_t q0 = REV ? (NV - 1 - p0) : p0;
    const int64_t step = REV ? -64 * (int64_t)sizeof(R) : 64 * (int64_t)sizeof(R);
    const int64_t t = REV ? T - 1 - r : r;
    const char* b = (const char*)si.in0 + ((t - si.first) * a.tile - si.shift + q0 * V) * esize<IDT>();
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const R wv = __builtin_nontemporal_load((const R*)(b + s * step));
        __builtin_memcpy(&x[s], &wv, sizeof(R));
    }
}

// A tile's total for the chunk totals (phase A): each thread sums each of
// its vectors serially and the vector sums pairwise, then a DPP wave sum;
// the caller adds the waves in order. A fixed order, so totals repeat
// exactly. It is not the order of phase B's in-tile scan (the two differ by
// rounding only; integer sums are exact), and it is no deeper: (V - 1) +
// log2(SLOTS) + 6 + 3 binary32 roundings per element at most, against the
// in-tile scan's (V - 1) + 6 + SLOTS + 4 + 2.
template <int IDT, int V, int SLOTS>
__device__ __forceinline__ local_t<IDT> chain_tile_sum(const vec<IDT, V> (&x)[SLOTS]) {
    using L = local_t<IDT>;
    L st[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        L t = (L)decode<IDT>(x[s].e[0]);
#pragma unroll
        for (int e = 1; e < V; ++e) t += (L)decode<IDT>(x[s].e[e]);
        st[s] = t;
    }
#pragma unroll
    for (int h = 1; h < SLOTS; h *= 2)
#pragma unroll
        for (int s = 0; s + h < SLOTS; s += 2 * h) st[s] += st[s + h];
    return wave_sum(st[0]);
}

template <int IDT, int ODT, bool C64, bool REV>
struct Chain {
    // phase B: int32 -> int64 reads 8-byte vectors, so that each lane's
    // outputs are one 16-byte store; phase A only sums, in any layout, so it
    // always reads whole 16-byte vectors (the same lines)
    static constexpr int V = (IDT == DR_I32 && ODT == DR_I64) ? 2 : vwidth<IDT>();
    static constexpr int SLOTS = kChainItems / V;
    static constexpr int VA = vwidth<IDT>();
    static constexpr int SLOTS_A = kChainItems / VA;
    using L = local_t<IDT>;
    using C = carry_t<IDT, C64>;
    using X = vec<IDT, V>;
    using XA = vec<IDT, VA>;
};

}  // namespace

template <int IDT, int ODT, bool C64, bool REV>
__global__ __launch_bounds__(kBlock) void k_scan_chain(LaunchArgs a) {
    using K = Chain<IDT, ODT, C64, REV>;
    constexpr int V = K::V, SLOTS = K::SLOTS, P = kChainP;
    using L = typename K::L;
    using C = typename K::C;
    using X = typename K::X;
    using XA = typename K::XA;
    constexpr int VA = K::VA, SLOTS_A = K::SLOTS_A;
    __shared__ L s_wt[P * kChainWaves];
    __shared__ C s_tot[2][P];
    __shared__ C s_w[kChainWaves];
    __shared__ int s_claim, s_last;

    const uint32_t tag = begin_launch(a.ws);
    TileMap tm;
    tm.init(a);
    if (!tm.ok) return;
    const int64_t T = tm.total_tiles;
    const int64_t NC = (T + P - 1) / P;
    const int64_t NSB = (NC + kChainSB - 1) / kChainSB;
    // the workspace holds a chunk word per chunk (at most tmax) and a
    // counter and a carry per superblock
    if (a.mode != DR_MODE_CONCAT || NC > a.tmax || (uint64_t)NSB + 2 > a.lay.npipe) {
        if (blockIdx.x == 0 && threadIdx.x == 0) flag_error(a, DR_DEVFLAG_BAD_TABLE);
        return;
    }
    const int64_t TW = a.lay.tile_words;
    uint64_t* tws = (uint64_t*)(a.ws + a.lay.off_tile);
    uint32_t* pc = (uint32_t*)(a.ws + a.lay.off_pipe);
    uint64_t* ew = (uint64_t*)(a.ws + a.lay.off_pipe_e);
    const int w = threadIdx.x >> 6, l = lane_id();
    const bool exc = (a.flags & DR_SCAN_EXCLUSIVE) != 0;
    const C init = (a.flags & kFlagHasInit) ? init_carry<C, IDT>(a) : (C)0;

    int buf = 0;
    int64_t cur = -1;
    if (threadIdx.x == 0) s_claim = (int)atomic_add32(pc, 1u);
    __syncthreads();
    int64_t nxt = s_claim;
    __syncthreads();
    // one chunk per iteration: phase A of the chunk claimed last, then phase
    // B of the one before it. The next claim is issued at the top of the
    // iteration and read at its end, so the counter's round trip overlaps
    // the chunk's work. Holding a claimed chunk while waiting cannot stall
    // the grid: a workgroup waits only for chunks below the one it is
    // finishing, and the chunk it holds is above that one, so every chain of
    // waits runs to ever lower chunks and ends.
    while (true) {
        uint32_t ahead = 0;
        if (threadIdx.x == 0 && nxt < NC) ahead = atomic_add32(pc, 1u);

        if (nxt < NC) {
            // ---- phase A of chunk nxt into buffer buf ^ 1 ----
            const int b = buf ^ 1;
            const int64_t r0 = nxt * P;
            XA x[P][SLOTS_A];
            SegInfo sc;
            if (chain_segment(a, tm, T, r0, P, REV, sc) &&
                chain_load_full<IDT, VA, SLOTS_A, REV>(a, sc, T, r0, x, w, l)) {
                // the common case: every tile full, all loads already issued
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const L wt = chain_tile_sum<IDT, VA, SLOTS_A>(x[p]);
                    if (l == 0) s_wt[p * kChainWaves + w] = wt;
                }
                __syncthreads();
                if (threadIdx.x < P) {
                    L tl = (L)0;
                    for (int i = 0; i < kChainWaves; ++i) tl += s_wt[threadIdx.x * kChainWaves + i];
                    s_tot[b][threadIdx.x] = (C)tl;
                }
                __syncthreads();
            } else {
                // a chunk with a segment edge (or past the last tile): tile
                // by tile, checked
                for (int p = 0; p < P; ++p) {
                    const int64_t r = r0 + p;
                    SegInfo si;
                    const bool ok = r < T && chain_find(a, tm, REV ? T - 1 - r : r, si);   // uniform
                    if (ok) {
                        const int64_t u0 = ((REV ? T - 1 - r : r) - si.first) * a.tile;
                        XA xc[SLOTS_A];
                        load_slots<IDT, SLOTS_A, VA, false>(xc, si.in0, si, u0, w, l, REV);
                        const L wt = chain_tile_sum<IDT, VA, SLOTS_A>(xc);   // elements outside read as 0
                        if (l == 0) s_wt[w] = wt;
                    }
                    __syncthreads();
                    if (threadIdx.x == 0) {
                        L tl = (L)0;
                        if (ok)
                            for (int i = 0; i < kChainWaves; ++i) tl += s_wt[i];
                        s_tot[b][p] = (C)tl;
                    }
                    __syncthreads();
                }
            }
            const int64_t sbk = nxt / kChainSB, c0 = sbk * kChainSB;
            const int64_t nsb = NC - c0 < kChainSB ? NC - c0 : kChainSB;
            if (threadIdx.x == 0) {
                C f = s_tot[b][0];
                for (int p = 1; p < P; ++p) f = f + s_tot[b][p];
                tagged_store(tws + nxt * TW + kAggWord, tag, to_bits(f));
                s_last = atomic_add32(pc + 1 + sbk, 1u) == (uint32_t)(nsb - 1);
            }
            __syncthreads();
            if (s_last) {
                // the superblock's last arrival publishes the running carry
                // at its end: E(sb - 1) + the sum of its chunk totals
                const C e = chain_sum<C>(a, tag, tws, TW, c0, c0 + nsb, sbk > 0 ? ew + 2 * (sbk - 1) : nullptr, s_w);
                if (threadIdx.x == 0) tagged_store(ew + 2 * sbk, tag, to_bits(e));
            }
        }

        if (cur >= 0) {
            // ---- phase B of chunk cur from buffer buf ----
            const int64_t r0b = cur * P;
            const int64_t sbk = cur / kChainSB, c0 = sbk * kChainSB;
            SegInfo sc;
            const bool one = chain_segment(a, tm, T, r0b, P, REV, sc);   // uniform
            if (one && chain_chunk_full<V, SLOTS, REV, P>(a, sc, T, r0b)) {
                // the common case, pipelined: each tile's re-read is issued
                // before the previous tile's stores (loads and stores share
                // one in-order counter, so a load issued after a store would
                // wait for the store), and the first one before the carry
                // wait
                X xb[2][SLOTS];
                chain_load_tile<IDT, V, SLOTS, REV>(a, sc, T, r0b, xb[0], w, l);
                C run = chain_sum<C>(a, tag, tws, TW, c0, cur, sbk > 0 ? ew + 2 * (sbk - 1) : nullptr, s_w);
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    if (p + 1 < P) chain_load_tile<IDT, V, SLOTS, REV>(a, sc, T, r0b + p + 1, xb[(p + 1) & 1], w, l);
                    const C excl = run;
                    run = run + s_tot[buf][p];
                    const int64_t t = REV ? T - 1 - (r0b + p) : r0b + p;
                    const int64_t u0 = (t - sc.first) * a.tile;
                    L v[SLOTS][V];
                    L base[SLOTS];
                    const L wt = tile_values<IDT, DR_OP_IDENTITY, false, SLOTS, REV, kCmbSum, V>(
                        xb[p & 1], xb[p & 1], (L)0, v, base, false, sc, u0, true);
                    if (l == 0) s_wt[w] = wt;
                    __syncthreads();
                    L woff = (L)0;
                    for (int i = 0; i < w; ++i) woff += s_wt[i];
                    tile_write<IDT, ODT, C64, SLOTS, REV, kCmbSum, V>(v, base, init + excl, woff, sc, u0, w, l, true,
                                                                      exc);
                    __syncthreads();   // s_wt is rewritten by the next tile
                }
            } else {
            C run = chain_sum<C>(a, tag, tws, TW, c0, cur, sbk > 0 ? ew + 2 * (sbk - 1) : nullptr, s_w);
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const C excl = run;
                run = run + s_tot[buf][p];
                const int64_t r = r0b + p;
                SegInfo si = sc;
                if (r >= T || (!one && !chain_find(a, tm, REV ? T - 1 - r : r, si))) continue;   // uniform
                const int64_t t = REV ? T - 1 - r : r;
                const int64_t u0 = (t - si.first) * a.tile;
                const bool full = tile_full<V, SLOTS>(si, u0);
                // the second and last read: non-temporal, so the lines
                // leave room for the chunks still to be re-read
                X xb[SLOTS];
                load_slots<IDT, SLOTS, V, true>(xb, si.in0, si, u0, w, l, REV);
                L v[SLOTS][V];
                L base[SLOTS];
                const L wt = tile_values<IDT, DR_OP_IDENTITY, false, SLOTS, REV, kCmbSum, V>(xb, xb, (L)0, v, base,
                                                                                           false, si, u0, full);
                if (l == 0) s_wt[w] = wt;
                __syncthreads();
                L woff = (L)0;
                for (int i = 0; i < w; ++i) woff += s_wt[i];
                tile_write<IDT, ODT, C64, SLOTS, REV, kCmbSum, V>(v, base, init + excl, woff, si, u0, w, l, full,
                                                                  exc);
                __syncthreads();   // s_wt is rewritten by the next tile
            }
            }
        }
        if (nxt >= NC) break;
        if (threadIdx.x == 0) s_claim = (int)ahead;
        __syncthreads();
        cur = nxt;
        nxt = s_claim;
        __syncthreads();
        buf ^= 1;
    }
}

namespace {

template <int IDT, int ODT, bool C64>
hipError_t launch_scan_chain(const LaunchArgs& a, int64_t, hipStream_t stream) {
    if (!(a.flags & kFlagChained)) return hipErrorNotSupported;
    hipError_t e = launch_prologue(a, stream);
    if (e != hipSuccess) return e;
    // two workgroups per CU: the registers allow no more (187-238 VGPRs),
    // and fewer measured slower
    static const int per_dev = [] {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 1;
        return 2 * cus;
    }();
    const int64_t chunks = (a.tmax + kChainP - 1) / kChainP;
    const int64_t g = chunks < per_dev ? (chunks < 1 ? 1 : chunks) : per_dev;
    if (a.flags & DR_SCAN_REVERSE)
        hipLaunchKernelGGL((k_scan_chain<IDT, ODT, C64, true>), dim3((uint32_t)g), dim3(kBlock), 0, stream, a);
    else
        hipLaunchKernelGGL((k_scan_chain<IDT, ODT, C64, false>), dim3((uint32_t)g), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

}  // namespace

LaunchFn find_scan_chain(int in_dt, int out_dt, int op, bool carry64, int items) {
    if (op != DR_OP_IDENTITY || items != kChainItems) return nullptr;
    if (in_dt == DR_F32 && out_dt == DR_F32)
        return carry64 ? launch_scan_chain<DR_F32, DR_F32, true> : launch_scan_chain<DR_F32, DR_F32, false>;
    if (in_dt == DR_I32 && out_dt == DR_I64) return launch_scan_chain<DR_I32, DR_I64, true>;
    if (in_dt == DR_I32 && out_dt == DR_I32) return launch_scan_chain<DR_I32, DR_I32, true>;
    return nullptr;
}

}  // namespace dr
