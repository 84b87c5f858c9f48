// k_scan.hip — single-pass inclusive_scan over a zip/transform view of a
// segmented range (section 4.3, "inclusive_scan"; Algorithm 4), and its
// fusion with a transform_reduce over the same rows.
//
// The paper scans each segment locally, scans the segment totals, then adds
// each segment's offset in a second pass over the data (the extra pass it
// blames for the scan's drop from one to two tiles, section 5.1). Here the
// offsets never take a second pass: one workgroup per tile, in block-index
// order, scans its elements in registers, publishes its aggregate, and wave
// 0 looks back over its predecessors' published
// aggregates / inclusive prefixes (Merrill & Garland, "Single-pass Parallel
// Prefix Scan with Decoupled Look-back", 2016) to get the tile's exclusive
// carry. The look-back runs across segment boundaries in CONCAT mode (the
// carry of segment k is the total of segments before it) and stops at the
// segment's first tile in BATCH mode. Results are written once.
//
// Precision: int32 inputs scan in int64 (exact). binary32 / bfloat16
// inputs scan in binary32 inside a tile; the carries between tiles are
// binary64 (or binary32 with DR_SCAN_CARRY_F32), and each output is the
// binary64 sum of the carry and the tile-local prefix rounded once to
// binary32. binary64 inputs scan in binary64.
//
// Reverse mode (suffix sums, the adjoint of the scan) processes tiles in
// reverse physical order and mirrors the element order inside each tile.
#include "dr_combine.hpp"

namespace dr {

template <int IDT> using local_t =
    typename std::conditional<IDT == DR_I32, int64_t,
                              typename std::conditional<IDT == DR_F64, double, float>::type>::type;

template <int IDT, bool C64> using carry_t =
    typename std::conditional<IDT == DR_I32, int64_t,
                              typename std::conditional<(IDT == DR_F64 || C64), double, float>::type>::type;

// Tile status words (64-bit): [0,1] aggregate, [2,3] inclusive prefix,
// [4,5] reduce partial (fused kernel only).
constexpr int kAggWord = 0;
constexpr int kInclWord = 2;

template <class T>
__device__ __forceinline__ T shfl_up1(T v) {
    // lane l gets lane l-1's value, lane 0 gets 0
    T u = __shfl_up(v, 1, 64);
    return lane_id() == 0 ? (T)0 : u;
}

// Exclusive carry of the tile at processing index r: the sum of the
// aggregates of tiles r-1, r-2, ... down to the nearest tile whose
// inclusive prefix is published (which is then added), or down to `stop`.
// The whole workgroup looks back at once: thread i examines predecessor
// hi - i, so one round trip to memory covers 256 predecessors. Tiles start
// so fast (hundreds per microsecond at full bandwidth) that the nearest
// published inclusive prefix is often hundreds of tiles back; a 64-wide
// window would need several round trips. Returns the carry in every thread.
template <class C>
__device__ __forceinline__ C look_back(const LaunchArgs& a, uint32_t tag, int64_t r, int64_t stop) {
    constexpr int WAVES = kBlock / 64;
    __shared__ uint64_t s_incl_m[WAVES], s_have_m[WAVES];
    __shared__ C s_part[WAVES];
    __shared__ int s_timeout;
    const uint64_t* tw = (const uint64_t*)(a.ws + a.lay.off_tile);
    const int64_t TW = a.lay.tile_words;
    const int tid = threadIdx.x, w = tid >> 6, l = lane_id();
    C acc = (C)0;
    int64_t hi = r - 1;
    Deadline dl(a.spin_ticks);
    while (true) {
        // 1. one thread waits, with growing back-off, until the nearest
        //    unconsumed predecessor has published something: polling with
        //    the whole workgroup would add memory traffic that queues
        //    behind the stream the scan itself is moving
        if (tid == 0) {
            int t_out = 0;
            if (hi >= stop) {
                const uint64_t* wp = tw + hi * TW;
                int nap = 1;
                while (true) {
                    const uint64_t a1 = atomic_ld(wp + kAggWord + 1), i1 = atomic_ld(wp + kInclWord + 1);
                    if ((uint32_t)(a1 >> 32) == tag || (uint32_t)(i1 >> 32) == tag) break;
                    if (dl.passed()) {
                        t_out = 1;
                        break;
                    }
                    for (int i = 0; i < nap; ++i) __builtin_amdgcn_s_sleep(2);
                    nap = nap < 16 ? 2 * nap : 16;
                }
            }
            s_timeout = t_out;
        }
        __syncthreads();
        if (s_timeout) {
            if (tid == 0) flag_error(a.ws, DR_DEVFLAG_TIMEOUT);
            break;
        }
        // 2. one read of the statuses of up to 256 predecessors
        const int64_t p = hi - tid;
        const bool inr = p >= stop;
        uint64_t ib = 0, ab = 0;
        bool iok = false, aok = false;
        if (inr) {
            const uint64_t* wp = tw + p * TW;
            const uint64_t a0 = atomic_ld(wp + kAggWord), a1 = atomic_ld(wp + kAggWord + 1);
            const uint64_t i0 = atomic_ld(wp + kInclWord), i1 = atomic_ld(wp + kInclWord + 1);
            iok = (uint32_t)(i0 >> 32) == tag && (uint32_t)(i1 >> 32) == tag;
            aok = (uint32_t)(a0 >> 32) == tag && (uint32_t)(a1 >> 32) == tag;
            ib = (uint64_t)(uint32_t)i0 | ((uint64_t)(uint32_t)i1 << 32);
            ab = (uint64_t)(uint32_t)a0 | ((uint64_t)(uint32_t)a1 << 32);
        }
        const uint64_t im = __ballot(!inr || iok);
        const uint64_t hm = __ballot(!inr || iok || aok);
        if (l == 0) {
            s_incl_m[w] = im;
            s_have_m[w] = hm;
        }
        __syncthreads();
        // f: first thread whose predecessor has an inclusive prefix (or lies
        // before the range start); z: first thread whose predecessor has
        // published nothing. The same in every thread.
        int f = kBlock, z = kBlock;
        for (int i = WAVES - 1; i >= 0; --i) {
            if (s_incl_m[i]) f = 64 * i + __builtin_ctzll(s_incl_m[i]);
            if (~s_have_m[i]) z = 64 * i + __builtin_ctzll(~s_have_m[i]);
        }
        C v = (C)0;
        int consumed;
        bool done = false;
        if (f <= z) {
            if (tid < f) v = from_bits<C>(ab);
            else if (tid == f && inr) v = from_bits<C>(ib);
            consumed = kBlock;
            done = f < kBlock;
        } else {
            if (tid < z) v = from_bits<C>(ab);
            consumed = z;
        }
        const C wsum = wave_sum(v);
        if (l == 0) s_part[w] = wsum;
        __syncthreads();
        for (int i = 0; i < WAVES; ++i) acc += s_part[i];
        __syncthreads();   // masks and partial sums are rewritten next round
        if (done) break;
        hi -= consumed;
    }
    return acc;
}

// Element value of the scanned view in the local type.
template <int IDT, int OP, class L>
__device__ __forceinline__ L scan_value(typename elem<IDT>::T x, typename elem<IDT>::T y, L alpha) {
    const L x0 = (L)decode<IDT>(x);
    if constexpr (OP == DR_OP_MUL || OP == DR_OP_AXPY) return view_apply<OP, L>(x0, (L)decode<IDT>(y), alpha);
    else return view_apply<OP, L>(x0, (L)0, alpha);
}

template <int IDT, int ODT, bool C64>
__device__ __forceinline__ typename elem<ODT>::T scan_out(carry_t<IDT, C64> carry, local_t<IDT> woff,
                                                           local_t<IDT> pre) {
    using O = typename elem<ODT>::T;
    if constexpr (IDT == DR_I32) {
        const int64_t v = carry + woff + pre;
        if constexpr (ODT == DR_I64) return v;
        else return (int32_t)(uint32_t)(uint64_t)v;
    } else if constexpr (IDT == DR_F64) {
        return carry + (woff + pre);
    } else if constexpr (C64) {
        return (O)(carry + ((double)woff + (double)pre));
    } else {
        return carry + (woff + pre);
    }
}

// One tile at processing index r (physical tile t). Whole workgroup.
// FUSED: also returns (thread 0) the tile's sum of ROP over (in0, in1)
// with accumulation RACC.
template <int IDT, int ODT, int OP, bool C64, bool FUSED, int ROP, int RACC, int ITEMS, bool REV>
__device__ __forceinline__ double scan_tile(const LaunchArgs& a, uint32_t tag, int64_t r, int64_t t, int64_t T,
                                            const SegInfo& si) {
    constexpr bool rev = REV;
    constexpr int V = vwidth<IDT>();
    constexpr int SLOTS = ITEMS / V;
    constexpr int WAVES = kBlock / 64;
    constexpr bool ZIP = (OP == DR_OP_MUL || OP == DR_OP_AXPY) ||
                         (FUSED && (ROP == DR_OP_MUL || ROP == DR_OP_AXPY));
    using L = local_t<IDT>;
    using C = carry_t<IDT, C64>;
    using O = typename elem<ODT>::T;
    __shared__ L s_wtot[WAVES];
    __shared__ double s_red[WAVES];

    const int64_t stop = a.mode == DR_MODE_BATCH ? (rev ? T - (si.first + si.ntiles) : si.first) : 0;
    const int w = threadIdx.x >> 6, l = lane_id();
    const int64_t u0 = (t - si.first) * a.tile;
    const L alpha = (L)a.alpha;

    const bool full = tile_full<V, SLOTS>(si, u0);
    vec<IDT> x[SLOTS], y[SLOTS];
    load_slots<IDT, SLOTS>(x, si.in0, si, u0, w, l, rev);
    if constexpr (ZIP) load_slots<IDT, SLOTS>(y, si.in1, si, u0, w, l, rev);

    // fused reduction of the second view (not order-sensitive), before the
    // scan values replace the loaded ones
    double rpart_thread = 0.0;
    if constexpr (FUSED && IDT == DR_F64) {
        double rs = 0.0;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
#pragma unroll
            for (int e = 0; e < V; ++e)
                rs += view_apply<ROP, double>(decode<IDT>(x[s].e[e]), decode<IDT>(y[s].e[e]), 0.0);
        }
        rpart_thread = rs;
    } else if constexpr (FUSED) {
        float rs = 0.0f, rc = 0.0f;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const float x0 = (float)decode<IDT>(x[s].e[e]);
                const float x1 = (float)decode<IDT>(y[s].e[e]);
                if constexpr (RACC == DR_ACC_COMPENSATED) {
                    float p, pe, err;
                    if constexpr (ROP == DR_OP_MUL) two_prod(x0, x1, p, pe);
                    else if constexpr (ROP == DR_OP_SQUARE) two_prod(x0, x0, p, pe);
                    else { p = x0; pe = 0.0f; }
                    two_sum(rs, p, rs, err);
                    rc += err + pe;
                } else {
                    rs += view_apply<ROP, float>(x0, x1, 0.0f);
                }
            }
        }
        rpart_thread = (double)rs + (double)rc;
    }

    // scan values in processing order; per slot, only the offset of the
    // slot's first element is kept: the serial prefix inside the slot is
    // recomputed (in the same order) when the outputs are formed
    L v[SLOTS][V];
    L base[SLOTS];
    L run = (L)0;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
#pragma unroll
        for (int e = 0; e < V; ++e)
            v[s][e] = scan_value<IDT, OP, L>(x[s].e[e], ZIP ? y[s].e[e] : zero_elem<IDT>(), alpha);
        mirror_if(v[s], rev);
        L tot = v[s][0];
#pragma unroll
        for (int e = 1; e < V; ++e) tot = tot + v[s][e];
        const L inc = wave_incl_scan(tot);
        base[s] = run + shfl_up1(inc);
        run = run + readlane(inc, 63);
    }
    if (l == 0) s_wtot[w] = run;
    __syncthreads();

    L woff = (L)0;
    for (int i = 0; i < w; ++i) woff += s_wtot[i];
    L tl = (L)0;
    for (int i = 0; i < WAVES; ++i) tl += s_wtot[i];
    const C agg = (C)tl;
    C excl = (C)0;
    uint64_t* tw = (uint64_t*)(a.ws + a.lay.off_tile) + r * (int64_t)a.lay.tile_words;
    if (r != stop) {
        if (threadIdx.x == 0) tagged_store(tw + kAggWord, tag, to_bits(agg));
        excl = look_back<C>(a, tag, r, stop);
    }
    if (threadIdx.x == 0) tagged_store(tw + kInclWord, tag, to_bits(excl + agg));
    if constexpr (FUSED) {
        const double wr = wave_sum(rpart_thread);
        if (l == 0) s_red[w] = wr;
        __syncthreads();
    }

#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        O o[V];
        L pre = v[s][0];
        o[0] = scan_out<IDT, ODT, C64>(excl, woff, base[s] + pre);
#pragma unroll
        for (int e = 1; e < V; ++e) {
            pre = pre + v[s][e];
            o[e] = scan_out<IDT, ODT, C64>(excl, woff, base[s] + pre);
        }
        mirror_if(o, rev);
        store_slot<O, V, SLOTS>(si.out0, si, u0, w, l, s, rev, full, o);
    }
    double part = 0.0;
    if constexpr (FUSED) {
        if (threadIdx.x == 0)
            for (int i = 0; i < WAVES; ++i) part += s_red[i];
    }
    return part;
}

// One workgroup per tile; the block index is the processing index r.
// Tile r waits only for tiles of lower index. Workgroups of a launch are
// assigned to the XCDs round-robin and each XCD starts its workgroups in
// increasing index order, so the lowest unfinished tile is always running
// or next to start on its XCD: every wait ends (and each is also bounded by
// a.spin_ticks, which turns a stuck wait into a device fault flag).
template <int IDT, int ODT, int OP, bool C64, bool FUSED, int ROP, int RACC, int ITEMS, bool REV>
__global__ __launch_bounds__(kBlock) void k_scan(LaunchArgs a) {
    const uint32_t tag = begin_launch(a.ws);
    TileMap tm;
    tm.init(a);
    if (!tm.ok) return;
    const int64_t T = tm.total_tiles;
    const int64_t r = blockIdx.x;
    if (r < T) {
        const int64_t t = REV ? T - 1 - r : r;
        SegInfo si;
        if (!tm.find(a, t, si)) {
            // malformed row (flagged): publish an inclusive 0 so that later
            // tiles' look-backs stop here instead of waiting
            if (threadIdx.x == 0) {
                uint64_t* tw = (uint64_t*)(a.ws + a.lay.off_tile) + r * (int64_t)a.lay.tile_words;
                tagged_store(tw + kInclWord, tag, 0);
            }
            return;
        }
        const double part = scan_tile<IDT, ODT, OP, C64, FUSED, ROP, RACC, ITEMS, REV>(a, tag, r, t, T, si);
        if constexpr (FUSED) {
            if (threadIdx.x >= 64) return;   // wave 0 publishes the partial and combines
            if (a.mode == DR_MODE_BATCH) combine_tile_batch<double>(a, tag, t, si, part);
            else combine_member<double>(a, tag, 0, 0, t, T, 0, part);
        }
    } else if (FUSED && r == 0 && threadIdx.x == 0) {   // no tiles at all
        if (a.mode == DR_MODE_BATCH) write_all_init<double>(a);
        else write_result<double>(a, 0, 0.0);
    }
}

template <int IDT, int ODT, int OP, bool C64, bool FUSED, int ROP, int RACC, int ITEMS>
hipError_t launch_scan(const LaunchArgs& a, int64_t grid, hipStream_t stream) {
    hipError_t e = launch_prologue(a, stream);
    if (e != hipSuccess) return e;
    if (a.flags & DR_SCAN_REVERSE)
        hipLaunchKernelGGL((k_scan<IDT, ODT, OP, C64, FUSED, ROP, RACC, ITEMS, true>), dim3((uint32_t)grid),
                           dim3(kBlock), 0, stream, a);
    else
        hipLaunchKernelGGL((k_scan<IDT, ODT, OP, C64, FUSED, ROP, RACC, ITEMS, false>), dim3((uint32_t)grid),
                           dim3(kBlock), 0, stream, a);
    return hipGetLastError();
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
    DR_SCAN_ID(DR_I32, DR_I32, true, 64)
    DR_SCAN_OPS(DR_F32, DR_F32, true, 16)
    DR_SCAN_ID(DR_F32, DR_F32, true, 32)
    DR_SCAN_ID(DR_F32, DR_F32, true, 64)
    DR_SCAN_OPS(DR_F32, DR_F32, false, 16)
    DR_SCAN_OPS(DR_BF16, DR_F32, true, 16)
    DR_SCAN_ID(DR_BF16, DR_F32, true, 64)
    DR_SCAN_OPS(DR_F64, DR_F64, true, 16)
    DR_SCAN_ID(DR_F64, DR_F64, true, 32)
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
