// k_scan_core.hpp — the parts of the scan shared by every translation unit
// that instantiates scan kernels: the tile scan in registers (values,
// outputs), the decoupled look-back and the single-pass look-back kernel
// k_scan, templated on the workgroup size (256 threads everywhere; the
// look-back kernel is also built at 512 and 1024 threads, k_scan_wide.hip).
// The forms themselves are described in k_scan.hip.
#pragma once
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
// hi - i, so one round trip to memory covers BLOCK predecessors. Tiles start
// so fast (hundreds per microsecond at full bandwidth) that the nearest
// published inclusive prefix is often hundreds of tiles back; a 64-wide
// window would need several round trips. Returns the carry in every thread.
template <class C, int BLOCK = kBlock>
__device__ __forceinline__ C look_back(const LaunchArgs& a, uint32_t tag, int64_t r, int64_t stop) {
    constexpr int WAVES = BLOCK / 64;
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
            if (tid == 0) flag_error(a, DR_DEVFLAG_TIMEOUT);
            break;
        }
        // 2. one read of the statuses of up to BLOCK predecessors
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
        int f = BLOCK, z = BLOCK;
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
            consumed = BLOCK;
            done = f < BLOCK;
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

// Output of the generic scan: the sum as above, or max / min of the carry,
// the wave offset and the prefix inside the wave (exact; int32 outputs hold
// the int64 value modulo 2^32).
template <int IDT, int ODT, bool C64, int CMB>
__device__ __forceinline__ typename elem<ODT>::T scan_out_cmb(carry_t<IDT, C64> carry, local_t<IDT> woff,
                                                               local_t<IDT> pre, bool mn) {
    if constexpr (CMB == kCmbSum) {
        return scan_out<IDT, ODT, C64>(carry, woff, pre);
    } else {
        using C = carry_t<IDT, C64>;
        using O = typename elem<ODT>::T;
        const C v = mm_op(carry, mm_op((C)woff, (C)pre, mn), mn);
        if constexpr (ODT == DR_I32) return (int32_t)(uint32_t)(uint64_t)v;
        else return (O)v;
    }
}

// Per-wave partial of the fused reduction (ROP over the zipped (in0, in1)
// elements of a loaded tile, accumulated as RACC; order-insensitive, so it
// is taken before the scan values replace the loaded ones): binary32 inputs
// in binary32 (a compensated pair, or a plain sum), binary64 inputs in
// binary64. The result is in every lane.
template <int IDT, int ROP, int RACC, int SLOTS>
__device__ __forceinline__ void fused_wave(const vec<IDT> (&x)[SLOTS], const vec<IDT> (&y)[SLOTS], float& s,
                                           float& c, double& d) {
    constexpr int V = vwidth<IDT>();
    s = 0.0f;
    c = 0.0f;
    d = 0.0;
    if constexpr (IDT == DR_F64) {
        double rs = 0.0;
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) {
#pragma unroll
            for (int e = 0; e < V; ++e)
                rs += view_apply<ROP, double>(decode<IDT>(x[q].e[e]), decode<IDT>(y[q].e[e]), 0.0);
        }
        d = wave_sum(rs);
    } else if constexpr (RACC == DR_ACC_COMPENSATED) {
        comp_accumulate<IDT, ROP, SLOTS>(x, y, 0.0f, s, c);
        wave_sum_pair(s, c);
    } else {
        plain_accumulate<IDT, ROP, SLOTS>(x, y, 0.0f, s);
        s = readlane(wave_incl_scan(s), 63);
    }
}

// The workgroup's fused partial from its WAVES per-wave partials, in wave
// order, widened to binary64 once.
template <int IDT, int RACC, int WAVES>
__device__ __forceinline__ double fused_block(const float* ws, const float* wc, const double* wd) {
    if constexpr (IDT == DR_F64) {
        double t = 0.0;
        for (int i = 0; i < WAVES; ++i) t += wd[i];
        return t;
    } else if constexpr (RACC == DR_ACC_COMPENSATED) {
        float ts = ws[0], tc = wc[0];
        for (int i = 1; i < WAVES; ++i) pair_add(ts, tc, ws[i], wc[i]);
        return pair_widen(ts, tc);
    } else {
        float ts = 0.0f;
        for (int i = 0; i < WAVES; ++i) ts += ws[i];
        return (double)ts;
    }
}

// Scan values of a loaded tile in processing order. Per slot only the
// offset of the slot's first element inside the wave is kept (base[s]);
// the serial prefix inside the slot is recomputed, in the same order, when
// the outputs are formed. Returns the wave's total (every lane).
// (si, u0, full): the tile's geometry. Elements outside the segment (only
// in tiles that are not full) were loaded as 0: the identity of a sum, and
// replaced by the operator's identity otherwise.
template <int IDT, int OP, bool ZIP, int SLOTS, bool REV, int CMB = kCmbSum, int V = vwidth<IDT>(),
          int BLOCK = kBlock>
__device__ __forceinline__ local_t<IDT> tile_values(const vec<IDT, V> (&x)[SLOTS], const vec<IDT, V> (&y)[SLOTS],
                                                    local_t<IDT> alpha, local_t<IDT> (&v)[SLOTS][V],
                                                    local_t<IDT> (&base)[SLOTS], bool mn, const SegInfo& si,
                                                    int64_t u0, bool full) {
    using L = local_t<IDT>;
    const L id = cmb_id<CMB, L>(mn);
    const int w = threadIdx.x >> 6, l = lane_id();
    L run = id;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            v[s][e] = scan_value<IDT, OP, L>(x[s].e[e], ZIP ? y[s].e[e] : zero_elem<IDT>(), alpha);
            if constexpr (CMB != kCmbSum)
                if (!full && !elem_in<V, SLOTS, BLOCK>(si, u0, w, l, s, e, REV)) v[s][e] = id;
        }
        mirror_if(v[s], REV);
        L tot = v[s][0];
#pragma unroll
        for (int e = 1; e < V; ++e) tot = cmb_op<CMB>(tot, v[s][e], mn);
        const L inc = wave_incl_scan_cmb<CMB>(tot, mn);
        L up = __shfl_up(inc, 1, 64);
        if (lane_id() == 0) up = id;
        base[s] = cmb_op<CMB>(run, up, mn);
        run = cmb_op<CMB>(run, readlane(inc, 63), mn);
    }
    return run;
}

// One form of tile_write below. FULL: the tile lies wholly inside its segment with aligned rows, so every
// slot is one unchecked vector store at a fixed stride from the lane's first
// vector; otherwise each slot is checked on its own.
template <int IDT, int ODT, bool C64, int SLOTS, bool REV, int CMB, int V, bool FULL, int BLOCK = kBlock>
__device__ __forceinline__ void tile_write_part(const local_t<IDT> (&v)[SLOTS][V],
                                                const local_t<IDT> (&base)[SLOTS], carry_t<IDT, C64> excl,
                                                local_t<IDT> woff, const SegInfo& si, int64_t u0, int w, int l,
                                                bool exc, bool mn) {
    using L = local_t<IDT>;
    using O = typename elem<ODT>::T;
    constexpr int64_t NV = (int64_t)BLOCK * SLOTS;
    constexpr int64_t step = (REV ? -64 : 64) * (int64_t)(V * sizeof(O));
    char* tb = nullptr;
    if constexpr (FULL) {
        const int64_t p0 = (int64_t)(w * SLOTS) * 64 + l;
        const int64_t q0 = REV ? NV - 1 - p0 : p0;
        tb = (char*)si.out0 + (u0 - si.shift + q0 * V) * (int64_t)sizeof(O);
    }
    const L id = cmb_id<CMB, L>(mn);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        O o[V];
        L pre = v[s][0];       // inclusive prefix inside the slot
        L before = id;         // exclusive prefix inside the slot
        o[0] = scan_out_cmb<IDT, ODT, C64, CMB>(excl, woff, exc ? base[s] : cmb_op<CMB>(base[s], pre, mn), mn);
#pragma unroll
        for (int e = 1; e < V; ++e) {
            before = pre;
            pre = cmb_op<CMB>(pre, v[s][e], mn);
            o[e] = scan_out_cmb<IDT, ODT, C64, CMB>(excl, woff, cmb_op<CMB>(base[s], exc ? before : pre, mn), mn);
        }
        (void)before;
        mirror_if(o, REV);
        if constexpr (FULL) store_run<O, V>(tb + s * step, 0, o);
        else store_slot<O, V, SLOTS, BLOCK>(si.out0, si, u0, w, l, s, REV, false, o);
    }
}

// Outputs of a tile: carry + offset of the wave + prefix inside the wave.
// `exc`: exclusive scan (each output combines the elements strictly before
// it in processing order). `full` (uniform) picks the unchecked form.
template <int IDT, int ODT, bool C64, int SLOTS, bool REV, int CMB = kCmbSum, int V = vwidth<IDT>(),
          int BLOCK = kBlock>
__device__ __forceinline__ void tile_write(const local_t<IDT> (&v)[SLOTS][V],
                                           const local_t<IDT> (&base)[SLOTS], carry_t<IDT, C64> excl,
                                           local_t<IDT> woff, const SegInfo& si, int64_t u0, int w, int l,
                                           bool full, bool exc = false, bool mn = false) {
    if (full)
        tile_write_part<IDT, ODT, C64, SLOTS, REV, CMB, V, true, BLOCK>(v, base, excl, woff, si, u0, w, l, exc,
                                                                       mn);
    else
        tile_write_part<IDT, ODT, C64, SLOTS, REV, CMB, V, false, BLOCK>(v, base, excl, woff, si, u0, w, l, exc,
                                                                        mn);
}

// The caller's initial value in the carry type (scans with kFlagHasInit).
template <class C, int IDT>
__device__ __forceinline__ C init_carry(const LaunchArgs& a) {
    if constexpr (IDT == DR_I32) return (C)a.init_i;
    else return (C)a.init_f;
}

template <int IDT, int OP, bool FUSED, int ROP>
constexpr bool zip_view() {
    return (OP == DR_OP_MUL || OP == DR_OP_AXPY) || (FUSED && (ROP == DR_OP_MUL || ROP == DR_OP_AXPY));
}

// Processing index of a BATCH segment's first tile (the look-back of a
// tile stops there); 0 in CONCAT mode.
template <bool REV>
__device__ __forceinline__ int64_t stop_of(const LaunchArgs& a, const SegInfo& si, int64_t T) {
    if (a.mode != DR_MODE_BATCH) return 0;
    return REV ? T - (si.first + si.ntiles) : si.first;
}

// One tile at processing index r (physical tile t). Whole workgroup of
// BLOCK threads. FUSED: also returns (thread 0) the tile's sum of ROP over
// (in0, in1) with accumulation RACC.
template <int IDT, int ODT, int OP, bool C64, bool FUSED, int ROP, int RACC, int ITEMS, bool REV,
          int BLOCK = kBlock>
__device__ __forceinline__ double scan_tile(const LaunchArgs& a, uint32_t tag, int64_t r, int64_t t, int64_t T,
                                            const SegInfo& si) {
    constexpr int V = vwidth<IDT>();
    constexpr int SLOTS = ITEMS / V;
    constexpr int WAVES = BLOCK / 64;
    constexpr bool ZIP = zip_view<IDT, OP, FUSED, ROP>();
    using L = local_t<IDT>;
    using C = carry_t<IDT, C64>;
    __shared__ L s_wtot[WAVES];
    __shared__ float s_rs[WAVES], s_rc[WAVES];
    __shared__ double s_rd[WAVES];

    const int64_t stop = stop_of<REV>(a, si, T);
    const int w = threadIdx.x >> 6, l = lane_id();
    const int64_t u0 = (t - si.first) * a.tile;

    const bool full = tile_full<V, SLOTS, BLOCK>(si, u0);
    vec<IDT> x[SLOTS], y[SLOTS];
    load_slots<IDT, SLOTS, V, true, BLOCK>(x, si.in0, si, u0, w, l, REV);
    if constexpr (ZIP) load_slots<IDT, SLOTS, V, true, BLOCK>(y, si.in1, si, u0, w, l, REV);
    float rs = 0.0f, rc = 0.0f;
    double rd = 0.0;
    if constexpr (FUSED) fused_wave<IDT, ROP, RACC, SLOTS>(x, y, rs, rc, rd);

    L v[SLOTS][V];
    L base[SLOTS];
    const L run = tile_values<IDT, OP, ZIP, SLOTS, REV, kCmbSum, V, BLOCK>(x, y, (L)a.alpha, v, base, false, si,
                                                                         u0, full);
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
        excl = look_back<C, BLOCK>(a, tag, r, stop);
    }
    if (threadIdx.x == 0) tagged_store(tw + kInclWord, tag, to_bits(excl + agg));
    if constexpr (FUSED) {
        if (l == 0) {
            s_rs[w] = rs;
            s_rc[w] = rc;
            s_rd[w] = rd;
        }
        __syncthreads();
    }
    // the initial value reaches the outputs only, never the published carries
    const C eo = (a.flags & kFlagHasInit) ? init_carry<C, IDT>(a) + excl : excl;
    tile_write<IDT, ODT, C64, SLOTS, REV, kCmbSum, V, BLOCK>(v, base, eo, woff, si, u0, w, l, full,
                                                           (a.flags & DR_SCAN_EXCLUSIVE) != 0);
    double part = 0.0;
    if constexpr (FUSED) {
        if (threadIdx.x == 0) part = fused_block<IDT, RACC, WAVES>(s_rs, s_rc, s_rd);
    }
    return part;
}

// One workgroup per tile; the block index is the processing index r.
// Tile r waits only for tiles of lower index. Workgroups of a launch are
// assigned to the XCDs round-robin and each XCD starts its workgroups in
// increasing index order, so the lowest unfinished tile is always running
// or next to start on its XCD: every wait ends (and each is also bounded by
// a.spin_ticks, which turns a stuck wait into a device fault flag).
template <int IDT, int ODT, int OP, bool C64, bool FUSED, int ROP, int RACC, int ITEMS, bool REV,
          int BLOCK = kBlock>
__global__ __launch_bounds__(BLOCK) void k_scan(LaunchArgs a) {
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
        const double part = scan_tile<IDT, ODT, OP, C64, FUSED, ROP, RACC, ITEMS, REV, BLOCK>(a, tag, r, t, T, si);
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

}  // namespace dr
