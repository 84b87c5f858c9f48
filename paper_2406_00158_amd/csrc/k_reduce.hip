// k_reduce.hip — transform_reduce over a zip/transform view of a segmented
// range (section 4.3, "reduce"; Algorithm 1 is the dot product
// zip | transform(l*r) | reduce, Algorithm 3 the per-segment partials that
// are combined afterwards).
//
// One workgroup per tile (a tile lies inside one segment). Each thread
// accumulates its ITEMS elements, the workgroup reduces them to one tile
// partial, and the partials are combined deterministically in the same
// launch (dr_combine.hpp): over the whole range in CONCAT mode, per segment
// in BATCH mode. No second pass, no host-side combine, and no atomic that
// every workgroup hits (a one-thread prologue bumps the launch epoch).
//
// Accumulation inside a workgroup (over its tile, or in the streaming form
// over all of its tiles):
//  - int32 inputs: int64, exact.
//  - binary32 / bfloat16 inputs, PLAIN: binary32 running sums per thread, a
//    binary32 tree over the wave and the waves in order, all in binary32;
//    only the workgroup's partial is widened to binary64.
//  - COMPENSATED: a binary32 (sum, error) pair per thread: TwoSum (Knuth) on
//    every addition and an FMA-based TwoProduct for products (bfloat16
//    products are exact in binary32 and need none), which keeps each
//    rounding error of the binary32 arithmetic; the pairs are added pairwise
//    (TwoSum of the sums, errors added) over the wave and the waves, still in
//    binary32, and only the workgroup's pair is widened (exactly) to binary64.
//  - binary64 inputs: binary64 sums.
// Workgroup partials are combined across workgroups and segments in binary64
// (or int64): the only binary64 arithmetic of a binary32 reduction.
#include "dr_combine.hpp"

namespace dr {

template <int IDT>
using partial_t = typename std::conditional<IDT == DR_I32, int64_t, double>::type;

// Per-thread max (min when mn) of the view values of one tile, each value
// formed as for_each stores it (binary32 arithmetic for binary32 / bfloat16
// inputs, binary64 for binary64, exact int64 for int32), widened exactly to
// the partial type.
// (si, u0): the tile's geometry; elements outside the segment (loaded as 0)
// are skipped.
template <int IDT, int OP, int SLOTS>
__device__ __forceinline__ partial_t<IDT> thread_tile_minmax(const vec<IDT> (&x)[SLOTS], const vec<IDT> (&y)[SLOTS],
                                                            double alpha_d, bool mn, const SegInfo& si,
                                                            int64_t u0) {
    constexpr int V = vwidth<IDT>();
    constexpr bool ZIP = (OP == DR_OP_MUL || OP == DR_OP_AXPY);
    const bool full = tile_full<V, SLOTS>(si, u0);
    const int w = threadIdx.x >> 6, l = lane_id();
    if constexpr (IDT == DR_F32 || IDT == DR_BF16) {
        const float alpha = (float)alpha_d;
        float m = mm_id<float>(mn);
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const float x1 = ZIP ? decode<IDT>(y[q].e[e]) : 0.0f;
                const float v = view_apply<OP, float>(decode<IDT>(x[q].e[e]), x1, alpha);
                if (full || elem_in<V, SLOTS>(si, u0, w, l, q, e, false)) m = mm_op(m, v, mn);
            }
        }
        return (double)m;
    } else {
        using P = partial_t<IDT>;
        const P alpha = (P)alpha_d;
        P m = mm_id<P>(mn);
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const P x1 = ZIP ? (P)decode<IDT>(y[q].e[e]) : (P)0;
                const P v = view_apply<OP, P>((P)decode<IDT>(x[q].e[e]), x1, alpha);
                if (full || elem_in<V, SLOTS>(si, u0, w, l, q, e, false)) m = mm_op(m, v, mn);
            }
        }
        return m;
    }
}

// Exact (int64) or binary64 sum of the view over a thread's loaded
// elements (int32 and binary64 inputs).
template <int IDT, int OP, int SLOTS>
__device__ __forceinline__ partial_t<IDT> thread_tile_exact(const vec<IDT> (&x)[SLOTS], const vec<IDT> (&y)[SLOTS],
                                                           double alpha_d) {
    constexpr int V = vwidth<IDT>();
    constexpr bool ZIP = (OP == DR_OP_MUL || OP == DR_OP_AXPY);
    using P = partial_t<IDT>;
    const P alpha = (P)alpha_d;
    P acc = (P)0;
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const P x1 = ZIP ? (P)decode<IDT>(y[q].e[e]) : (P)0;
            acc += view_apply<OP, P>((P)decode<IDT>(x[q].e[e]), x1, alpha);
        }
    }
    return acc;
}

// Sum of the view over one tile, returned in thread 0 (whole workgroup).
template <int IDT, int OP, int ACC, int ITEMS>
__device__ __forceinline__ partial_t<IDT> tile_partial(const LaunchArgs& a, const SegInfo& si, int64_t t) {
    constexpr int V = vwidth<IDT>();
    constexpr int SLOTS = ITEMS / V;
    constexpr bool ZIP = (OP == DR_OP_MUL || OP == DR_OP_AXPY);
    constexpr int WAVES = kBlock / 64;
    using P = partial_t<IDT>;
    constexpr bool F32PATH = (IDT == DR_F32 || IDT == DR_BF16);
    __shared__ P s_wave[WAVES];
    __shared__ float s_ws[WAVES], s_wc[WAVES];

    const int w = threadIdx.x >> 6, l = lane_id();
    const int64_t u0 = (t - si.first) * a.tile;
    vec<IDT> x[SLOTS], y[SLOTS];
    load_slots<IDT, SLOTS>(x, si.in0, si, u0, w, l, false);
    if constexpr (ZIP) load_slots<IDT, SLOTS>(y, si.in1, si, u0, w, l, false);

    P part = (P)0;
    if constexpr (ACC == kAccMinMax) {
        const bool mn = (a.flags & kFlagMin) != 0;
        const P m = wave_reduce_cmb<kCmbMinMax>(thread_tile_minmax<IDT, OP, SLOTS>(x, y, a.alpha, mn, si, u0), mn);
        if (l == 0) s_wave[w] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            part = mm_id<P>(mn);
            for (int i = 0; i < WAVES; ++i) part = mm_op(part, s_wave[i], mn);
        }
    } else if constexpr (F32PATH) {
        constexpr bool COMP = ACC == DR_ACC_COMPENSATED;
        float fs = 0.0f, fc = 0.0f;
        if constexpr (COMP) comp_accumulate<IDT, OP, SLOTS>(x, y, (float)a.alpha, fs, fc);
        else plain_accumulate<IDT, OP, SLOTS>(x, y, (float)a.alpha, fs);
        part = block_partial_f32<COMP, WAVES>(fs, fc, s_ws, s_wc);
    } else {
        // int32 -> int64 exact, or binary64
        const P wsum = wave_sum(thread_tile_exact<IDT, OP, SLOTS>(x, y, a.alpha));
        if (l == 0) s_wave[w] = wsum;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int i = 0; i < WAVES; ++i) part += s_wave[i];
    }
    return part;
}

// One workgroup per tile (tile = block index).
template <int IDT, int OP, int ACC, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_reduce(LaunchArgs a) {
    using P = partial_t<IDT>;
    constexpr int CMB = ACC == kAccMinMax ? kCmbMinMax : kCmbSum;
    const uint32_t tag = begin_launch(a.ws);
    TileMap tm;
    tm.init(a);
    if (!tm.ok) return;
    const int64_t T = tm.total_tiles;
    const int64_t t = blockIdx.x;
    if (t < T) {
        SegInfo si;
        if (!tm.find(a, t, si)) return;
        const P part = tile_partial<IDT, OP, ACC, ITEMS>(a, si, t);
        if (threadIdx.x >= 64) return;   // waves 1..3 are done; wave 0 publishes and combines
        if (a.mode == DR_MODE_BATCH) combine_tile_batch<P, CMB>(a, tag, t, si, part);
        else combine_member<P, CMB>(a, tag, 0, 0, t, T, 0, part);
    } else if (t == 0 && threadIdx.x == 0) {   // no tiles at all
        if (a.mode == DR_MODE_BATCH) write_all_init<P, CMB>(a);
        else write_result<P, CMB>(a, 0, cmb_id<CMB, P>((a.flags & kFlagMin) != 0));
    }
}

// CONCAT streaming form: a grid of resident workgroups, workgroup b taking
// tiles b, b + G, b + 2G, ... with the loads of its next tile in flight while
// it sums the current one. Each thread accumulates all of its elements in
// binary32 (a compensated pair, or a plain sum; int64 / binary64 for int32 /
// binary64 inputs), the workgroup reduces its threads in binary32 and
// publishes one binary64 partial, and the partials of the G workgroups are
// combined in workgroup order. The tile-to-workgroup map is fixed for a
// given grid, so the result is the same from run to run.
template <int IDT, int OP, int ACC, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_reduce_stream(LaunchArgs a) {
    constexpr int V = vwidth<IDT>();
    constexpr int SLOTS = ITEMS / V;
    constexpr bool ZIP = (OP == DR_OP_MUL || OP == DR_OP_AXPY);
    constexpr int WAVES = kBlock / 64;
    using P = partial_t<IDT>;
    constexpr int CMB = ACC == kAccMinMax ? kCmbMinMax : kCmbSum;
    constexpr bool F32PATH = (IDT == DR_F32 || IDT == DR_BF16) && CMB == kCmbSum;
    constexpr bool COMP = ACC == DR_ACC_COMPENSATED;
    __shared__ P s_wave[WAVES];
    __shared__ float s_ws[WAVES], s_wc[WAVES];
    const uint32_t tag = begin_launch(a.ws);
    TileMap tm;
    tm.init(a);
    if (!tm.ok) return;
    const int64_t T = tm.total_tiles;
    const int64_t G = gridDim.x;
    const int w = threadIdx.x >> 6, l = lane_id();
    const bool mn = (a.flags & kFlagMin) != 0;
    const float alpha_f = (float)a.alpha;
    // the thread's accumulators over its tiles: binary32 (fs, fc), or a
    // binary64 / int64 sum, or max / min
    float fs = 0.0f, fc = 0.0f;
    P mine = cmb_id<CMB, P>(mn);
    auto merge = [&](const vec<IDT> (&x)[SLOTS], const vec<IDT> (&y)[SLOTS], const SegInfo& si, int64_t tt) {
        if constexpr (CMB == kCmbMinMax)
            mine = mm_op(mine, thread_tile_minmax<IDT, OP, SLOTS>(x, y, a.alpha, mn, si, (tt - si.first) * a.tile),
                         mn);
        else if constexpr (F32PATH && COMP) comp_accumulate<IDT, OP, SLOTS>(x, y, alpha_f, fs, fc);
        else if constexpr (F32PATH) plain_accumulate<IDT, OP, SLOTS>(x, y, alpha_f, fs);
        else mine += thread_tile_exact<IDT, OP, SLOTS>(x, y, a.alpha);
    };
    vec<IDT> xa[SLOTS], ya[SLOTS], xb[SLOTS], yb[SLOTS];
    int64_t t = blockIdx.x;
    SegInfo sa, sb;
    bool ha = t < T && tm.find(a, t, sa);
    if (ha) {
        load_slots<IDT, SLOTS>(xa, sa.in0, sa, (t - sa.first) * a.tile, w, l, false);
        if constexpr (ZIP) load_slots<IDT, SLOTS>(ya, sa.in1, sa, (t - sa.first) * a.tile, w, l, false);
    }
    while (ha) {
        const int64_t tb = t + G;
        const bool hb = tb < T && tm.find(a, tb, sb);
        if (hb) {
            load_slots<IDT, SLOTS>(xb, sb.in0, sb, (tb - sb.first) * a.tile, w, l, false);
            if constexpr (ZIP) load_slots<IDT, SLOTS>(yb, sb.in1, sb, (tb - sb.first) * a.tile, w, l, false);
        }
        merge(xa, ya, sa, t);
        if (!hb) break;
        const int64_t ta = tb + G;
        ha = ta < T && tm.find(a, ta, sa);
        if (ha) {
            load_slots<IDT, SLOTS>(xa, sa.in0, sa, (ta - sa.first) * a.tile, w, l, false);
            if constexpr (ZIP) load_slots<IDT, SLOTS>(ya, sa.in1, sa, (ta - sa.first) * a.tile, w, l, false);
        }
        merge(xb, yb, sb, tb);
        t = ta;
    }
    P part = cmb_id<CMB, P>(mn);
    if constexpr (F32PATH) {
        part = (P)block_partial_f32<COMP, WAVES>(fs, fc, s_ws, s_wc);
        if (threadIdx.x >= 64) return;
    } else {
        const P wsum = wave_reduce_cmb<CMB>(mine, mn);
        if (l == 0) s_wave[w] = wsum;
        __syncthreads();
        if (threadIdx.x >= 64) return;
        if (l == 0)
            for (int i = 0; i < WAVES; ++i) part = cmb_op<CMB>(part, s_wave[i], mn);
    }
    combine_member<P, CMB>(a, tag, 0, 0, blockIdx.x, G, 0, part);
}

template <int IDT, int OP, int ACC, int ITEMS>
hipError_t launch_reduce(const LaunchArgs& a, int64_t grid, hipStream_t stream) {
    hipError_t e = launch_prologue(a, stream);
    if (e != hipSuccess) return e;
    if (a.mode == DR_MODE_CONCAT && (a.flags & kFlagTilePerBlock) == 0) {
        static const int resident = resident_grid((const void*)k_reduce_stream<IDT, OP, ACC, ITEMS>);
        if (grid > resident) grid = resident;
        hipLaunchKernelGGL((k_reduce_stream<IDT, OP, ACC, ITEMS>), dim3((uint32_t)grid), dim3(kBlock), 0,
                           stream, a);
    } else {
        hipLaunchKernelGGL((k_reduce<IDT, OP, ACC, ITEMS>), dim3((uint32_t)grid), dim3(kBlock), 0,
                           stream, a);
    }
    return hipGetLastError();
}

#define DR_RED_OPS(IDT, ACC, ITEMS)                                                   \
    if (in_dt == IDT && acc == ACC && items == ITEMS) {                               \
        switch (op) {                                                                 \
        case DR_OP_IDENTITY: return launch_reduce<IDT, DR_OP_IDENTITY, ACC, ITEMS>;   \
        case DR_OP_SQUARE: return launch_reduce<IDT, DR_OP_SQUARE, ACC, ITEMS>;       \
        case DR_OP_MUL: return launch_reduce<IDT, DR_OP_MUL, ACC, ITEMS>;             \
        case DR_OP_AXPY: return launch_reduce<IDT, DR_OP_AXPY, ACC, ITEMS>;           \
        default: return nullptr;                                                      \
        }                                                                             \
    }

// max / min reductions (every op, 16 items; bfloat16 also 32, its default).
LaunchFn find_reduce_minmax(int in_dt, int op, int items) {
    const int acc = kAccMinMax;
    if (in_dt == DR_F32) { DR_RED_OPS(DR_F32, kAccMinMax, 16) }
    if (in_dt == DR_BF16) { DR_RED_OPS(DR_BF16, kAccMinMax, 16) }
    if (in_dt == DR_BF16) { DR_RED_OPS(DR_BF16, kAccMinMax, 32) }
    if (in_dt == DR_F64) { DR_RED_OPS(DR_F64, kAccMinMax, 16) }
    if (in_dt == DR_I32) { DR_RED_OPS(DR_I32, kAccMinMax, 16) }
    return nullptr;
}

LaunchFn find_reduce(int in_dt, int op, int acc, int items) {
    // integer and binary64 reductions ignore `acc`
    if (in_dt == DR_I32 || in_dt == DR_F64) acc = DR_ACC_PLAIN;
    DR_RED_OPS(DR_F32, DR_ACC_COMPENSATED, 16)
    DR_RED_OPS(DR_F32, DR_ACC_COMPENSATED, 32)
    DR_RED_OPS(DR_F32, DR_ACC_COMPENSATED, 64)
    DR_RED_OPS(DR_F32, DR_ACC_PLAIN, 16)
    DR_RED_OPS(DR_F32, DR_ACC_PLAIN, 32)
    DR_RED_OPS(DR_F32, DR_ACC_PLAIN, 64)
    DR_RED_OPS(DR_BF16, DR_ACC_COMPENSATED, 16)
    DR_RED_OPS(DR_BF16, DR_ACC_COMPENSATED, 32)
    DR_RED_OPS(DR_BF16, DR_ACC_COMPENSATED, 64)
    DR_RED_OPS(DR_BF16, DR_ACC_PLAIN, 16)
    DR_RED_OPS(DR_BF16, DR_ACC_PLAIN, 32)
    DR_RED_OPS(DR_BF16, DR_ACC_PLAIN, 64)
    DR_RED_OPS(DR_I32, DR_ACC_PLAIN, 16)
    DR_RED_OPS(DR_F64, DR_ACC_PLAIN, 16)
    return nullptr;
}

}  // namespace dr
