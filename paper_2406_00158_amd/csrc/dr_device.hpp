// dr_device.hpp — device-side building blocks shared by the gfx950 kernels:
// element types and 16-byte vector access, the view transforms, wave64
// scans/reductions on DPP, epoch-tagged status words for cross-workgroup
// communication, and the segment/tile geometry of a launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <limits>
#include <type_traits>

#include "dr.h"
#include "dr_internal.hpp"

namespace dr {

// ---------------------------------------------------------------------------
// Element types
// ---------------------------------------------------------------------------

struct bf16_t { uint16_t bits; };

template <int DT> struct elem;
template <> struct elem<DR_I32> { using T = int32_t; using acc = int64_t; };
template <> struct elem<DR_F32> { using T = float; using acc = float; };
template <> struct elem<DR_BF16> { using T = uint16_t; using acc = float; };
template <> struct elem<DR_F64> { using T = double; using acc = double; };
template <> struct elem<DR_I64> { using T = int64_t; using acc = int64_t; };

template <int DT> constexpr int esize() { return (int)sizeof(typename elem<DT>::T); }
template <int DT> constexpr int vwidth() { return 16 / esize<DT>(); }   // elements per 16 B

// Exact decode of one stored element into the arithmetic type of the view:
// bfloat16 is the upper half of a binary32 pattern.
__device__ __forceinline__ float bf16_decode(uint16_t b) {
    return __uint_as_float(((uint32_t)b) << 16);
}

template <int DT> __device__ __forceinline__ typename elem<DT>::acc decode(typename elem<DT>::T v);
template <> __device__ __forceinline__ int64_t decode<DR_I32>(int32_t v) { return (int64_t)v; }
template <> __device__ __forceinline__ float decode<DR_F32>(float v) { return v; }
template <> __device__ __forceinline__ float decode<DR_BF16>(uint16_t v) { return bf16_decode(v); }
template <> __device__ __forceinline__ double decode<DR_F64>(double v) { return v; }

// Vector of V elements (16 bytes by default; 8 bytes where a kernel wants
// narrower loads), accessed as one 4- or 2-dword load.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <int NB> struct vbits;
template <> struct vbits<16> { using T = u32x4; };
template <> struct vbits<8> { using T = u32x2; };

template <int DT, int V = vwidth<DT>()>
struct vec {
    typename elem<DT>::T e[V];
};

// NT: a non-temporal (streaming) load; otherwise a plain load, whose line
// stays in L2 for a later re-read.
template <int DT, int V = vwidth<DT>(), bool NT = true>
__device__ __forceinline__ vec<DT, V> load_vec(const void* base, int64_t j) {
    using R = typename vbits<V * esize<DT>()>::T;
    const R* p = (const R*)((const char*)base + j * esize<DT>());
    R w = NT ? __builtin_nontemporal_load(p) : *p;
    vec<DT, V> v;
    __builtin_memcpy(&v, &w, sizeof(R));
    return v;
}

template <int DT>
__device__ __forceinline__ typename elem<DT>::T load_one(const void* base, int64_t j) {
    return ((const typename elem<DT>::T*)base)[j];
}

// Store V consecutive elements of type OT (V * sizeof(OT) is a multiple of
// 16 and the address is 16-byte aligned) with 16-byte stores.
template <class OT, int V>
__device__ __forceinline__ void store_run(void* base, int64_t j, const OT (&v)[V]) {
    static_assert((V * sizeof(OT)) % 16 == 0, "store run must be whole vectors");
    u32x4* p = (u32x4*)((char*)base + j * (int64_t)sizeof(OT));
    const u32x4* src = (const u32x4*)v;
#pragma unroll
    for (int i = 0; i < (int)(V * sizeof(OT) / 16); ++i) __builtin_nontemporal_store(src[i], p + i);
}

// ---------------------------------------------------------------------------
// Wave64 primitives (DPP)
// ---------------------------------------------------------------------------

// DPP controls (GFX9 encoding).
enum : int {
    DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114, DPP_ROW_SHR8 = 0x118,
    DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143
};

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp32(uint32_t x) {
    // lanes whose source is out of the row, or whose row is masked off, get 0
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, false);
}

template <int CTRL, int ROW_MASK, class T>
__device__ __forceinline__ T dpp_move(T x) {
    if constexpr (sizeof(T) == 4) {
        uint32_t u = __builtin_bit_cast(uint32_t, x);
        return __builtin_bit_cast(T, dpp32<CTRL, ROW_MASK>(u));
    } else {
        uint64_t u = __builtin_bit_cast(uint64_t, x);
        uint32_t lo = dpp32<CTRL, ROW_MASK>((uint32_t)u);
        uint32_t hi = dpp32<CTRL, ROW_MASK>((uint32_t)(u >> 32));
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}

// Inclusive scan over the 64 lanes of a wave (lane order), identity 0.
template <class T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    x = x + dpp_move<DPP_ROW_SHR1, 0xf>(x);
    x = x + dpp_move<DPP_ROW_SHR2, 0xf>(x);
    x = x + dpp_move<DPP_ROW_SHR4, 0xf>(x);
    x = x + dpp_move<DPP_ROW_SHR8, 0xf>(x);
    x = x + dpp_move<DPP_ROW_BCAST15, 0xa>(x);
    x = x + dpp_move<DPP_ROW_BCAST31, 0xc>(x);
    return x;
}

template <class T>
__device__ __forceinline__ T readlane(T x, int lane) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), lane));
    } else {
        uint64_t u = __builtin_bit_cast(uint64_t, x);
        uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
        uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}

// Sum over the wave in a fixed tree order, result in every lane.
template <class T>
__device__ __forceinline__ T wave_sum(T x) {
    return readlane(wave_incl_scan(x), 63);
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// ---------------------------------------------------------------------------
// Combine operators of the generic algorithms
// ---------------------------------------------------------------------------
//
// kCmbSum: +. kCmbMinMax: max, or min when `mn` (a launch-wide flag); NaN
// operands are ignored (IEEE maxNum / minNum) unless both are NaN. Sums keep
// their own code paths (compensation, carries); these helpers carry the
// operator through the scan and combine structure.

constexpr int kCmbSum = 0;
constexpr int kCmbMinMax = 1;

template <class T>
__device__ __forceinline__ T mm_op(T a, T b, bool mn) {
    if constexpr (sizeof(T) == 4 && std::is_floating_point<T>::value) {
        return mn ? __builtin_fminf(a, b) : __builtin_fmaxf(a, b);
    } else if constexpr (std::is_floating_point<T>::value) {
        return mn ? __builtin_fmin(a, b) : __builtin_fmax(a, b);
    } else {
        return mn ? (a < b ? a : b) : (a > b ? a : b);
    }
}

template <class T>
__device__ __forceinline__ T mm_id(bool mn) {
    if constexpr (std::is_floating_point<T>::value) return mn ? (T)__builtin_inf() : -(T)__builtin_inf();
    else return mn ? std::numeric_limits<T>::max() : std::numeric_limits<T>::min();
}

template <int CMB, class T>
__device__ __forceinline__ T cmb_op(T a, T b, bool mn) {
    if constexpr (CMB == kCmbSum) return a + b;
    else return mm_op(a, b, mn);
}

template <int CMB, class T>
__device__ __forceinline__ T cmb_id(bool mn) {
    if constexpr (CMB == kCmbSum) return (T)0;
    else return mm_id<T>(mn);
}

// DPP move whose lanes without a source receive `old` instead of 0.
template <int CTRL, int ROW_MASK, class T>
__device__ __forceinline__ T dpp_move_or(T x, T old) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                                 __builtin_bit_cast(int, x), CTRL, ROW_MASK,
                                                                 0xf, false));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, x), o = __builtin_bit_cast(uint64_t, old);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)u, CTRL,
                                                                  ROW_MASK, 0xf, false);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32),
                                                                  (int)(uint32_t)(u >> 32), CTRL, ROW_MASK,
                                                                  0xf, false);
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}

// Inclusive scan over the wave with the operator (the sum uses the plain
// DPP scan above).
template <int CMB, class T>
__device__ __forceinline__ T wave_incl_scan_cmb(T x, bool mn) {
    if constexpr (CMB == kCmbSum) {
        return wave_incl_scan(x);
    } else {
        const T id = mm_id<T>(mn);
        x = mm_op(x, dpp_move_or<DPP_ROW_SHR1, 0xf>(x, id), mn);
        x = mm_op(x, dpp_move_or<DPP_ROW_SHR2, 0xf>(x, id), mn);
        x = mm_op(x, dpp_move_or<DPP_ROW_SHR4, 0xf>(x, id), mn);
        x = mm_op(x, dpp_move_or<DPP_ROW_SHR8, 0xf>(x, id), mn);
        x = mm_op(x, dpp_move_or<DPP_ROW_BCAST15, 0xa>(x, id), mn);
        x = mm_op(x, dpp_move_or<DPP_ROW_BCAST31, 0xc>(x, id), mn);
        return x;
    }
}

template <int CMB, class T>
__device__ __forceinline__ T wave_reduce_cmb(T x, bool mn) {
    return readlane(wave_incl_scan_cmb<CMB>(x, mn), 63);
}

// ---------------------------------------------------------------------------
// Error-free transformations (binary32)
// ---------------------------------------------------------------------------

// Knuth's TwoSum: s + e == a + b exactly, s = fl(a + b).
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    float bb = s - a;
    float aa = s - bb;
    e = (a - aa) + (b - bb);
}

// FMA-based TwoProduct: p + e == a * b exactly, p = fl(a * b).
__device__ __forceinline__ void two_prod(float a, float b, float& p, float& e) {
    p = a * b;
    e = __builtin_fmaf(a, b, -p);
}

// Compensated binary32 accumulation of the view values of loaded elements
// into (s, c): s is the running binary32 sum, c collects the exact rounding
// errors of the products (TwoProduct) and of the additions (TwoSum). The
// product of two bfloat16 values has at most 16 significant bits and is
// exact in binary32 (barring underflow below 2^-110, where TwoProduct's
// error term is itself rounded), so its error term is not formed.
template <int IDT, int OP, int SLOTS>
__device__ __forceinline__ void comp_accumulate(const vec<IDT> (&x)[SLOTS], const vec<IDT> (&y)[SLOTS], float alpha,
                                                float& s, float& c) {
    constexpr int V = vwidth<IDT>();
    constexpr bool EXACT_PROD = IDT == DR_BF16 && (OP == DR_OP_SQUARE || OP == DR_OP_MUL);
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const float x0 = decode<IDT>(x[q].e[e]);
            float p, pe = 0.0f;
            if constexpr (OP == DR_OP_IDENTITY) {
                p = x0;
            } else if constexpr (OP == DR_OP_SQUARE) {
                if constexpr (EXACT_PROD) p = x0 * x0;
                else two_prod(x0, x0, p, pe);
            } else if constexpr (OP == DR_OP_MUL) {
                const float x1 = decode<IDT>(y[q].e[e]);
                if constexpr (EXACT_PROD) p = x0 * x1;
                else two_prod(x0, x1, p, pe);
            } else {   // axpy: x0 + alpha * x1
                float m, me, r;
                two_prod(alpha, decode<IDT>(y[q].e[e]), m, me);
                two_sum(x0, m, p, r);
                pe = r + me;
            }
            float err;
            two_sum(s, p, s, err);
            if constexpr (OP == DR_OP_IDENTITY || EXACT_PROD) c += err;
            else c += err + pe;
        }
    }
}

// Plain binary32 accumulation of the view values into s (one rounding per
// operation; the product of a mul view is rounded before the sum).
template <int IDT, int OP, int SLOTS>
__device__ __forceinline__ void plain_accumulate(const vec<IDT> (&x)[SLOTS], const vec<IDT> (&y)[SLOTS], float alpha,
                                                 float& s) {
    constexpr int V = vwidth<IDT>();
    constexpr bool ZIP = (OP == DR_OP_MUL || OP == DR_OP_AXPY);
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const float x0 = decode<IDT>(x[q].e[e]);
            const float x1 = ZIP ? decode<IDT>(y[q].e[e]) : 0.0f;
            float v;
            if constexpr (OP == DR_OP_IDENTITY) v = x0;
            else if constexpr (OP == DR_OP_SQUARE) v = x0 * x0;
            else if constexpr (OP == DR_OP_MUL) v = x0 * x1;
            else {
                const float t = alpha * x1;
                v = x0 + t;
            }
            s += v;
        }
    }
}

// (s, c) += (s2, c2) for compensated pairs: TwoSum of the two sums, and the
// new rounding error with both error terms into c, in a fixed order.
__device__ __forceinline__ void pair_add(float& s, float& c, float s2, float c2) {
    float e;
    two_sum(s, s2, s, e);
    c = c + (c2 + e);
}

// Sum of the lanes' compensated pairs over the wave, over a fixed tree
// (pair_add at every level; lanes without a partner add (0, 0), exactly);
// the result in every lane.
__device__ __forceinline__ void wave_sum_pair(float& s, float& c) {
    pair_add(s, c, dpp_move<DPP_ROW_SHR1, 0xf>(s), dpp_move<DPP_ROW_SHR1, 0xf>(c));
    pair_add(s, c, dpp_move<DPP_ROW_SHR2, 0xf>(s), dpp_move<DPP_ROW_SHR2, 0xf>(c));
    pair_add(s, c, dpp_move<DPP_ROW_SHR4, 0xf>(s), dpp_move<DPP_ROW_SHR4, 0xf>(c));
    pair_add(s, c, dpp_move<DPP_ROW_SHR8, 0xf>(s), dpp_move<DPP_ROW_SHR8, 0xf>(c));
    pair_add(s, c, dpp_move<DPP_ROW_BCAST15, 0xa>(s), dpp_move<DPP_ROW_BCAST15, 0xa>(c));
    pair_add(s, c, dpp_move<DPP_ROW_BCAST31, 0xc>(s), dpp_move<DPP_ROW_BCAST31, 0xc>(c));
    s = readlane(s, 63);
    c = readlane(c, 63);
}

// A compensated pair widened to binary64 (s + c, exact unless the
// exponents of s and c are more than 29 apart; a non-finite sum is
// returned as is).
__device__ __forceinline__ double pair_widen(float s, float c) {
    return __builtin_isfinite(s) ? (double)s + (double)c : (double)s;
}

// Partial of a workgroup of WAVES waves in binary64, from the per-thread
// binary32 accumulators: the waves' sums (compensated pairs or plain
// sums), then the waves in order in thread 0, all in binary32; only the
// workgroup's result is widened. Every thread must call it; the result is
// valid in thread 0. `sp`/`cp` are WAVES floats of LDS each.
template <bool COMP, int WAVES>
__device__ __forceinline__ double block_partial_f32(float s, float c, float* sp, float* cp) {
    const int w = threadIdx.x >> 6;
    if constexpr (COMP) wave_sum_pair(s, c);
    else s = readlane(wave_incl_scan(s), 63);
    if (lane_id() == 0) {
        sp[w] = s;
        if constexpr (COMP) cp[w] = c;
    }
    __syncthreads();
    double part = 0.0;
    if (threadIdx.x == 0) {
        float ts = sp[0], tc = COMP ? cp[0] : 0.0f;
        for (int i = 1; i < WAVES; ++i) {
            if constexpr (COMP) pair_add(ts, tc, sp[i], cp[i]);
            else ts += sp[i];
        }
        part = COMP ? pair_widen(ts, tc) : (double)ts;
    }
    return part;
}

// ---------------------------------------------------------------------------
// Cross-workgroup status words
// ---------------------------------------------------------------------------
//
// A 64-bit value published by one workgroup and read by others is stored as
// two 64-bit words, each = (tag << 32) | 32 bits of the value. The tag is
// the launch epoch, so words written by earlier launches never look valid
// and the workspace needs no clearing between launches. Every access is an
// agent-scope atomic, which keeps it coherent across the eight XCDs' L2s
// without fences; a reader accepts the value only when both tags match.

__device__ __forceinline__ uint64_t atomic_ld(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_st(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t atomic_ld32(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_st32(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t atomic_add32(uint32_t* p, uint32_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_or32(uint32_t* p, uint32_t v) {
    __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void tagged_store(uint64_t* w, uint32_t tag, uint64_t v) {
    atomic_st(w, ((uint64_t)tag << 32) | (uint32_t)v);
    atomic_st(w + 1, ((uint64_t)tag << 32) | (uint32_t)(v >> 32));
}

// Returns true and the value when both halves carry `tag`.
__device__ __forceinline__ bool tagged_load(const uint64_t* w, uint32_t tag, uint64_t& v) {
    uint64_t a = atomic_ld(w);
    uint64_t b = atomic_ld(w + 1);
    v = (uint64_t)(uint32_t)a | ((uint64_t)(uint32_t)b << 32);
    return (uint32_t)(a >> 32) == tag && (uint32_t)(b >> 32) == tag;
}

template <class T> __device__ __forceinline__ uint64_t to_bits(T v) {
    if constexpr (sizeof(T) == 8) return __builtin_bit_cast(uint64_t, v);
    else return (uint64_t)__builtin_bit_cast(uint32_t, v);
}
template <class T> __device__ __forceinline__ T from_bits(uint64_t b) {
    if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, b);
    else return __builtin_bit_cast(T, (uint32_t)b);
}

// Bounded spin: true while the deadline (wall clock, 100 MHz) is not past.
__device__ __forceinline__ uint64_t now_ticks() { return wall_clock64(); }

__device__ __forceinline__ Header* header(uint8_t* ws) { return (Header*)ws; }

__device__ __forceinline__ uint32_t epoch_tag(uint32_t epoch) {
    return (epoch % 0xFFFFFFFEu) + 1u;   // never 0 (fresh workspace) nor ~0
}

// Record a device-detected fault: in the launch's workspace (when it has
// one) and in the device's library-wide fault word, so that a call made
// without a workspace can report it too (dr_check_device_error).
__device__ __forceinline__ void flag_error(const LaunchArgs& a, uint32_t bit) {
    if (a.ws != nullptr) atomic_or32(&header(a.ws)->error, bit);
    if (a.gfault != nullptr) atomic_or32(a.gfault, bit);
}

// Tag of the running launch: the prologue kernel that precedes every
// launch using tags has already bumped the workspace epoch (and zeroed the
// launch's arrival counters), so a plain load, ordered after the prologue by
// the stream, gives every workgroup the same value without any atomic.
__device__ __forceinline__ uint32_t begin_launch(const uint8_t* ws) {
    return epoch_tag(((const Header*)ws)->epoch);
}

// ---------------------------------------------------------------------------
// Segment / tile geometry
// ---------------------------------------------------------------------------
//
// A segment of n elements whose first input starts `a` elements past a
// 16-byte boundary is covered by tiles in a shifted index u = j + a: tile s
// holds u in [s*TILE, (s+1)*TILE). Every tile but the first starts on a
// 16-byte boundary of every pointer of the row, so interior vectors are
// whole aligned 16-byte accesses. A row whose pointers are misaligned
// relative to each other gets a = 0 and element-wise access (vec_ok = 0).
// Tiles never straddle segments; the tiles of all segments are numbered
// consecutively in segment order ("physical" tile index).

struct SegInfo {
    const void* in0;
    const void* in1;
    const void* in2;
    const void* in3;
    void* out0;
    void* out1;
    int64_t n;        // length
    int64_t first;    // physical index of the segment's first tile
    int64_t ntiles;
    int64_t k;        // segment index
    int32_t shift;    // a
    int32_t vec_ok;
};

// Shift of a row: how many elements its first input starts past a 16-byte
// boundary (0 when the pointer is not even element-aligned).
__device__ __forceinline__ int32_t row_shift(const void* in0, int ies) {
    const uintptr_t b0 = (uintptr_t)in0;
    if (b0 % ies != 0) return 0;
    return (int32_t)((b0 % 16) / ies);
}

// Load of data that no kernel writes while the reading kernel runs (table
// rows, plan words, the plan key): through the constant address space, so
// that a wave-uniform address becomes a scalar load. Scalar loads count in
// their own counter, so such a lookup does not wait behind the wave's
// outstanding tile loads.
template <class T>
__device__ __forceinline__ T ld_const(const T* p) {
    return *(const __attribute__((address_space(4))) T*)p;
}

__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The fields of a table row that the kernels use, read one by one (zips of
// at most 4 inputs and at most 2 outputs).
struct Row {
    const void* in0;
    const void* in1;
    const void* in2;
    const void* in3;
    void* out0;
    void* out1;
    int64_t n;
};

__device__ __forceinline__ Row load_row(const dr_segment* rows, int64_t k) {
    const dr_segment* p = rows + k;
    Row r;
    r.in0 = ld_const(&p->in[0]);
    r.in1 = ld_const(&p->in[1]);
    r.in2 = ld_const(&p->in[2]);
    r.in3 = ld_const(&p->in[3]);
    r.out0 = ld_const(&p->out[0]);
    r.out1 = ld_const(&p->out[1]);
    r.n = ld_const(&p->length);
    return r;
}

__device__ __forceinline__ bool aligned_at(const void* p, uintptr_t j0, int es) {
    return (((uintptr_t)p + j0 * (uintptr_t)es) % 16) == 0;
}

// Whether every pointer of the row is 16-byte aligned at the first index
// where the first input is (so whole 16-byte vectors can be used).
__device__ __forceinline__ int32_t row_vec_ok(const Row& r, int32_t shift, int arity, int nout, int ies,
                                              int oes) {
    const int V = 16 / ies;
    const uintptr_t j0 = (uintptr_t)((V - shift) % V);
    bool ok = aligned_at(r.in0, j0, ies);
    if (arity > 1) ok = ok && aligned_at(r.in1, j0, ies);
    if (arity > 2) ok = ok && aligned_at(r.in2, j0, ies);
    if (arity > 3) ok = ok && aligned_at(r.in3, j0, ies);
    if (nout > 0) ok = ok && aligned_at(r.out0, j0, oes);
    if (nout > 1) ok = ok && aligned_at(r.out1, j0, oes);
    return ok ? 1 : 0;
}

__device__ __forceinline__ int64_t tiles_of(int64_t n, int32_t shift, int64_t tile) {
    return n > 0 ? (n + shift + tile - 1) / tile : 0;
}

__device__ __forceinline__ bool row_bad(const Row& r, int arity, int nout) {
    if (r.n < 0) return true;
    if (r.n == 0) return false;
    if (r.in0 == nullptr) return true;
    if (arity > 1 && r.in1 == nullptr) return true;
    if (arity > 2 && r.in2 == nullptr) return true;
    if (arity > 3 && r.in3 == nullptr) return true;
    if (nout > 0 && r.out0 == nullptr) return true;
    if (nout > 1 && r.out1 == nullptr) return true;
    return false;
}

// The tiles of the launch as seen by one wave (every lane must call the
// methods). Small tables (m <= DR_SMALL_TABLE) are planned here, one row
// per lane; large ones read the plan dr_plan left in the workspace, whose
// key (rows, m, total, tile, input element size) must match the launch.
struct TileMap {
    int64_t total_tiles = 0;
    bool ok = false;
    // small-table state, one row per lane
    int64_t cnt = 0, incl = 0, n = 0;
    int32_t shift = 0, vec_ok = 0;
    uint32_t plan_tag = 0;   // large tables: tag of the plan words

    __device__ __forceinline__ void init(const LaunchArgs& a) {
        const int lane = lane_id();
        if (a.m <= DR_SMALL_TABLE) {
            bool bad = false;
            if (lane < a.m) {
                const Row r = load_row(a.rows, lane);
                bad = row_bad(r, a.arity, a.nout);
                if (!bad) {
                    n = r.n;
                    shift = row_shift(r.in0, a.ies);
                    vec_ok = row_vec_ok(r, shift, a.arity, a.nout, a.ies, a.oes);
                }
            }
            cnt = tiles_of(n, shift, a.tile);
            incl = wave_incl_scan(cnt);
            const int64_t nsum = wave_sum(n);
            const bool anybad = __ballot(bad) != 0;
            total_tiles = readlane(incl, 63);
            ok = !anybad && nsum == a.total && total_tiles <= a.tmax;
            if (!ok) {
                if (threadIdx.x == 0)
                    flag_error(a, (anybad || nsum != a.total) ? DR_DEVFLAG_BAD_TABLE
                                                                 : DR_DEVFLAG_TOO_MANY_TILES);
                total_tiles = 0;
            }
            return;
        }
        const Header* h = (const Header*)a.ws;
        ok = a.ws != nullptr && ld_const(&h->plan_m) == a.m &&
             ld_const(&h->plan_rows) == (uint64_t)(uintptr_t)a.rows && ld_const(&h->plan_tile) == a.tile &&
             ld_const(&h->plan_ies) == a.ies && ld_const(&h->plan_total) == a.total;
        plan_tag = ok ? ld_const(&h->plan_tag) : 0u;
        if (!ok) {
            if (threadIdx.x == 0) flag_error(a, DR_DEVFLAG_PLAN);
            return;
        }
        total_tiles = ld_const(&h->plan_tiles);
        if (total_tiles > a.tmax) {
            if (threadIdx.x == 0) flag_error(a, DR_DEVFLAG_TOO_MANY_TILES);
            total_tiles = 0;
            ok = false;
        }
    }

    // Segment owning physical tile t (0 <= t < total_tiles). Returns false
    // (and flags the fault) when the row lacks a pointer the launch needs.
    __device__ __forceinline__ bool find(const LaunchArgs& a, int64_t t, SegInfo& si) const {
        int k;
        if (a.m <= DR_SMALL_TABLE) {
            const uint64_t le = __ballot(lane_id() < a.m && incl <= t);
            k = __builtin_popcountll(le);   // segments ending at or before tile t
            si.first = readlane(incl - cnt, k);
            si.ntiles = readlane(cnt, k);
            si.n = readlane(n, k);
            si.shift = readlane(shift, k);
            si.vec_ok = readlane(vec_ok, k);
        } else {
            const uint64_t* F = (const uint64_t*)(a.ws + a.lay.off_plan_first);
            const uint64_t* tseg = (const uint64_t*)(a.ws + a.lay.off_plan_tseg);
            const uint64_t wk = ld_const(tseg + uniform64(t));
            const uint32_t kk = (uint32_t)wk;
            const bool kok = (uint32_t)(wk >> 32) == plan_tag && (int64_t)kk < a.m;
            const uint64_t f0 = kok ? ld_const(F + kk) : 0, f1 = kok ? ld_const(F + kk + 1) : 0;
            if (!kok || (uint32_t)(f0 >> 32) != plan_tag || (uint32_t)(f1 >> 32) != plan_tag) {
                if (threadIdx.x == 0) flag_error(a, DR_DEVFLAG_PLAN);
                return false;
            }
            k = (int)kk;
            si.first = (uint32_t)f0;
            si.ntiles = (int64_t)(uint32_t)f1 - (int64_t)(uint32_t)f0;
            const Row r = load_row(a.rows, k);
            if (row_bad(r, a.arity, a.nout)) {
                if (threadIdx.x == 0) flag_error(a, DR_DEVFLAG_BAD_TABLE);
                return false;
            }
            si.n = r.n;
            si.shift = row_shift(r.in0, a.ies);
            si.vec_ok = row_vec_ok(r, si.shift, a.arity, a.nout, a.ies, a.oes);
        }
        si.k = k;
        const Row r = load_row(a.rows, k);
        si.in0 = r.in0;
        si.in1 = r.in1;
        si.in2 = r.in2;
        si.in3 = r.in3;
        si.out0 = r.out0;
        si.out1 = r.out1;
        return true;
    }
};

// Bounded wait helper.
struct Deadline {
    uint64_t end;
    __device__ __forceinline__ explicit Deadline(uint64_t ticks) : end(now_ticks() + ticks) {}
    __device__ __forceinline__ bool passed() const { return now_ticks() > end; }
};

// ---------------------------------------------------------------------------
// Tile access
// ---------------------------------------------------------------------------
//
// A tile of TILE = 256 * ITEMS elements is SLOTS = ITEMS / V vectors per
// thread. Wave w owns the contiguous run of vectors [w*SLOTS*64,
// (w+1)*SLOTS*64) of the tile, and slot s of lane l is vector
// (w*SLOTS + s)*64 + l: each load instruction of a wave covers 1 KiB of
// consecutive memory. In reverse mode the vector order of the tile is
// mirrored (vector p in processing order is vector NV-1-p in memory).

template <int DT> __device__ __forceinline__ typename elem<DT>::T zero_elem() {
    return (typename elem<DT>::T)0;
}

// True when the whole tile lies inside its segment and every pointer of the
// row is 16-byte aligned there: all accesses are whole 16-byte vectors with
// no bounds checks (the common case; only a segment's first and last tiles,
// and misaligned rows, take the checked path).
template <int V, int SLOTS, int BLOCK = kBlock>
__device__ __forceinline__ bool tile_full(const SegInfo& si, int64_t u0) {
    constexpr int64_t TILE = (int64_t)BLOCK * SLOTS * V;
    const int64_t j0 = u0 - si.shift;
    return si.vec_ok && j0 >= 0 && j0 + TILE <= si.n;
}

// The slots of a full tile (tile_full): whole vectors, no checks.
template <int DT, int SLOTS, int V = vwidth<DT>(), bool NT = true, int BLOCK = kBlock>
__device__ __forceinline__ void load_slots_full(vec<DT, V> (&x)[SLOTS], const void* base, const SegInfo& si,
                                                int64_t u0, int w, int l, bool rev) {
    using R = typename vbits<V * esize<DT>()>::T;
    constexpr int64_t NV = (int64_t)BLOCK * SLOTS;
    const int64_t p0 = (int64_t)(w * SLOTS) * 64 + l;
    const int64_t q0 = rev ? (NV - 1 - p0) : p0;
    const char* b = (const char*)base + (u0 - si.shift + q0 * V) * esize<DT>();
    const int64_t step = rev ? -64 * (int64_t)sizeof(R) : 64 * (int64_t)sizeof(R);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        R wv = NT ? __builtin_nontemporal_load((const R*)(b + s * step)) : *(const R*)(b + s * step);
        __builtin_memcpy(&x[s], &wv, sizeof(R));
    }
}

// The slots of any tile, each element checked against the segment (the
// elements outside it read as 0).
template <int DT, int SLOTS, int V = vwidth<DT>(), bool NT = true, int BLOCK = kBlock>
__device__ __forceinline__ void load_slots_checked(vec<DT, V> (&x)[SLOTS], const void* base, const SegInfo& si,
                                                   int64_t u0, int w, int l, bool rev) {
    constexpr int64_t NV = (int64_t)BLOCK * SLOTS;
    const int64_t p0 = (int64_t)(w * SLOTS) * 64 + l;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int64_t p = p0 + (int64_t)s * 64;
        const int64_t q = rev ? (NV - 1 - p) : p;
        const int64_t j = u0 + q * V - si.shift;
        if (si.vec_ok && j >= 0 && j + V <= si.n) {
            x[s] = load_vec<DT, V, NT>(base, j);
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int64_t jj = j + e;
                typename elem<DT>::T v = zero_elem<DT>();
                if (jj >= 0 && jj < si.n) v = load_one<DT>(base, jj);
                x[s].e[e] = v;
            }
        }
    }
}

template <int DT, int SLOTS, int V = vwidth<DT>(), bool NT = true, int BLOCK = kBlock>
__device__ __forceinline__ void load_slots(vec<DT, V> (&x)[SLOTS], const void* base, const SegInfo& si,
                                           int64_t u0, int w, int l, bool rev) {
    if (tile_full<V, SLOTS, BLOCK>(si, u0)) load_slots_full<DT, SLOTS, V, NT, BLOCK>(x, base, si, u0, w, l, rev);
    else load_slots_checked<DT, SLOTS, V, NT, BLOCK>(x, base, si, u0, w, l, rev);
}

// The two inputs of a zipped view (y only when ZIP) under one branch on
// tile_full, so that a full tile issues both inputs' loads before any wait
// (see load_slots_k).
template <bool ZIP, int DT, int SLOTS, int V = vwidth<DT>(), int BLOCK = kBlock>
__device__ __forceinline__ void load_pair(vec<DT, V> (&x)[SLOTS], vec<DT, V> (&y)[SLOTS], const SegInfo& si,
                                          int64_t u0, int w, int l, bool rev) {
    if (tile_full<V, SLOTS, BLOCK>(si, u0)) {
        load_slots_full<DT, SLOTS, V, true, BLOCK>(x, si.in0, si, u0, w, l, rev);
        if constexpr (ZIP) load_slots_full<DT, SLOTS, V, true, BLOCK>(y, si.in1, si, u0, w, l, rev);
    } else {
        load_slots_checked<DT, SLOTS, V, true, BLOCK>(x, si.in0, si, u0, w, l, rev);
        if constexpr (ZIP) load_slots_checked<DT, SLOTS, V, true, BLOCK>(y, si.in1, si, u0, w, l, rev);
    }
}

// load_slots with the tile's fullness known at compile time. A kernel that
// loads several inputs calls this for each inside one branch on tile_full,
// so the loads of a full tile are all issued before the first wait (with a
// branch inside each call, the compiler joins the unchecked loads of one
// input with the checked ones before the next input's, and that join waits
// for every load in flight: the vector memory counter is in order).
template <bool FULL, int DT, int SLOTS, int V = vwidth<DT>(), int BLOCK = kBlock>
__device__ __forceinline__ void load_slots_k(vec<DT, V> (&x)[SLOTS], const void* base, const SegInfo& si,
                                             int64_t u0, int w, int l, bool rev) {
    if constexpr (FULL) load_slots_full<DT, SLOTS, V, true, BLOCK>(x, base, si, u0, w, l, rev);
    else load_slots<DT, SLOTS, V, true, BLOCK>(x, base, si, u0, w, l, rev);
}

// Whether element e (memory order) of slot s of lane l of wave w lies
// inside the segment; the loads fill the others with 0, which only a sum may
// combine.
template <int V, int SLOTS, int BLOCK = kBlock>
__device__ __forceinline__ bool elem_in(const SegInfo& si, int64_t u0, int w, int l, int s, int e, bool rev) {
    constexpr int64_t NV = (int64_t)BLOCK * SLOTS;
    const int64_t p = (int64_t)(w * SLOTS + s) * 64 + l;
    const int64_t q = rev ? (NV - 1 - p) : p;
    const int64_t j = u0 + q * V - si.shift + e;
    return j >= 0 && j < si.n;
}

// Store the V outputs of slot s (given in memory order). `full` is
// tile_full() of the tile.
template <class OT, int V, int SLOTS, int BLOCK = kBlock>
__device__ __forceinline__ void store_slot(void* base, const SegInfo& si, int64_t u0, int w, int l,
                                           int s, bool rev, bool full, const OT (&o)[V]) {
    constexpr int64_t NV = (int64_t)BLOCK * SLOTS;
    const int64_t p = (int64_t)(w * SLOTS + s) * 64 + l;
    const int64_t q = rev ? (NV - 1 - p) : p;
    const int64_t j = u0 + q * V - si.shift;
    if (full || (si.vec_ok && j >= 0 && j + V <= si.n)) {
        store_run<OT, V>(base, j, o);
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const int64_t jj = j + e;
            if (jj >= 0 && jj < si.n) ((OT*)base)[jj] = o[e];
        }
    }
}

// store_slot with the tile's fullness known at compile time: a full tile
// (whole in its segment, rows aligned) stores each slot as one unchecked
// vector, so the kernel branches once per tile rather than once per slot.
template <bool FULL, class OT, int V, int SLOTS, int BLOCK = kBlock>
__device__ __forceinline__ void store_slot_k(void* base, const SegInfo& si, int64_t u0, int w, int l, int s,
                                             bool rev, const OT (&o)[V]) {
    if constexpr (FULL) {
        constexpr int64_t NV = (int64_t)BLOCK * SLOTS;
        const int64_t p = (int64_t)(w * SLOTS + s) * 64 + l;
        const int64_t q = rev ? (NV - 1 - p) : p;
        store_run<OT, V>(base, u0 + q * V - si.shift, o);
    } else {
        store_slot<OT, V, SLOTS, BLOCK>(base, si, u0, w, l, s, rev, false, o);
    }
}

// Mirror the element order of a small register array when `rev` (static
// indices, so the compiler emits selects rather than indexed registers).
template <class T, int V>
__device__ __forceinline__ void mirror_if(T (&v)[V], bool rev) {
#pragma unroll
    for (int e = 0; e < V / 2; ++e) {
        T a = v[e], b = v[V - 1 - e];
        v[e] = rev ? b : a;
        v[V - 1 - e] = rev ? a : b;
    }
}

// ---------------------------------------------------------------------------
// View transforms
// ---------------------------------------------------------------------------

// Value of the view in the accumulation type of a reduction/scan (the
// product of two binary32 values is formed in binary32 here; the
// compensated reduction recovers its rounding error separately).
template <int OP, class A>
__device__ __forceinline__ A view_apply(A x0, A x1, A alpha) {
    if constexpr (OP == DR_OP_IDENTITY) return x0;
    else if constexpr (OP == DR_OP_SQUARE) return x0 * x0;
    else if constexpr (OP == DR_OP_MUL) return x0 * x1;
    else return x0 + alpha * x1;
}

}  // namespace dr
