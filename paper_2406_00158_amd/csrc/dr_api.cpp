// dr_api.cpp — host side of the C ABI declared in include/dr.h: argument
// checks, workspace layout, kernel selection and launch. Every entry point
// checks everything it can on the host before enqueuing anything, and
// returns a dr_status; nothing throws across the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "dr.h"
#include "dr_internal.hpp"

namespace {

using namespace dr;

thread_local std::string g_err;

dr_status fail(dr_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

dr_status ok() {
    g_err.clear();
    return DR_OK;
}

dr_status hip_fail(hipError_t e, const char* what) {
    return fail(DR_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int dtype_size(int dt) {
    switch (dt) {
    case DR_I32: return 4;
    case DR_F32: return 4;
    case DR_BF16: return 2;
    case DR_F64: return 8;
    case DR_I64: return 8;
    default: return 0;
    }
}

int op_arity(int op) {
    switch (op) {
    case DR_OP_IDENTITY: return 1;
    case DR_OP_SQUARE: return 1;
    case DR_OP_MUL: return 2;
    case DR_OP_AXPY: return 2;
    case DR_OP_BLACK_SCHOLES: return 4;
    default: return 0;
    }
}

uint64_t align256(uint64_t v) { return (v + 255) & ~(uint64_t)255; }

// Items per thread without a tuning: 16, except bfloat16 reductions, which
// take 32 (the same 64 bytes per thread and input as a binary32 tile; the
// bfloat16 dot product was measured 12 % faster than with 16).
int default_items(int algo, int in_dt) {
    return (algo == DR_ALGO_REDUCE && in_dt == DR_BF16) ? 32 : 16;
}

// Bound of the wait loops, in wall-clock ticks (about 2.7 s at 100 MHz);
// DR_SPIN_TICKS overrides it (tests of the timeout path), read at every call.
uint64_t spin_ticks() {
    const char* e = std::getenv("DR_SPIN_TICKS");
    if (e && *e) return (uint64_t)std::strtoull(e, nullptr, 10);
    return (uint64_t)1 << 28;
}

dr_status check_view(const dr_view* v, bool int_ok) {
    if (!v) return fail(DR_ERR_INVALID_ARG, "view is NULL");
    if (v->reserved != 0) return fail(DR_ERR_INVALID_ARG, "view.reserved must be 0");
    const int ar = op_arity(v->op);
    if (ar == 0) return fail(DR_ERR_INVALID_ARG, "unknown op %d", (int)v->op);
    if (v->arity != ar)
        return fail(DR_ERR_INVALID_ARG, "view arity %d does not match op %d (arity %d)", (int)v->arity,
                    (int)v->op, ar);
    if (v->in_dtype != DR_I32 && v->in_dtype != DR_F32 && v->in_dtype != DR_BF16 && v->in_dtype != DR_F64)
        return fail(DR_ERR_UNSUPPORTED, "input dtype %d is not supported", (int)v->in_dtype);
    if (v->in_dtype == DR_I32) {
        if (!int_ok) return fail(DR_ERR_UNSUPPORTED, "int32 inputs are not supported by this call");
        if (v->op == DR_OP_AXPY && (v->alpha != std::floor(v->alpha) || std::fabs(v->alpha) > 2147483647.0))
            return fail(DR_ERR_INVALID_ARG, "int32 axpy needs an integer alpha");
    }
    if (!std::isfinite(v->alpha) && v->op == DR_OP_AXPY)
        return fail(DR_ERR_INVALID_ARG, "alpha must be finite");
    return DR_OK;
}

dr_status check_table(const dr_table* t) {
    if (!t) return fail(DR_ERR_INVALID_ARG, "table is NULL");
    if (t->reserved != 0) return fail(DR_ERR_INVALID_ARG, "table.reserved must be 0");
    if (t->n_segments < 0) return fail(DR_ERR_INVALID_ARG, "n_segments < 0");
    if (t->n_segments > INT32_MAX) return fail(DR_ERR_UNSUPPORTED, "more than 2^31-1 segments");
    if (t->total_length < 0) return fail(DR_ERR_INVALID_ARG, "total_length < 0");
    if (t->total_length >= ((int64_t)1 << 40)) return fail(DR_ERR_UNSUPPORTED, "total_length >= 2^40");
    if (t->mode != DR_MODE_CONCAT && t->mode != DR_MODE_BATCH)
        return fail(DR_ERR_INVALID_ARG, "unknown mode %d", (int)t->mode);
    if (t->n_segments > 0 && !t->rows) return fail(DR_ERR_INVALID_ARG, "rows is NULL");
    return DR_OK;
}

struct Interval {
    uintptr_t lo, hi;   // [lo, hi)
    int64_t row;
    int kind;           // 0 input, 1 output
};

// Host mirror checks: lengths, NULLs, element alignment, sum, overlap.
dr_status check_host_rows(const dr_table* t, int arity, int nout, int ies, int oes, bool inplace_ok) {
    const dr_segment* r = t->host_rows;
    if (!r) return DR_OK;
    int64_t sum = 0;
    std::vector<Interval> iv;
    iv.reserve((size_t)t->n_segments * (arity + nout));
    for (int64_t k = 0; k < t->n_segments; ++k) {
        const dr_segment& s = r[k];
        if (s.reserved != 0) return fail(DR_ERR_INVALID_ARG, "row %lld: reserved must be 0", (long long)k);
        if (s.length < 0) return fail(DR_ERR_INVALID_ARG, "row %lld: negative length", (long long)k);
        sum += s.length;
        if (s.length == 0) continue;
        for (int i = 0; i < arity; ++i) {
            if (!s.in[i]) return fail(DR_ERR_INVALID_ARG, "row %lld: in[%d] is NULL", (long long)k, i);
            if ((uintptr_t)s.in[i] % ies)
                return fail(DR_ERR_INVALID_ARG, "row %lld: in[%d] is not aligned to its element size",
                            (long long)k, i);
            iv.push_back({(uintptr_t)s.in[i], (uintptr_t)s.in[i] + (uintptr_t)s.length * ies, k, 0});
        }
        for (int i = 0; i < nout; ++i) {
            if (!s.out[i]) return fail(DR_ERR_INVALID_ARG, "row %lld: out[%d] is NULL", (long long)k, i);
            if ((uintptr_t)s.out[i] % oes)
                return fail(DR_ERR_INVALID_ARG, "row %lld: out[%d] is not aligned to its element size",
                            (long long)k, i);
            iv.push_back({(uintptr_t)s.out[i], (uintptr_t)s.out[i] + (uintptr_t)s.length * oes, k, 1});
        }
    }
    if (sum != t->total_length)
        return fail(DR_ERR_INVALID_ARG, "total_length %lld != sum of lengths %lld",
                    (long long)t->total_length, (long long)sum);
    if (nout == 0) return DR_OK;
    // an output may coincide exactly with an input of its own row (in place,
    // same element size); any other overlap that involves an output is an error
    std::sort(iv.begin(), iv.end(), [](const Interval& a, const Interval& b) { return a.lo < b.lo; });
    for (size_t i = 0; i < iv.size(); ++i) {
        for (size_t j = i + 1; j < iv.size() && iv[j].lo < iv[i].hi; ++j) {
            const Interval &a = iv[i], &b = iv[j];
            if (a.kind == 0 && b.kind == 0) continue;   // inputs may overlap each other
            const bool same = a.lo == b.lo && a.hi == b.hi && a.row == b.row && a.kind != b.kind;
            if (same && inplace_ok && ies == oes) continue;
            return fail(DR_ERR_INVALID_ARG, "row %lld: an output overlaps %s of row %lld",
                        (long long)(a.kind ? a.row : b.row), (a.kind && b.kind) ? "an output" : "an input",
                        (long long)(a.kind ? b.row : a.row));
        }
    }
    return DR_OK;
}

// Items per thread and workgroup size of a call: the defaults, or the
// tuning's. 512- and 1024-thread workgroups run the look-back scan only.
dr_status resolve_shape(const dr_tuning* tu, int algo, int in_dt, int& items, int& block) {
    items = default_items(algo, in_dt);
    block = kBlock;
    if (!tu) return DR_OK;
    const int32_t forms = DR_TUNE_TILE_PER_BLOCK | DR_TUNE_SPECIALIZED | DR_TUNE_TWO_PASS | DR_TUNE_CHAINED;
    if ((tu->flags & ~forms) || tu->reserved) return fail(DR_ERR_INVALID_ARG, "unknown tuning bits");
    const int32_t f = tu->flags & forms;
    if (f & (f - 1)) return fail(DR_ERR_INVALID_ARG, "at most one form flag (DR_TUNE_*) per call");
    if (tu->block_threads != 0 && tu->block_threads != kBlock) {
        if (tu->block_threads != 512 && tu->block_threads != 1024)
            return fail(DR_ERR_UNSUPPORTED, "block_threads must be 256, 512 or 1024");
        if ((algo != DR_ALGO_SCAN && algo != DR_ALGO_SCAN_REDUCE) || f != DR_TUNE_TILE_PER_BLOCK)
            return fail(DR_ERR_UNSUPPORTED, "block_threads %d: only the look-back scan (DR_TUNE_TILE_PER_BLOCK) "
                                            "is built with more than %d threads", (int)tu->block_threads, kBlock);
        block = tu->block_threads;
    }
    if (tu->items_per_thread != 0) items = tu->items_per_thread;
    return DR_OK;
}

int64_t tmax_for(int64_t m, int64_t total, int64_t tile, int ies) {
    const int V = 16 / ies;
    const int64_t t = (total + m * (int64_t)(V - 1) + tile - 1) / tile + m;
    return t < 1 ? 1 : t;
}

bool uses_combine(int algo) { return algo == DR_ALGO_REDUCE || algo == DR_ALGO_SCAN_REDUCE; }

WsLayout layout_for(int algo, int64_t m, int64_t tmax) {
    WsLayout L{};
    uint64_t off = kFixedBytes;
    L.off_plan_first = off;
    if (m > DR_SMALL_TABLE) off += align256((uint64_t)(m + 1) * 8);
    L.off_plan_tseg = off;
    if (m > DR_SMALL_TABLE) off += align256((uint64_t)tmax * 8);
    L.tile_words = algo == DR_ALGO_REDUCE ? 2 : algo == DR_ALGO_SCAN ? 4 : algo == DR_ALGO_SCAN_REDUCE ? 6 : 0;
    L.part_word = algo == DR_ALGO_REDUCE ? 0 : 4;
    L.off_tile = off;
    off += align256((uint64_t)tmax * L.tile_words * 8);
    const uint64_t ngroups = uses_combine(algo) ? (uint64_t)(tmax / kGroupTiles + m + 2) : 0;
    L.ngroups = ngroups;
    L.off_gcnt = off;
    off += align256(ngroups * 4);
    L.off_gpart = off;
    off += align256(ngroups * 16);
    const uint64_t nunits = uses_combine(algo) ? (uint64_t)std::max<int64_t>(m, 1) : 0;
    L.nunits = nunits;
    L.off_ucnt = off;
    off += align256(nunits * 4);
    L.off_chunk = off;
    const bool scan = algo == DR_ALGO_SCAN || algo == DR_ALGO_SCAN_REDUCE;
    if (scan) off += align256((uint64_t)(4 + 4 * kMaxChunks) * 8);
    // chained single pass: chunks of at least one tile, so at most
    // ceil(tmax / kChainSB) superblocks
    L.npipe = scan ? (uint64_t)(1 + (tmax + kChainSB - 1) / kChainSB + 1) : 0;
    L.off_pipe = off;
    off += align256(L.npipe * 4);
    L.off_pipe_e = off;
    off += align256(L.npipe * 16);
    L.bytes = off;
    return L;
}

// Everything a launch needs besides the kernel.
struct Prepared {
    LaunchArgs a;
    int64_t grid;
    int block;   // threads per workgroup
};

dr_status prepare(const dr_table* t, int algo, int in_dt, int out_dt, int arity, int nout,
                  const dr_tuning* tu, void* ws, size_t ws_bytes, bool ws_required, bool inplace_ok,
                  Prepared& p, int& items) {
    dr_status s = check_table(t);
    if (s) return s;
    const int ies = dtype_size(in_dt);
    const int oes = nout > 0 ? dtype_size(out_dt) : 0;
    s = check_host_rows(t, arity, nout, ies, oes, inplace_ok);
    if (s) return s;
    int block = kBlock;
    s = resolve_shape(tu, algo, in_dt, items, block);
    if (s) return s;
    const int V = 16 / ies;
    if (items <= 0 || items % V != 0) return fail(DR_ERR_UNSUPPORTED, "items_per_thread %d", items);
    const int64_t tile = (int64_t)block * items;
    const int64_t tmax = tmax_for(t->n_segments, t->total_length, tile, ies);
    if (tmax >= ((int64_t)1 << 31)) return fail(DR_ERR_UNSUPPORTED, "too many tiles (%lld)", (long long)tmax);
    const WsLayout lay = layout_for(algo, t->n_segments, tmax);
    const bool need_ws = ws_required || t->n_segments > DR_SMALL_TABLE;
    if (need_ws && !ws) return fail(DR_ERR_WORKSPACE, "a workspace is required");
    if (ws) {   // an optional workspace, once given, is used and checked like a required one
        if ((uintptr_t)ws % 256) return fail(DR_ERR_WORKSPACE, "workspace must be 256-byte aligned");
        if (ws_bytes < lay.bytes)
            return fail(DR_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %llu needed", ws_bytes,
                        (unsigned long long)lay.bytes);
    }
    LaunchArgs& a = p.a;
    std::memset(&a, 0, sizeof a);
    a.rows = t->rows;
    a.m = t->n_segments;
    a.total = t->total_length;
    a.tile = tile;
    a.tmax = tmax;
    a.ies = ies;
    a.oes = oes;
    a.mode = t->mode;
    a.arity = arity;
    a.nout = nout;
    a.ws = (uint8_t*)ws;
    a.lay = lay;
    a.spin_ticks = spin_ticks();
    p.grid = tmax;
    p.block = block;
    return DR_OK;
}

}  // namespace

dr_status dr::set_error(dr_status s, const char* fmt, ...) {
    char buf[768];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

int dr::resident_grid(const void* kernel, int threads) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess) per = 1;
    return std::max(cus, 1) * std::max(per, 1);
}

namespace {

// The device fault word of the stream's device (the first HIP call of an
// entry point: every host-side check has passed by then).
dr_status bind_device(Prepared& p, void* stream) {
    DeviceGlobals dg;
    const hipError_t e = device_globals((hipStream_t)stream, dg);
    if (e != hipSuccess) return hip_fail(e, "device fault word lookup");
    p.a.gfault = dg.fault;
    return DR_OK;
}

dr_status launch(LaunchFn fn, Prepared& p, void* stream, const char* what) {
    dr_status s = bind_device(p, stream);
    if (s) return s;
    hipError_t e = fn(p.a, p.grid, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, what);
    return ok();
}

// The sum-scan kernel of a call: the 256-thread kernels (every form) at the
// usual tiles, else a shape built for the look-back form only
// (k_scan_wide.hip), which the call must have asked for.
LaunchFn scan_kernel(int in, int out, int op, bool c64, int items, int block, const dr_tuning* tu) {
    if (block == kBlock)
        if (LaunchFn f = find_scan(in, out, op, c64, items)) return f;
    const bool tpb = tu && (tu->flags & DR_TUNE_TILE_PER_BLOCK);
    return tpb ? find_scan_wide(in, out, op, c64, false, 0, items, block) : nullptr;
}

LaunchFn scan_reduce_kernel(int in, int rop, int acc, int items, int block, const dr_tuning* tu) {
    if (block == kBlock)
        if (LaunchFn f = find_scan_reduce(in, rop, acc, items)) return f;
    const bool tpb = tu && (tu->flags & DR_TUNE_TILE_PER_BLOCK);
    return tpb && rop == DR_OP_MUL ? find_scan_wide(in, in, DR_OP_IDENTITY, true, true, acc, items, block) : nullptr;
}

}  // namespace

extern "C" {

int dr_abi_version(void) { return DR_ABI_VERSION; }

const char* dr_status_string(dr_status s) {
    switch (s) {
    case DR_OK: return "ok";
    case DR_ERR_INVALID_ARG: return "invalid argument";
    case DR_ERR_UNSUPPORTED: return "unsupported combination";
    case DR_ERR_WORKSPACE: return "workspace missing or too small";
    case DR_ERR_HIP: return "HIP runtime error";
    case DR_ERR_NOT_ALIGNED: return "zip inputs are not aligned";
    case DR_ERR_DEVICE: return "device-side fault flagged";
    default: return "unknown status";
    }
}

const char* dr_last_error(void) { return g_err.c_str(); }

int dr_tuning_supported(int32_t algo, const dr_view* v, int32_t out_dtype, const dr_tuning* tu) {
    if (!v) return 0;
    int items = 0, block = kBlock;
    if (resolve_shape(tu, algo, v->in_dtype, items, block) != DR_OK) return 0;
    switch (algo) {
    case DR_ALGO_FOR_EACH: return find_for_each(v->in_dtype, out_dtype, v->op, items) != nullptr;
    case DR_ALGO_REDUCE:
        return find_reduce(v->in_dtype, v->op, out_dtype /* acc */, items) != nullptr;
    case DR_ALGO_SCAN:
        if (tu && (tu->flags & DR_TUNE_CHAINED))
            return block == kBlock && find_scan_chain(v->in_dtype, out_dtype, v->op, true, items) != nullptr;
        return scan_kernel(v->in_dtype, out_dtype, v->op, true, items, block, tu) != nullptr;
    case DR_ALGO_SCAN_REDUCE:
        if (tu && (tu->flags & DR_TUNE_CHAINED)) return 0;
        return scan_reduce_kernel(v->in_dtype, DR_OP_MUL, DR_ACC_COMPENSATED, items, block, tu) != nullptr;
    case DR_ALGO_BROADCAST_MUL: return find_broadcast_mul(v->in_dtype, v->op, items) != nullptr;
    default: return 0;
    }
}

dr_status dr_workspace_bytes(int32_t algo, int64_t n_segments, int64_t total_length, const dr_view* view,
                             const dr_tuning* tuning, size_t* bytes) {
    if (!bytes) return fail(DR_ERR_INVALID_ARG, "bytes is NULL");
    if (!view) return fail(DR_ERR_INVALID_ARG, "view is NULL");
    if (algo < DR_ALGO_FOR_EACH || algo > DR_ALGO_BROADCAST_MUL) return fail(DR_ERR_INVALID_ARG, "unknown algo");
    if (n_segments < 0 || total_length < 0) return fail(DR_ERR_INVALID_ARG, "negative size");
    const int ies = dtype_size(view->in_dtype);
    if (ies == 0) return fail(DR_ERR_UNSUPPORTED, "input dtype %d", (int)view->in_dtype);
    int items = 0, block = kBlock;
    dr_status s = resolve_shape(tuning, algo, view->in_dtype, items, block);
    if (s) return s;
    if (items <= 0 || items % (16 / ies)) return fail(DR_ERR_UNSUPPORTED, "items_per_thread %d", items);
    const int64_t tmax = tmax_for(n_segments, total_length, (int64_t)block * items, ies);
    *bytes = (size_t)layout_for(algo, n_segments, tmax).bytes;
    return ok();
}

dr_status dr_workspace_init(void* ws, size_t ws_bytes, void* stream) {
    if (!ws) return fail(DR_ERR_WORKSPACE, "workspace is NULL");
    if ((uintptr_t)ws % 256) return fail(DR_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < kFixedBytes) return fail(DR_ERR_WORKSPACE, "workspace smaller than its fixed part");
    hipError_t e = launch_zero(ws, ws_bytes, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "workspace init");
    return ok();
}

dr_status dr_plan(const dr_table* table, int32_t algo, const dr_view* view, const dr_tuning* tuning, void* ws,
                  size_t ws_bytes, void* stream) {
    dr_status s = check_view(view, true);
    if (s) return s;
    if (algo < DR_ALGO_FOR_EACH || algo > DR_ALGO_BROADCAST_MUL) return fail(DR_ERR_INVALID_ARG, "unknown algo");
    Prepared p;
    int items;
    const int arity = algo == DR_ALGO_SCAN_REDUCE ? 2 : view->arity;
    s = prepare(table, algo, view->in_dtype, view->in_dtype, arity, 0, tuning, ws, ws_bytes, true, false, p,
                items);
    if (s) return s;
    if (table->n_segments <= DR_SMALL_TABLE) return ok();   // planned inside every launch
    s = bind_device(p, stream);
    if (s) return s;
    hipError_t e = launch_plan(p.a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "plan");
    return ok();
}

dr_status dr_for_each(const dr_table* table, const dr_view* view, int32_t out_dtype, void* ws, size_t ws_bytes,
                      const dr_tuning* tuning, void* stream) {
    dr_status s = check_view(view, true);
    if (s) return s;
    const int in = view->in_dtype;
    const bool bs = view->op == DR_OP_BLACK_SCHOLES;
    if (bs && (in != DR_F32 || out_dtype != DR_F32))
        return fail(DR_ERR_UNSUPPORTED, "the Black-Scholes view is built for binary32 in and out");
    if (bs && !std::isfinite(view->alpha)) return fail(DR_ERR_INVALID_ARG, "the rate (alpha) must be finite");
    const bool okpair = (in == DR_F32 && out_dtype == DR_F32) || (in == DR_BF16 && out_dtype == DR_F32) ||
                        (in == DR_F64 && out_dtype == DR_F64) || (in == DR_I32 && out_dtype == DR_I32) ||
                        (in == DR_I32 && out_dtype == DR_I64);
    if (!okpair) return fail(DR_ERR_UNSUPPORTED, "for_each %d -> %d is not supported", in, (int)out_dtype);
    Prepared p;
    int items;
    s = prepare(table, DR_ALGO_FOR_EACH, in, out_dtype, view->arity, bs ? 2 : 1, tuning, ws, ws_bytes, false,
                !bs, p, items);
    if (s) return s;
    LaunchFn fn = bs ? find_black_scholes(items) : find_for_each(in, out_dtype, view->op, items);
    if (!fn) return fail(DR_ERR_UNSUPPORTED, "for_each kernel not built for items_per_thread %d", items);
    p.a.alpha = view->alpha;
    return launch(fn, p, stream, "for_each launch");
}

dr_status dr_transform_reduce(const dr_table* table, const dr_view* view, int32_t acc, const void* init,
                              void* result, void* ws, size_t ws_bytes, const dr_tuning* tuning, void* stream) {
    dr_status s = check_view(view, true);
    if (s) return s;
    if (acc != DR_ACC_PLAIN && acc != DR_ACC_COMPENSATED) return fail(DR_ERR_INVALID_ARG, "unknown acc %d", acc);
    if (!init) return fail(DR_ERR_INVALID_ARG, "init is NULL");
    if (!result && !(table && table->mode == DR_MODE_BATCH && table->n_segments == 0))
        return fail(DR_ERR_INVALID_ARG, "result is NULL");
    Prepared p;
    int items;
    s = prepare(table, DR_ALGO_REDUCE, view->in_dtype, 0, view->arity, 0, tuning, ws, ws_bytes, true, false, p,
                items);
    if (s) return s;
    LaunchFn fn = find_reduce(view->in_dtype, view->op, acc, items);
    if (!fn) return fail(DR_ERR_UNSUPPORTED, "reduce kernel not built for items_per_thread %d", items);
    p.a.alpha = view->alpha;
    p.a.result = result;
    if (tuning && (tuning->flags & DR_TUNE_TILE_PER_BLOCK)) p.a.flags |= kFlagTilePerBlock;
    if (view->in_dtype == DR_I32) p.a.init_i = *(const int64_t*)init;
    else p.a.init_f = *(const double*)init;
    return launch(fn, p, stream, "transform_reduce launch");
}

// Default form of an integer sum scan (no tuning given): up to 2^22
// elements one kernel with a decoupled look-back has the lower latency (two
// launches instead of three, about 11 us against 14 us); integer carries are
// exact either way. Floating-point scans never take the look-back by
// default: its carries depend on timing, while the two passes' and the
// chained pass's are sums in a fixed order, so results repeat exactly.
static bool prefer_single_pass(const dr_table* t, int in_dt, const dr_tuning* tu) {
    return !tu && in_dt == DR_I32 && t && t->total_length <= ((int64_t)1 << 22);
}

// The form of a sum scan (launch flag): an explicit DR_TUNE_* form, else
// the look-back for small int32 scans (prefer_single_pass), else the
// reduce-then-scan passes. Max / min scans always run the two passes.
static uint32_t sum_scan_form(const dr_table* t, int in_dt, const dr_tuning* tu) {
    const int32_t f = tu ? tu->flags : 0;
    if (f & DR_TUNE_TILE_PER_BLOCK) return kFlagTilePerBlock;
    if (prefer_single_pass(t, in_dt, tu)) return kFlagTilePerBlock;
    return 0u;
}

// Without a tuning, a sum of the identity view over one range (CONCAT) of
// more than 2^22 binary32 / int32 elements runs the chained single pass:
// the input is read from HBM once instead of twice (2^28 binary32 elements
// in 16 segments: 500-508 us against 527-540 for the two passes; 2^30
// int32 -> int64 2.96 ms against 3.14, -> int32 2.08 against 2.26), and its
// carries, like the two passes', are sums in a fixed order. `tmp` holds
// the tuning it stands for.
static const dr_tuning* default_scan_tuning(const dr_table* t, int in_dt, int out_dt, int op, bool c64,
                                            const dr_tuning* tu, dr_tuning& tmp) {
    if (tu || !t || t->mode != DR_MODE_CONCAT || op != DR_OP_IDENTITY ||
        t->total_length <= ((int64_t)1 << 22) || !find_scan_chain(in_dt, out_dt, op, c64, 16))
        return tu;
    tmp = dr_tuning{0, 16, DR_TUNE_CHAINED, 0};
    return &tmp;
}

// The chained single pass (DR_TUNE_CHAINED), on request: sums of the
// identity view of one range (CONCAT) at 16 items per thread, for the
// dtypes find_scan_chain names. `fn` is its kernel when requested (and
// nullptr otherwise).
static dr_status chained_kernel(const dr_tuning* tu, const dr_table* t, int in_dt, int out_dt, int op,
                                bool c64, bool sum, LaunchFn& fn) {
    fn = nullptr;
    if (!tu || !(tu->flags & DR_TUNE_CHAINED)) return DR_OK;
    if (!sum) return fail(DR_ERR_UNSUPPORTED, "the chained single pass (DR_TUNE_CHAINED) runs sums only");
    if (t && t->mode != DR_MODE_CONCAT)
        return fail(DR_ERR_UNSUPPORTED, "the chained single pass (DR_TUNE_CHAINED) scans one range (CONCAT); "
                                        "batches of ranges run the look-back or the two-pass form");
    fn = find_scan_chain(in_dt, out_dt, op, c64, tu->items_per_thread ? tu->items_per_thread : 16);
    if (!fn)
        return fail(DR_ERR_UNSUPPORTED, "the chained single pass is built for sums of the identity view "
                                        "(binary32, int32 -> int64 / int32) at 16 items per thread");
    return DR_OK;
}

// The single pass with specialised waves, on request (DR_TUNE_SPECIALIZED,
// at the form's own tile size). It is not the default: at 2^28 binary32
// elements it measured level with the two passes (513-517 us against
// 511 us), and the fused form (16 items per thread, twice the tiles for its
// carry chain) 1108 us against 725 us. On success `use` is the tuning to
// prepare with and `on` says whether the form runs.
static dr_status specialized_tuning(int in_dt, int out_dt, int op, bool fused, bool c64,
                                    int acc, const dr_tuning* tu, dr_tuning& tmp, const dr_tuning*& use,
                                    bool& on) {
    use = tu;
    on = false;
    const int items = ws_items_for(in_dt, fused);
    const bool built = op == DR_OP_IDENTITY && items > 0 && !(in_dt == DR_I32 && out_dt == DR_I64) &&
                       (fused ? find_scan_reduce(in_dt, DR_OP_MUL, acc, items) != nullptr
                              : find_scan(in_dt, out_dt, op, c64, items) != nullptr);
    if (tu && (tu->flags & DR_TUNE_SPECIALIZED)) {
        if (tu->flags & DR_TUNE_TILE_PER_BLOCK)
            return fail(DR_ERR_INVALID_ARG, "DR_TUNE_SPECIALIZED and DR_TUNE_TILE_PER_BLOCK exclude each other");
        if (!built)
            return fail(DR_ERR_UNSUPPORTED, "the specialised-wave scan is built for sums of the identity view "
                                            "(binary32, bfloat16, binary64, int32 -> int32; fused: binary32)");
        if (tu->items_per_thread != items)
            return fail(DR_ERR_UNSUPPORTED, "the specialised-wave scan of this dtype is built for %d items per thread",
                        items);
        tmp = *tu;
        use = &tmp;
        on = true;
        return DR_OK;
    }
    return DR_OK;
}

// Without a tuning, int32 -> int64 sums of the identity view over more than
// 2^22 elements use tiles of 64 items per thread: the apply pass writes
// twice the bytes it reads, and larger tiles were measured 6 % faster at
// 2^30 elements. The workspace a default-sized caller holds is large enough
// (fewer, larger tiles need fewer tile words). Only tables that need no plan
// (at most DR_SMALL_TABLE rows) take it, since a plan is built for the tile
// size of the tuning it was made with.
static const dr_tuning* scan_tuning(const dr_table* t, int in_dt, int out_dt, int op, const dr_tuning* tu,
                                    dr_tuning& tmp) {
    if (tu || in_dt != DR_I32 || out_dt != DR_I64 || op != DR_OP_IDENTITY || !t ||
        t->total_length <= ((int64_t)1 << 22) || t->n_segments > DR_SMALL_TABLE)
        return tu;
    tmp = dr_tuning{0, 64, 0, 0};
    return &tmp;
}

dr_status dr_inclusive_scan(const dr_table* table, const dr_view* view, int32_t out_dtype, uint32_t flags,
                            void* ws, size_t ws_bytes, const dr_tuning* tuning, void* stream) {
    dr_status s = check_view(view, true);
    if (s) return s;
    const int in = view->in_dtype;
    const bool okpair = (in == DR_I32 && (out_dtype == DR_I64 || out_dtype == DR_I32)) ||
                        (in == DR_F32 && out_dtype == DR_F32) || (in == DR_BF16 && out_dtype == DR_F32) ||
                        (in == DR_F64 && out_dtype == DR_F64);
    if (!okpair) return fail(DR_ERR_UNSUPPORTED, "inclusive_scan %d -> %d is not supported", in, (int)out_dtype);
    if (flags & ~(uint32_t)(DR_SCAN_REVERSE | DR_SCAN_CARRY_F32))
        return fail(DR_ERR_INVALID_ARG, "unknown scan flags 0x%x", flags);
    if ((flags & DR_SCAN_CARRY_F32) && in != DR_F32 && in != DR_BF16)
        return fail(DR_ERR_INVALID_ARG, "DR_SCAN_CARRY_F32 applies to binary32/bfloat16 inputs only");
    dr_tuning chained_dflt;
    tuning = default_scan_tuning(table, in, out_dtype, view->op, (flags & DR_SCAN_CARRY_F32) == 0, tuning,
                                 chained_dflt);
    LaunchFn chain = nullptr;
    s = chained_kernel(tuning, table, in, out_dtype, view->op, (flags & DR_SCAN_CARRY_F32) == 0, true, chain);
    if (s) return s;
    Prepared p;
    int items;
    dr_tuning dflt, wst;
    const dr_tuning* wsu = nullptr;
    bool ws_on = false;
    s = specialized_tuning(in, out_dtype, view->op, false, (flags & DR_SCAN_CARRY_F32) == 0, 0, tuning, wst,
                           wsu, ws_on);
    if (s) return s;
    s = prepare(table, DR_ALGO_SCAN, in, out_dtype, view->arity, 1,
                ws_on ? wsu : scan_tuning(table, in, out_dtype, view->op, tuning, dflt), ws, ws_bytes, true,
                view->op == DR_OP_IDENTITY, p, items);
    if (s) return s;
    const bool c64 = (flags & DR_SCAN_CARRY_F32) == 0;
    LaunchFn fn = chain ? chain : scan_kernel(in, out_dtype, view->op, c64, items, p.block, tuning);
    if (!fn) return fail(DR_ERR_UNSUPPORTED, "scan kernel not built for this combination");
    p.a.alpha = view->alpha;
    p.a.flags = flags;
    if (chain) p.a.flags |= kFlagChained;
    else if (ws_on) p.a.flags |= kFlagSpecialized;
    else p.a.flags |= sum_scan_form(table, in, tuning);
    return launch(fn, p, stream, "inclusive_scan launch");
}

dr_status dr_reduce(const dr_table* table, const dr_view* view, int32_t combine, int32_t acc, const void* init,
                    void* result, void* ws, size_t ws_bytes, const dr_tuning* tuning, void* stream) {
    if (combine == DR_COMBINE_SUM) {
        const int64_t zero_i = 0;
        const double zero_f = 0.0;
        const void* iv = init ? init : (view && view->in_dtype == DR_I32 ? (const void*)&zero_i : (const void*)&zero_f);
        return dr_transform_reduce(table, view, acc, iv, result, ws, ws_bytes, tuning, stream);
    }
    if (combine != DR_COMBINE_MAX && combine != DR_COMBINE_MIN)
        return fail(DR_ERR_INVALID_ARG, "unknown combine %d", combine);
    dr_status s = check_view(view, true);
    if (s) return s;
    if (!result && !(table && table->mode == DR_MODE_BATCH && table->n_segments == 0))
        return fail(DR_ERR_INVALID_ARG, "result is NULL");
    Prepared p;
    int items;
    s = prepare(table, DR_ALGO_REDUCE, view->in_dtype, 0, view->arity, 0, tuning, ws, ws_bytes, true, false, p,
                items);
    if (s) return s;
    LaunchFn fn = find_reduce_minmax(view->in_dtype, view->op, items);
    if (!fn)
        return fail(DR_ERR_UNSUPPORTED, "max / min reductions are built for the default items per thread "
                                        "(16; bfloat16 16 or 32), not %d", items);
    const bool mn = combine == DR_COMBINE_MIN;
    p.a.alpha = view->alpha;
    p.a.result = result;
    if (mn) p.a.flags |= kFlagMin;
    if (tuning && (tuning->flags & DR_TUNE_TILE_PER_BLOCK)) p.a.flags |= kFlagTilePerBlock;
    if (view->in_dtype == DR_I32)
        p.a.init_i = init ? *(const int64_t*)init : (mn ? INT64_MAX : INT64_MIN);
    else
        p.a.init_f = init ? *(const double*)init : (mn ? HUGE_VAL : -HUGE_VAL);
    return launch(fn, p, stream, "reduce launch");
}

dr_status dr_scan(const dr_table* table, const dr_view* view, int32_t out_dtype, int32_t combine, uint32_t flags,
                  const void* init, void* ws, size_t ws_bytes, const dr_tuning* tuning, void* stream) {
    if (combine != DR_COMBINE_SUM && combine != DR_COMBINE_MAX && combine != DR_COMBINE_MIN)
        return fail(DR_ERR_INVALID_ARG, "unknown combine %d", combine);
    dr_status s = check_view(view, true);
    if (s) return s;
    const int in = view->in_dtype;
    const bool okpair = (in == DR_I32 && (out_dtype == DR_I64 || out_dtype == DR_I32)) ||
                        (in == DR_F32 && out_dtype == DR_F32) || (in == DR_BF16 && out_dtype == DR_F32) ||
                        (in == DR_F64 && out_dtype == DR_F64);
    if (!okpair) return fail(DR_ERR_UNSUPPORTED, "scan %d -> %d is not supported", in, (int)out_dtype);
    if (flags & ~(uint32_t)(DR_SCAN_REVERSE | DR_SCAN_CARRY_F32 | DR_SCAN_EXCLUSIVE))
        return fail(DR_ERR_INVALID_ARG, "unknown scan flags 0x%x", flags);
    if ((flags & DR_SCAN_CARRY_F32) && in != DR_F32 && in != DR_BF16)
        return fail(DR_ERR_INVALID_ARG, "DR_SCAN_CARRY_F32 applies to binary32/bfloat16 inputs only");
    const bool mm = combine != DR_COMBINE_SUM;
    if (mm) {
        if (view->op != DR_OP_IDENTITY)
            return fail(DR_ERR_UNSUPPORTED, "max / min scans are built for the identity view");
        if (flags & DR_SCAN_CARRY_F32) return fail(DR_ERR_UNSUPPORTED, "DR_SCAN_CARRY_F32 applies to sums");
        if (tuning && (tuning->flags & DR_TUNE_TILE_PER_BLOCK))
            return fail(DR_ERR_UNSUPPORTED, "max / min scans run in the reduce-then-scan form only");
        if (tuning && tuning->items_per_thread != 0 && tuning->items_per_thread != 16)
            return fail(DR_ERR_UNSUPPORTED, "max / min scans are built for 16 items per thread");
    }
    if (mm && tuning && (tuning->flags & (DR_TUNE_SPECIALIZED | DR_TUNE_CHAINED)))
        return fail(DR_ERR_UNSUPPORTED, "max / min scans run in the reduce-then-scan form only");
    dr_tuning chained_dflt;
    if (!mm)
        tuning = default_scan_tuning(table, in, out_dtype, view->op, (flags & DR_SCAN_CARRY_F32) == 0, tuning,
                                     chained_dflt);
    LaunchFn chain = nullptr;
    s = chained_kernel(tuning, table, in, out_dtype, view->op, (flags & DR_SCAN_CARRY_F32) == 0, !mm, chain);
    if (s) return s;
    Prepared p;
    int items;
    dr_tuning dflt, wst;
    const dr_tuning* wsu = nullptr;
    bool ws_on = false;
    if (!mm) {
        s = specialized_tuning(in, out_dtype, view->op, false, (flags & DR_SCAN_CARRY_F32) == 0, 0, tuning,
                               wst, wsu, ws_on);
        if (s) return s;
    }
    s = prepare(table, DR_ALGO_SCAN, in, out_dtype, view->arity, 1,
                mm ? tuning : ws_on ? wsu : scan_tuning(table, in, out_dtype, view->op, tuning, dflt), ws, ws_bytes,
                true, view->op == DR_OP_IDENTITY, p, items);
    if (s) return s;
    LaunchFn fn = mm    ? find_scan_minmax(in, out_dtype)
                  : chain ? chain
                          : scan_kernel(in, out_dtype, view->op, (flags & DR_SCAN_CARRY_F32) == 0, items, p.block,
                                        tuning);
    if (!fn) return fail(DR_ERR_UNSUPPORTED, "scan kernel not built for this combination");
    p.a.alpha = view->alpha;
    p.a.flags = flags;
    if (chain) p.a.flags |= kFlagChained;
    else if (ws_on) p.a.flags |= kFlagSpecialized;
    else if (!mm) p.a.flags |= sum_scan_form(table, in, tuning);
    if (combine == DR_COMBINE_MIN) p.a.flags |= kFlagMin;
    if (init) {
        p.a.flags |= kFlagHasInit;
        if (in == DR_I32) p.a.init_i = *(const int64_t*)init;
        else p.a.init_f = *(const double*)init;
    }
    return launch(fn, p, stream, "scan launch");
}

dr_status dr_scan_reduce(const dr_table* table, const dr_view* scan_view, const dr_view* reduce_view,
                         int32_t acc, const void* init, void* result, uint32_t flags, void* ws, size_t ws_bytes,
                         const dr_tuning* tuning, void* stream) {
    dr_status s = check_view(scan_view, false);
    if (s) return s;
    s = check_view(reduce_view, false);
    if (s) return s;
    const int in = scan_view->in_dtype;
    if (scan_view->op != DR_OP_IDENTITY || (in != DR_F32 && in != DR_F64))
        return fail(DR_ERR_UNSUPPORTED, "fused scan: the scan view must be identity over binary32/64 in[0]");
    if (reduce_view->in_dtype != in || reduce_view->op != DR_OP_MUL)
        return fail(DR_ERR_UNSUPPORTED, "fused scan: the reduce view must be mul over in[0], in[1] of the "
                                        "scanned type");
    if (acc != DR_ACC_PLAIN && acc != DR_ACC_COMPENSATED) return fail(DR_ERR_INVALID_ARG, "unknown acc %d", acc);
    if (flags & ~(uint32_t)DR_SCAN_REVERSE) return fail(DR_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    if (!init) return fail(DR_ERR_INVALID_ARG, "init is NULL");
    if (!result && !(table && table->mode == DR_MODE_BATCH && table->n_segments == 0))
        return fail(DR_ERR_INVALID_ARG, "result is NULL");
    if (tuning && (tuning->flags & DR_TUNE_CHAINED))
        return fail(DR_ERR_UNSUPPORTED, "the chained single pass (DR_TUNE_CHAINED) is not built for the fused "
                                        "scan + reduce");
    Prepared p;
    int items;
    dr_tuning wst;
    const dr_tuning* wsu = nullptr;
    bool ws_on = false;
    s = specialized_tuning(in, in, DR_OP_IDENTITY, true, true, acc, tuning, wst, wsu, ws_on);
    if (s) return s;
    s = prepare(table, DR_ALGO_SCAN_REDUCE, in, in, 2, 1, ws_on ? wsu : tuning, ws, ws_bytes, true, true, p, items);
    if (s) return s;
    LaunchFn fn = scan_reduce_kernel(in, reduce_view->op, acc, items, p.block, tuning);
    if (!fn) return fail(DR_ERR_UNSUPPORTED, "fused scan kernel not built for this combination");
    p.a.flags = flags;
    if (ws_on) p.a.flags |= kFlagSpecialized;
    else p.a.flags |= sum_scan_form(table, in, tuning);
    p.a.result = result;
    p.a.init_f = *(const double*)init;
    return launch(fn, p, stream, "scan_reduce launch");
}

dr_status dr_broadcast_mul(const dr_table* table, const dr_view* view, const double* g, int32_t n_grads,
                           void* ws, size_t ws_bytes, const dr_tuning* tuning, void* stream) {
    dr_status s = check_view(view, false);
    if (s) return s;
    if (!g) return fail(DR_ERR_INVALID_ARG, "g is NULL");
    if (n_grads < 1 || n_grads > view->arity)
        return fail(DR_ERR_INVALID_ARG, "n_grads must be 1..%d", (int)view->arity);
    const int in = view->in_dtype;
    const int out = in == DR_F64 ? DR_F64 : DR_F32;
    Prepared p;
    int items;
    s = prepare(table, DR_ALGO_BROADCAST_MUL, in, out, view->arity, n_grads, tuning, ws, ws_bytes, false, false,
                p, items);
    if (s) return s;
    LaunchFn fn = find_broadcast_mul(in, view->op, items);
    if (!fn) return fail(DR_ERR_UNSUPPORTED, "broadcast_mul kernel not built for this combination");
    p.a.alpha = view->alpha;
    p.a.g = g;
    return launch(fn, p, stream, "broadcast_mul launch");
}

dr_status dr_check_device_error(uint32_t* flags, void* stream) {
    if (!flags) return fail(DR_ERR_INVALID_ARG, "flags is NULL");
    hipStream_t st = (hipStream_t)stream;
    DeviceGlobals dg;
    hipError_t e = device_globals(st, dg);
    if (e != hipSuccess) return hip_fail(e, "device fault word lookup");
    uint32_t host = 0;
    e = hipMemcpyAsync(&host, dg.fault, sizeof host, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "device fault word read");
    *flags = host;
    if (host != 0) {
        const uint32_t zero = 0;
        e = hipMemcpyAsync(dg.fault, &zero, sizeof zero, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "device fault word clear");
        return fail(DR_ERR_DEVICE, "device fault flags 0x%x", host);
    }
    return ok();
}

dr_status dr_device_status(void* ws, uint32_t* flags, void* stream) {
    if (!ws) return fail(DR_ERR_WORKSPACE, "workspace is NULL");
    if (!flags) return fail(DR_ERR_INVALID_ARG, "flags is NULL");
    hipStream_t st = (hipStream_t)stream;
    uint32_t host = 0;
    void* dev = (char*)ws + offsetof(Header, error);
    hipError_t e = hipMemcpyAsync(&host, dev, sizeof host, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "device status read");
    *flags = host;
    if (host != 0) {
        const uint32_t zero = 0;
        e = hipMemcpyAsync(dev, &zero, sizeof zero, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "device status clear");
        return fail(DR_ERR_DEVICE, "device fault flags 0x%x", host);
    }
    return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Segment algebra (section 4.4): host-only computations on segment lists
// ---------------------------------------------------------------------------

namespace {

dr_status check_range(const dr_range* r, const char* what) {
    if (!r) return fail(DR_ERR_INVALID_ARG, "%s is NULL", what);
    if (r->elem_size <= 0) return fail(DR_ERR_INVALID_ARG, "%s: elem_size must be positive", what);
    if (r->reserved != 0) return fail(DR_ERR_INVALID_ARG, "%s: reserved field must be 0", what);
    if (r->n_spans < 0) return fail(DR_ERR_INVALID_ARG, "%s: negative span count", what);
    if (r->n_spans > 0 && !r->spans) return fail(DR_ERR_INVALID_ARG, "%s: spans is NULL", what);
    for (int64_t k = 0; k < r->n_spans; ++k)
        if (r->spans[k].length < 0) return fail(DR_ERR_INVALID_ARG, "%s: span %lld has a negative length", what,
                                                (long long)k);
    return DR_OK;
}

void* advance(void* p, int64_t elems, int32_t size) {
    return p ? (void*)((char*)p + elems * (int64_t)size) : nullptr;
}

}  // namespace

dr_status dr_trim_segments(const dr_range* r, int64_t first, int64_t last, dr_span* out, int64_t capacity,
                           int64_t* n_out) {
    dr_status s = check_range(r, "range");
    if (s) return s;
    if (!n_out) return fail(DR_ERR_INVALID_ARG, "n_out is NULL");
    int64_t total = 0;
    for (int64_t k = 0; k < r->n_spans; ++k) total += r->spans[k].length;
    first = std::min(std::max<int64_t>(first, 0), total);
    last = std::min(std::max<int64_t>(last, 0), total);
    // count first, so that a too-small `out` is rejected before any write
    int64_t n = 0, o = 0;
    for (int64_t k = 0; k < r->n_spans; ++k) {
        const int64_t b = std::max(o, first), e = std::min(o + r->spans[k].length, last);
        if (e > b) ++n;
        o += r->spans[k].length;
    }
    if (n > 0 && !out) return fail(DR_ERR_INVALID_ARG, "out is NULL");
    if (n > capacity) return fail(DR_ERR_INVALID_ARG, "capacity %lld < %lld spans", (long long)capacity,
                                  (long long)n);
    int64_t i = 0;
    o = 0;
    for (int64_t k = 0; k < r->n_spans; ++k) {
        const int64_t len = r->spans[k].length;
        const int64_t b = std::max(o, first), e = std::min(o + len, last);
        if (e > b) out[i++] = dr_span{advance(r->spans[k].ptr, b - o, r->elem_size), e - b};
        o += len;
    }
    *n_out = n;
    return ok();
}

dr_status dr_zip_segments(const dr_range* ins, int32_t n_in, const dr_range* outs, int32_t n_out,
                          dr_segment* rows, int64_t capacity, int64_t* n_rows, int64_t* length) {
    if (n_in < 1 || n_in > DR_MAX_ARITY) return fail(DR_ERR_INVALID_ARG, "n_in must be 1..%d", DR_MAX_ARITY);
    if (n_out < 0 || n_out > DR_MAX_OUTPUTS) return fail(DR_ERR_INVALID_ARG, "n_out must be 0..%d", DR_MAX_OUTPUTS);
    if (!ins || (n_out > 0 && !outs)) return fail(DR_ERR_INVALID_ARG, "ranges are NULL");
    if (!n_rows || !length) return fail(DR_ERR_INVALID_ARG, "n_rows / length is NULL");
    const int R = n_in + n_out;
    const dr_range* rs[DR_MAX_ARITY + DR_MAX_OUTPUTS];
    for (int i = 0; i < n_in; ++i) rs[i] = &ins[i];
    for (int j = 0; j < n_out; ++j) rs[n_in + j] = &outs[j];
    for (int i = 0; i < R; ++i) {
        dr_status s = check_range(rs[i], i < n_in ? "input range" : "output range");
        if (s) return s;
    }
    // Two passes over the same walk: count the rows, then (if they fit) write them.
    for (int pass = 0; pass < 2; ++pass) {
        int64_t seg[DR_MAX_ARITY + DR_MAX_OUTPUTS] = {0};   // current segment of each range
        int64_t off[DR_MAX_ARITY + DR_MAX_OUTPUTS] = {0};   // elements already taken from it
        int64_t n = 0, len = 0;
        while (true) {
            bool done = false;
            int64_t piece = INT64_MAX;
            for (int i = 0; i < R; ++i) {
                // step over exhausted (and empty) segments
                while (seg[i] < rs[i]->n_spans && off[i] == rs[i]->spans[seg[i]].length) {
                    ++seg[i];
                    off[i] = 0;
                }
                if (seg[i] == rs[i]->n_spans) {
                    done = true;
                    break;
                }
                piece = std::min(piece, rs[i]->spans[seg[i]].length - off[i]);
            }
            if (done) break;
            if (pass == 1) {
                dr_segment& row = rows[n];
                std::memset(&row, 0, sizeof row);
                for (int i = 0; i < n_in; ++i)
                    row.in[i] = advance(rs[i]->spans[seg[i]].ptr, off[i], rs[i]->elem_size);
                for (int j = 0; j < n_out; ++j) {
                    const int i = n_in + j;
                    row.out[j] = advance(rs[i]->spans[seg[i]].ptr, off[i], rs[i]->elem_size);
                }
                row.length = piece;
            }
            for (int i = 0; i < R; ++i) off[i] += piece;
            ++n;
            len += piece;
        }
        if (pass == 0) {
            if (n > 0 && !rows) return fail(DR_ERR_INVALID_ARG, "rows is NULL");
            if (n > capacity)
                return fail(DR_ERR_INVALID_ARG, "capacity %lld < %lld rows", (long long)capacity, (long long)n);
        } else {
            *n_rows = n;
            *length = len;
        }
    }
    return ok();
}

