// k_plan.hip — tile plan of a large segment table, and the zero fill of a
// fresh workspace.
//
// The plan words are tagged with the plan launch's epoch (high 32 bits), so
// launches that later reuse the workspace with another layout cannot be
// mistaken for a plan. A distributed range exposes how it is split into
// segments (section 3,
// "Distributed Range"); the plan turns that split into the work list of one
// launch: the index of each segment's first tile (a prefix sum of
// per-segment tile counts) and, for every tile, its segment. Small tables
// (up to 64 rows) are planned by every workgroup on the fly; this plan is
// for larger ones (for example 10,000 ragged ranges), built once per table
// and tile shape and then reused by every launch on that workspace.
#include "dr_device.hpp"

namespace dr {

constexpr int kPlanBlock = 1024;

// One workgroup: per-segment tile counts, their exclusive prefix F[0..m],
// validation of every row, and the plan key in the header.
__global__ __launch_bounds__(kPlanBlock) void k_plan_prefix(LaunchArgs a) {
    __shared__ int64_t s_wave[kPlanBlock / 64];
    __shared__ int64_t s_carry, s_len;
    __shared__ int s_bad;
    Header* h = header(a.ws);
    // the plan launch is alone on the workspace: it bumps the epoch itself
    const uint32_t epoch = h->epoch + 1u;
    const uint32_t tag = epoch_tag(epoch);
    uint64_t* F = (uint64_t*)(a.ws + a.lay.off_plan_first);
    const int w = threadIdx.x >> 6, l = lane_id();
    __syncthreads();
    if (threadIdx.x == 0) {
        h->epoch = epoch;
        s_carry = 0;
        s_len = 0;
        s_bad = 0;
        h->plan_m = -1;   // invalid until complete
    }
    __syncthreads();
    for (int64_t base = 0; base < a.m; base += kPlanBlock) {
        const int64_t k = base + threadIdx.x;
        int64_t cnt = 0, n = 0;
        if (k < a.m) {
            const Row r = load_row(a.rows, k);
            if (row_bad(r, a.arity, 0)) {
                s_bad = 1;
            } else {
                n = r.n;
                cnt = tiles_of(n, row_shift(r.in0, a.ies), a.tile);
            }
        }
        const int64_t inc = wave_incl_scan(cnt);
        const int64_t nsum = wave_sum(n);
        if (l == 63) s_wave[w] = inc;
        if (l == 0) atomicAdd((unsigned long long*)&s_len, (unsigned long long)nsum);
        __syncthreads();
        int64_t woff = 0;
        for (int i = 0; i < w; ++i) woff += s_wave[i];
        if (k < a.m) F[k] = ((uint64_t)tag << 32) | (uint64_t)(s_carry + woff + inc - cnt);
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t tot = 0;
            for (int i = 0; i < kPlanBlock / 64; ++i) tot += s_wave[i];
            s_carry += tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        F[a.m] = ((uint64_t)tag << 32) | (uint64_t)s_carry;
        if (s_bad || s_len != a.total) {
            flag_error(a, DR_DEVFLAG_BAD_TABLE);
        } else if (s_carry > a.tmax) {
            flag_error(a, DR_DEVFLAG_TOO_MANY_TILES);
        } else {
            h->plan_rows = (uint64_t)(uintptr_t)a.rows;
            h->plan_tile = a.tile;
            h->plan_total = a.total;
            h->plan_tiles = s_carry;
            h->plan_ies = a.ies;
            h->plan_arity = a.arity;
            h->plan_tag = tag;
            h->plan_m = a.m;
        }
    }
}

// tile -> segment: the last segment whose first tile is at or before t
// (empty segments share their successor's first tile and are skipped).
__global__ __launch_bounds__(256) void k_plan_tiles(LaunchArgs a) {
    const Header* h = (const Header*)a.ws;
    if (h->plan_m != a.m) return;   // prefix step failed
    const int64_t T = h->plan_tiles;
    const uint64_t tag = h->plan_tag;
    const uint64_t* F = (const uint64_t*)(a.ws + a.lay.off_plan_first);
    uint64_t* tseg = (uint64_t*)(a.ws + a.lay.off_plan_tseg);
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < T; t += (int64_t)gridDim.x * 256) {
        int64_t lo = 0, hi = a.m - 1;   // invariant: F[lo] <= t, answer in [lo, hi]
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if ((int64_t)(uint32_t)F[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        tseg[t] = (tag << 32) | (uint64_t)lo;
    }
}

__global__ __launch_bounds__(256) void k_zero(uint64_t* p, int64_t words) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (int64_t)gridDim.x * 256)
        p[i] = 0;
}

hipError_t launch_plan(const LaunchArgs& a, hipStream_t stream) {
    hipLaunchKernelGGL(k_plan_prefix, dim3(1), dim3(kPlanBlock), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int64_t blocks = (a.tmax + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_plan_tiles, dim3((uint32_t)blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

// Prologue of a launch that uses tags: epoch + 1 (workgroup 0), and the
// group / unit arrival counters and the chained scan's counters of the
// launch's layout set to 0.
__global__ __launch_bounds__(256) void k_prologue(uint8_t* ws, uint64_t off_g, uint64_t ng, uint64_t off_u,
                                                  uint64_t nu, uint64_t off_p, uint64_t np) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Header* h = (Header*)ws;
        h->epoch = h->epoch + 1u;
    }
    uint32_t* g = (uint32_t*)(ws + off_g);
    uint32_t* u = (uint32_t*)(ws + off_u);
    uint32_t* q = (uint32_t*)(ws + off_p);
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < ng; i += stride) g[i] = 0u;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < nu; i += stride) u[i] = 0u;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < np; i += stride) q[i] = 0u;
}

hipError_t launch_prologue(const LaunchArgs& a, hipStream_t stream) {
    uint64_t n = a.lay.ngroups > a.lay.nunits ? a.lay.ngroups : a.lay.nunits;
    if (a.lay.npipe > n) n = a.lay.npipe;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 256) blocks = 256;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_prologue, dim3((uint32_t)blocks), dim3(256), 0, stream, a.ws, a.lay.off_gcnt,
                       a.lay.ngroups, a.lay.off_ucnt, a.lay.nunits, a.lay.off_pipe, a.lay.npipe);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t stream) {
    const int64_t words = (int64_t)(bytes / 8);
    int64_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero, dim3((uint32_t)blocks), dim3(256), 0, stream, (uint64_t*)p, words);
    return hipGetLastError();
}

}  // namespace dr
