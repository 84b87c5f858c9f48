// dr_internal.hpp — layout of the caller's workspace and the launcher
// registry shared by the host API (dr_api.cpp) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dr.h"

namespace dr {

// Device fault flags (dr_device_status).
enum : uint32_t {
    DR_DEVFLAG_BAD_TABLE = 1u,
    DR_DEVFLAG_TIMEOUT = 2u,
    DR_DEVFLAG_PLAN = 4u,
    DR_DEVFLAG_TOO_MANY_TILES = 8u
};

constexpr int kBlock = 256;            // threads per workgroup (4 waves)
constexpr int kGroupTiles = 64;        // tiles per first-level combine group
constexpr int kMaxChunks = 2048;        // workgroups of a scan's first (tile totals) pass

// First 256 bytes of every workspace.
struct Header {
    uint32_t error;      // DR_DEVFLAG_* bits, sticky until dr_device_status
    uint32_t epoch;      // launches on this workspace; bumped by each launch's prologue
    uint32_t plan_tag;   // tag of the launch that wrote the plan words
    uint32_t pad0;
    uint64_t plan_rows;  // key of the plan built by dr_plan
    int64_t plan_m;
    int64_t plan_tile;
    int64_t plan_total;
    int64_t plan_tiles;  // tile count of the planned table
    int32_t plan_ies;
    int32_t plan_arity;
    uint8_t pad[256 - 4 * 4 - 8 * 5 - 4 * 2];
};
static_assert(sizeof(Header) == 256, "header is 256 bytes");

// Fixed part of every workspace: the header. Variable sections follow.
constexpr uint64_t kFixedBytes = sizeof(Header);

// Byte offsets of the variable workspace sections (all 256-byte aligned).
// Every 64-bit word in them is tagged with the epoch of the launch (or
// plan) that wrote it, so stale contents of any layout are never mistaken
// for current ones.
struct WsLayout {
    uint64_t off_plan_first;   // tagged [m + 1]: first tile of each segment (large tables)
    uint64_t off_plan_tseg;    // tagged [tmax]: segment of each tile (large tables)
    uint64_t off_tile;         // [tmax * tile_words]: per-tile (or per-workgroup) tagged words
    uint64_t off_gcnt;         // uint32 [ngroups]: arrivals per combine group (zeroed by the prologue)
    uint64_t off_gpart;        // [ngroups * 2]: tagged group partials
    uint64_t off_ucnt;         // uint32 [nunits]: arrived groups per result (zeroed by the prologue)
    uint64_t off_chunk;        // scans: [4 + 4 * kMaxChunks] chunk records of the reduce-then-scan form
    uint64_t off_pipe;         // scans: uint32 [npipe]: the chained pass's chunk counter, then one arrival
                               // counter per superblock (zeroed by the prologue)
    uint64_t npipe;
    uint64_t off_pipe_e;       // scans: tagged [2 * npipe]: the running carry at the end of each superblock
    uint64_t bytes;            // total size
    uint64_t ngroups;          // counters at off_gcnt
    uint64_t nunits;           // counters at off_ucnt
    int32_t tile_words;        // 64-bit words per tile
    int32_t part_word;         // first word of the reduce partial inside a tile's words
};

// Launch-wide arguments shared by the kernels (passed by value).
struct LaunchArgs {
    const dr_segment* rows;
    int64_t m;
    int64_t total;
    int64_t tile;         // elements per tile
    int64_t tmax;         // grid size = bound on the tile count
    int32_t ies;          // input element size
    int32_t oes;          // output element size (0: no output)
    int32_t mode;
    uint32_t flags;
    int32_t arity;
    int32_t nout;
    double alpha;
    uint8_t* ws;
    WsLayout lay;
    void* result;
    double init_f;
    int64_t init_i;
    const double* g;
    uint64_t spin_ticks;  // bound of every wait, wall-clock ticks
    uint32_t* gfault;     // the device's library-wide fault word (device address)
};

// Launches the kernel with `grid` workgroups, one per tile (kernels that use
// tags are preceded by the epoch prologue).
typedef hipError_t (*LaunchFn)(const LaunchArgs& a, int64_t grid, hipStream_t stream);

// Internal launch flag (LaunchArgs.flags, above the public scan flags):
// CONCAT reduce with one workgroup per tile instead of the streaming grid.
constexpr uint32_t kFlagTilePerBlock = 1u << 16;
constexpr uint32_t kFlagHasInit = 1u << 17;   // scans: combine init into every output
constexpr uint32_t kFlagMin = 1u << 18;       // min/max kernels: min (else max)
constexpr int kAccMinMax = 2;                 // reduce kernels: max / min instead of a sum
constexpr uint32_t kFlagSpecialized = 1u << 19;   // scans: the single pass with specialised waves
constexpr uint32_t kFlagChained = 1u << 20;       // scans: the chained single pass (chunks re-read from L2)

// Chunks per superblock of the chained single pass: a chunk's carry folds
// the totals of at most this many chunks before it.
constexpr int kChainSB = 128;

// Items per thread of the scans' specialised-wave form for an input dtype
// (0: not built).
int ws_items_for(int in_dt, bool fused);

// Workgroups of `kernel` (of `threads` threads) that can be resident at once.
int resident_grid(const void* kernel, int threads = kBlock);

// The prologue of every launch that uses tags: epoch + 1, and the launch's
// arrival counters (if any) set to 0.
hipError_t launch_prologue(const LaunchArgs& a, hipStream_t stream);

// Kernel lookup. `items` is the elements per thread of the tile. Each
// returns nullptr when the combination is not built.
LaunchFn find_for_each(int in_dt, int out_dt, int op, int items);
LaunchFn find_reduce(int in_dt, int op, int acc, int items);
LaunchFn find_reduce_minmax(int in_dt, int op, int items);
LaunchFn find_scan_minmax(int in_dt, int out_dt);
LaunchFn find_scan(int in_dt, int out_dt, int op, bool carry64, int items);
LaunchFn find_scan_reduce(int in_dt, int reduce_op, int acc, int items);
// The look-back scan at the shapes k_scan.hip does not build (512 / 1024
// threads, or 4 / 8 items per thread): binary32 sums with binary64 carries,
// plain (fused = false) or fused with the compensated dot.
LaunchFn find_scan_wide(int in_dt, int out_dt, int op, bool carry64, bool fused, int acc, int items, int block);
// The chained single pass (k_scan_chain.hip): sums of the identity view of
// one range (CONCAT), binary32 and int32 -> int64 / int32, 16 items.
LaunchFn find_scan_chain(int in_dt, int out_dt, int op, bool carry64, int items);
LaunchFn find_broadcast_mul(int in_dt, int op, int items);
LaunchFn find_black_scholes(int items);
hipError_t launch_plan(const LaunchArgs& a, hipStream_t stream);     // prefix + tile -> segment map
hipError_t launch_zero(void* p, size_t bytes, hipStream_t stream);  // fill with 0 (graph safe)

// Device addresses of the library's static device memory on the device of
// `stream`: the fault word every kernel also reports to, and the scratch
// area of the calls that allocate nothing. Looked up once per device.
struct DeviceGlobals {
    uint32_t* fault;
    uint8_t* scratch;
    size_t scratch_bytes;
    int device;
};
hipError_t device_globals(hipStream_t stream, DeviceGlobals& g);

// Record `s` with a formatted reason as the calling thread's last error
// (dr_last_error) and return it.
dr_status set_error(dr_status s, const char* fmt, ...);


}  // namespace dr
