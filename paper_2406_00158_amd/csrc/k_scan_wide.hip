// k_scan_wide.hip — the single-pass look-back scan (DR_TUNE_TILE_PER_BLOCK)
// at other launch shapes than the 256-thread tiles of k_scan.hip: 512- and
// 1024-thread workgroups, and 4 or 8 items per thread at 256 threads. These
// are the shapes the autotuner adds for the batched scans (many short
// ranges, whose look-backs stop at their range's first tile): the binary32
// sum of the identity view with binary64 carries, and its fusion with the
// compensated dot. A larger workgroup forms a larger tile with the same
// items per thread (fewer look-backs, fewer registers per thread than the
// same tile at 256 threads); a 1024-thread workgroup may use 128 registers
// per thread, so it is built up to 16 items.
#include "k_scan_core.hpp"

namespace dr {

template <int IDT, int ODT, int OP, bool C64, bool FUSED, int ROP, int RACC, int ITEMS, int BLOCK>
hipError_t launch_scan_wide(const LaunchArgs& a, int64_t grid, hipStream_t stream) {
    // the host selects these shapes with DR_TUNE_TILE_PER_BLOCK only
    if (!(a.flags & kFlagTilePerBlock)) return hipErrorNotSupported;
    hipError_t e = launch_prologue(a, stream);
    if (e != hipSuccess) return e;
    if (a.flags & DR_SCAN_REVERSE)
        hipLaunchKernelGGL((k_scan<IDT, ODT, OP, C64, FUSED, ROP, RACC, ITEMS, true, BLOCK>), dim3((uint32_t)grid),
                           dim3(BLOCK), 0, stream, a);
    else
        hipLaunchKernelGGL((k_scan<IDT, ODT, OP, C64, FUSED, ROP, RACC, ITEMS, false, BLOCK>), dim3((uint32_t)grid),
                           dim3(BLOCK), 0, stream, a);
    return hipGetLastError();
}

#define DR_WIDE(ITEMS, BLOCK)                                                                                  \
    if (items == ITEMS && block == BLOCK) {                                                                    \
        if (fused) return launch_scan_wide<DR_F32, DR_F32, DR_OP_IDENTITY, true, true, DR_OP_MUL,             \
                                           DR_ACC_COMPENSATED, ITEMS, BLOCK>;                                  \
        return launch_scan_wide<DR_F32, DR_F32, DR_OP_IDENTITY, true, false, 0, 0, ITEMS, BLOCK>;              \
    }

LaunchFn find_scan_wide(int in_dt, int out_dt, int op, bool carry64, bool fused, int acc, int items, int block) {
    if (in_dt != DR_F32 || out_dt != DR_F32 || op != DR_OP_IDENTITY) return nullptr;
    if (fused ? acc != DR_ACC_COMPENSATED : !carry64) return nullptr;
    DR_WIDE(4, 256)
    DR_WIDE(8, 256)
    DR_WIDE(8, 512)
    DR_WIDE(16, 512)
    DR_WIDE(32, 512)
    DR_WIDE(4, 1024)
    DR_WIDE(8, 1024)
    DR_WIDE(16, 1024)
    return nullptr;
}

}  // namespace dr
