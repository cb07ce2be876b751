// Launchers of the fused step kernel (step_kernel.hpp) without equilibrium walls.
#include "step_kernel.hpp"

namespace mlbm {

template <int PAT, int ST, bool CHECK>
static hipError_t launch_one(const StepArgs &a, int grid, int block, hipStream_t s)
{
    hipLaunchKernelGGL((step_kernel<PAT, ST, CHECK, false>), dim3(grid), dim3(block), 0, s, a);
    return hipGetLastError();
}

template <int PAT, int ST>
static hipError_t launch_pst(const StepArgs &a, bool check, int grid, int block, hipStream_t s)
{
    return check ? launch_one<PAT, ST, true>(a, grid, block, s) : launch_one<PAT, ST, false>(a, grid, block, s);
}

template <int PAT>
static hipError_t launch_pat(const StepArgs &a, int st, bool check, int grid, int block, hipStream_t s)
{
    switch (st) {
    case ST_F64: return launch_pst<PAT, ST_F64>(a, check, grid, block, s);
    case ST_F32: return launch_pst<PAT, ST_F32>(a, check, grid, block, s);
    case ST_F16: return launch_pst<PAT, ST_F16>(a, check, grid, block, s);
    case ST_F32D: return launch_pst<PAT, ST_F32D>(a, check, grid, block, s);
    default: return launch_pst<PAT, ST_BF16>(a, check, grid, block, s);
    }
}

hipError_t launch_step_plain(const StepArgs &a, int pat, int st, bool check, int grid, int block, hipStream_t s)
{
    switch (pat) {
    case PAT_CYL: return launch_pat<PAT_CYL>(a, st, check, grid, block, s);
    case PAT_ELL: return launch_pat<PAT_ELL>(a, st, check, grid, block, s);
    default: return launch_pat<PAT_GEN>(a, st, check, grid, block, s);
    }
}

hipError_t launch_step(const StepArgs &a0, int pat, int st, bool check, bool eqw, int grid, int block, hipStream_t s)
{
    // Tile order. Grouped by XCD, the x3 pulls that straddle a cache line at
    // a tile boundary find it in their own L2: the 16-bit formats then fetch
    // 1.02x their algorithmic bytes instead of 1.39x at the same speed (they
    // are bound by arithmetic). The wide formats are bound by HBM, and there
    // interleaved tiles are faster (68.7 % against 66.4 % of 8 TB/s on the
    // cylinder sweep in FP32, 70.5 % against 65.1 % on the 96x192x192
    // instance): all XCDs then stream through neighbouring memory at once.
    // FP32 deals the queue in runs of four tiles: the four theta slabs of
    // a 256-column row (or four neighbouring chunks of a longer one) then
    // share the cross-section geometry and the straddled lines in one L2:
    // 68.3 % against 66.9 % of 8 TB/s on the uneven ellipsoid batch, equal
    // on the cylinder sweep and on the 96x192x192 instance. FP64 keeps every
    // eighth tile (72.3 % against 71.8 % with runs, same instance).
    StepArgs a = a0;
    a.xcd_group = (st == ST_F16 || st == ST_BF16) ? 1 : 0;
    a.group_log2 = st == ST_F32 ? 2 : 0;
    return eqw ? launch_step_eq(a, pat, st, check, grid, block, s) : launch_step_plain(a, pat, st, check, grid, block, s);
}

}  // namespace mlbm
