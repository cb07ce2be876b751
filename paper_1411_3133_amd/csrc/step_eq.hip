// Launchers of the fused step kernel (step_kernel.hpp) for batches with equilibrium walls (Sec. III).
#include "step_kernel.hpp"

namespace mlbm {

template <int PAT, int ST, bool CHECK>
static hipError_t launch_one(const StepArgs &a, int grid, int block, hipStream_t s)
{
    hipLaunchKernelGGL((step_kernel<PAT, ST, CHECK, true>), dim3(grid), dim3(block), 0, s, a);
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

hipError_t launch_step_eq(const StepArgs &a, int pat, int st, bool check, int grid, int block, hipStream_t s)
{
    switch (pat) {
    case PAT_CYL: return launch_pat<PAT_CYL>(a, st, check, grid, block, s);
    case PAT_ELL: return launch_pat<PAT_ELL>(a, st, check, grid, block, s);
    default: return launch_pat<PAT_GEN>(a, st, check, grid, block, s);
    }
}

}  // namespace mlbm
