// mm_fused.hip -- kernels of the fused stage pass and of the fused adjoint stage
// (bodies in mm_fused.hpp), the choice of row pairs per work-group, and their
// dispatch by padded x length.
#include "mm_fused.hpp"

namespace mm {

constexpr int kFusedPrefetchGroups = 256;

template <typename T, int P, int L, bool PREFETCH>
__global__ __launch_bounds__((fused_threads<P, L>())) void k_fused_stage(FusedStageArgs<T> a)
{
    __shared__ cpx<T> lds[3 * fused_region<P, L>()];
    __shared__ T cell[3 * 2 * L * (P / 2)];
    body_fused_stage<T, P, L, PREFETCH>(a, xcd_tile(blockIdx.x, gridDim.x), lds, cell);
}

template <typename T, int P, int L>
__global__ __launch_bounds__((fused_threads<P, L>())) void k_fused_adjoint(FusedAdjArgs<T> a)
{
    __shared__ cpx<T> lds[3 * fused_region<P, L>()];
    __shared__ T cell[3 * 2 * L * (P / 2)];
    body_fused_adjoint<T, P, L>(a, xcd_tile(blockIdx.x, gridDim.x), lds, cell);
}

template <typename T, int P>
static bool fused_dispatch(const FusedStageArgs<T>& a, int L, hipStream_t s)
{
    constexpr int TL = P / Sched<P>::R0;
    // launches of at most kFusedPrefetchGroups work-groups (no more than one per CU)
    // are latency-bound: their stage-update loads go out with the gather's.  On the
    // 128x128x1 film 49.9 -> 47.8 us per RK4 step; with more work-groups the lower
    // occupancy costs more (256x256x16 FP32 388 -> 404 us, 64^3 FP64 297 -> 318 us)
    auto go = [&](auto kern, auto kern_pre, int lines, int threads) {
        const int grid = a.g.nz * ((a.g.ny + 2 * lines - 1) / (2 * lines));
        if (grid <= kFusedPrefetchGroups)
            hipLaunchKernelGGL(kern_pre, dim3(grid), dim3(threads), 0, s, a);
        else
            hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), 0, s, a);
        return true;
    };
    if constexpr (fused_lds_bytes<T, P, 4>() <= kLdsBudget && 3 * 4 * TL <= 1024)
        if (L == 4) return go(k_fused_stage<T, P, 4, false>, k_fused_stage<T, P, 4, true>, 4, fused_threads<P, 4>());
    if constexpr (fused_lds_bytes<T, P, 2>() <= kLdsBudget && 3 * 2 * TL <= 1024)
        if (L == 2) return go(k_fused_stage<T, P, 2, false>, k_fused_stage<T, P, 2, true>, 2, fused_threads<P, 2>());
    if constexpr (fused_lds_bytes<T, P, 1>() <= kLdsBudget && 3 * TL <= 1024)
        if (L == 1) return go(k_fused_stage<T, P, 1, false>, k_fused_stage<T, P, 1, true>, 1, fused_threads<P, 1>());
    return false;
}

template <typename T>
bool launch_fused_stage(const FusedStageArgs<T>& a, int Px, int L, hipStream_t s)
{
    if (a.g.ny <= 0 || a.g.nz <= 0) return true;
    if (2 * a.g.nx > Px || a.g.per != 0) return false;
    switch (Px) {
    case 16: return fused_dispatch<T, 16>(a, L, s);
    case 32: return fused_dispatch<T, 32>(a, L, s);
    case 64: return fused_dispatch<T, 64>(a, L, s);
    case 96: return fused_dispatch<T, 96>(a, L, s);
    case 128: return fused_dispatch<T, 128>(a, L, s);
    case 160: return fused_dispatch<T, 160>(a, L, s);
    case 192: return fused_dispatch<T, 192>(a, L, s);
    case 224: return fused_dispatch<T, 224>(a, L, s);
    case 256: return fused_dispatch<T, 256>(a, L, s);
    case 512: return fused_dispatch<T, 512>(a, L, s);
    case 1024: return fused_dispatch<T, 1024>(a, L, s);
    default: return false;
    }
}

template <typename T, int P>
static bool fused_adj_dispatch(const FusedAdjArgs<T>& a, int L, hipStream_t s)
{
    constexpr int TL = P / Sched<P>::R0;
    auto go = [&](auto kern, int lines, int threads) {
        const int grid = a.a.nz * ((a.a.ny + 2 * lines - 1) / (2 * lines));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), 0, s, a);
        return true;
    };
    if constexpr (fused_lds_bytes<T, P, 4>() <= kLdsBudget && 3 * 4 * TL <= 1024)
        if (L == 4) return go(k_fused_adjoint<T, P, 4>, 4, fused_threads<P, 4>());
    if constexpr (fused_lds_bytes<T, P, 2>() <= kLdsBudget && 3 * 2 * TL <= 1024)
        if (L == 2) return go(k_fused_adjoint<T, P, 2>, 2, fused_threads<P, 2>());
    if constexpr (fused_lds_bytes<T, P, 1>() <= kLdsBudget && 3 * TL <= 1024)
        if (L == 1) return go(k_fused_adjoint<T, P, 1>, 1, fused_threads<P, 1>());
    return false;
}

template <typename T>
bool launch_fused_adjoint(const FusedAdjArgs<T>& a, int Px, int L, hipStream_t s)
{
    if (a.a.ny <= 0 || a.a.nz <= 0) return true;
    if (2 * a.a.nx > Px || a.a.per != 0) return false;
    switch (Px) {
    case 16: return fused_adj_dispatch<T, 16>(a, L, s);
    case 32: return fused_adj_dispatch<T, 32>(a, L, s);
    case 64: return fused_adj_dispatch<T, 64>(a, L, s);
    case 96: return fused_adj_dispatch<T, 96>(a, L, s);
    case 128: return fused_adj_dispatch<T, 128>(a, L, s);
    case 160: return fused_adj_dispatch<T, 160>(a, L, s);
    case 192: return fused_adj_dispatch<T, 192>(a, L, s);
    case 224: return fused_adj_dispatch<T, 224>(a, L, s);
    case 256: return fused_adj_dispatch<T, 256>(a, L, s);
    case 512: return fused_adj_dispatch<T, 512>(a, L, s);
    case 1024: return fused_adj_dispatch<T, 1024>(a, L, s);
    default: return false;
    }
}

// Lines per work-group: about 256 work-groups or more where the grid has the rows
// (ny nz of them; latency-bound sizes gain from spreading over CUs), within the
// LDS budget.
template <typename T, int P>
static int fused_lines_for(int rows)
{
    constexpr int TL = P / Sched<P>::R0;
    // at most 512 threads (two waves per SIMD leave 256 registers a thread), and one
    // line at 512 points or more: the larger FP64 shapes spill, and in FP32 two lines
    // of 512 (154 instead of 126 registers) measured slower on the 256x256x16 film
    // (423 against 392 us per RK4 step)
    const int want = P >= 512 ? 1 : (rows >= 2048 ? 4 : (rows >= 1024 ? 2 : 1));
    for (int L = want; L >= 1; L /= 2) {
        if (L == 4 && fused_lds_bytes<T, P, 4>() <= kLdsBudget && 12 * TL <= 512) return 4;
        if (L == 2 && fused_lds_bytes<T, P, 2>() <= kLdsBudget && 6 * TL <= 512) return 2;
        if (L == 1 && fused_lds_bytes<T, P, 1>() <= kLdsBudget && 3 * TL <= 512) return 1;
    }
    return 0;
}

template <typename T>
static int fused_lines_t(int Px, int rows)
{
    switch (Px) {
    case 16: return fused_lines_for<T, 16>(rows);
    case 32: return fused_lines_for<T, 32>(rows);
    case 64: return fused_lines_for<T, 64>(rows);
    case 96: return fused_lines_for<T, 96>(rows);
    case 128: return fused_lines_for<T, 128>(rows);
    case 160: return fused_lines_for<T, 160>(rows);
    case 192: return fused_lines_for<T, 192>(rows);
    case 224: return fused_lines_for<T, 224>(rows);
    case 256: return fused_lines_for<T, 256>(rows);
    case 512: return fused_lines_for<T, 512>(rows);
    case 1024: return fused_lines_for<T, 1024>(rows);
    default: return 0;
    }
}

int fused_stage_lines(int Px, int nx, int rows, size_t esz)
{
    if (2 * nx > Px) return 0;
    return esz == 8 ? fused_lines_t<double>(Px, rows) : fused_lines_t<float>(Px, rows);
}

template bool launch_fused_stage<float>(const FusedStageArgs<float>&, int, int, hipStream_t);
template bool launch_fused_adjoint<float>(const FusedAdjArgs<float>&, int, int, hipStream_t);
template bool launch_fused_adjoint<double>(const FusedAdjArgs<double>&, int, int, hipStream_t);
template bool launch_fused_stage<double>(const FusedStageArgs<double>&, int, int, hipStream_t);

}  // namespace mm
