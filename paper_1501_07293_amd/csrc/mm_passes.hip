// mm_passes.hip -- the FFT passes of the demag convolution (Sec. 2.3, Eq. 14
// with the zero padding of Fig. 1 / Listing 4), as LDS-staged batched FFTs.
//
// Per field evaluation on an nx x ny x nz grid padded to Px x Py x Pz:
//   row_r2c : x, real -> half spectrum, input pruned to nx of Px
//   col_fft : y forward (input pruned to ny of Py)             [3-D grids]
//   kspace  : last axis forward, Eq. 14 product, last axis inverse
//   col_fft : y inverse (output truncated to ny)               [3-D grids]
//   row_c2r : x inverse, output truncated to nx
// The padded array is never materialised: pruned inputs are zeros filled in
// LDS and truncated outputs are never stored.
#include "mm_generic.hpp"

namespace mm {

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_row_r2c(RowR2CArgs a)
{
    __shared__ cpx<T> lds[lds_elems(NT)];
    body_row_r2c<T, NT>(a, a.pl, xcd_tile(blockIdx.x, gridDim.x), lds);
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_row_c2r(RowC2RArgs a)
{
    __shared__ cpx<T> lds[lds_elems(NT)];
    body_row_c2r<T, NT>(a, a.pl, xcd_tile(blockIdx.x, gridDim.x), lds);
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_col_fft(ColArgs a)
{
    __shared__ cpx<T> lds[lds_elems(NT)];
    body_col_fft<T, NT>(a, a.pl, xcd_tile(blockIdx.x, gridDim.x), lds);
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_kspace_yz(KyzArgs a)
{
    __shared__ cpx<T> lds[lds_elems(NT)];
    body_kspace_yz<T, NT>(a, xcd_tile(blockIdx.x, gridDim.x), lds);
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_demag_1wg(Demag1Args a)
{
    __shared__ cpx<T> lds[lds_elems(NT)];
    body_demag_1wg<T, NT>(a, lds);
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_kspace(KspArgs a)
{
    __shared__ cpx<T> lds[lds_elems(NT)];
    body_kspace<T, NT>(a, a.pl, xcd_tile(blockIdx.x, gridDim.x), lds);
}

// The last-axis k-space pass for power-of-two lengths beyond the register-resident
// z pass (PZ >= 128): the same body with the length fixed at compile time (every
// radix, span and twiddle stride a constant); a work-group of NT threads holds
// 16 NT / (3 PZ) columns.
template <typename T, int NT, int PZ>
__global__ __launch_bounds__(NT) void k_kspace_fixed(KspArgs a)
{
    __shared__ cpx<T> lds[lds_elems(NT)];
    body_kspace<T, NT, PZ>(a, a.pl, xcd_tile(blockIdx.x, gridDim.x), lds);
}

template <typename T, int NT, int PZ>
static bool kspace_fixed_go(KspArgs a, hipStream_t s)
{
    constexpr int TW = kElemsPerThread * NT / (3 * PZ);
    static_assert(TW >= 1 && lds_elems(NT) * sizeof(cpx<T>) <= 160 * 1024, "k-space tile");
    a.tw_cols = TW;
    const int grid = (a.ncols + TW - 1) / TW;
    if (grid > 0) hipLaunchKernelGGL((k_kspace_fixed<T, NT, PZ>), dim3(grid), dim3(NT), 0, s, a);
    return true;
}

template <typename T>
bool launch_kspace_fixed(const KspArgs& a, int P, hipStream_t s)
{
    // 256 threads: 5 columns at PZ = 256 and 4 work-groups per CU (FP32) measured
    // faster than 384 (8 columns) or 768 (16 columns, one work-group per CU).  At
    // PZ = 512, 256 threads hold 2 columns; 512 threads (5 columns) measured faster
    // on the 256^3 cube (Euler step FP32 3.04 -> 2.97 ms, FP64 5.30 -> 5.08 ms),
    // 1024 threads (10 columns, FP32) no better (3.09 ms)
    constexpr int NT = 256;
    switch (P) {
    case 128: return kspace_fixed_go<T, NT, 128>(a, s);
    case 256: return kspace_fixed_go<T, NT, 256>(a, s);
    case 512: return kspace_fixed_go<T, 512, 512>(a, s);
    case 1024: return kspace_fixed_go<T, NT, 1024>(a, s);
    default: return false;
    }
}

// ------------------------------------------------------------------ launchers
#define MM_LAUNCH_NT(kern, T, grid, nt, s, arg)                                              \
    do {                                                                                     \
        if ((nt) == 512)                                                                     \
            hipLaunchKernelGGL((kern<T, 512>), dim3(grid), dim3(512), 0, s, arg);            \
        else                                                                                 \
            hipLaunchKernelGGL((kern<T, 256>), dim3(grid), dim3(256), 0, s, arg);            \
    } while (0)

template <typename T>
hipError_t launch_row_r2c(const RowR2CArgs& a, int nt, hipStream_t s)
{
    const int npairs = (a.nrows + 1) / 2;
    const int grid = (npairs + a.lines_per_wg - 1) / a.lines_per_wg;
    if (grid <= 0) return hipSuccess;
    MM_LAUNCH_NT(k_row_r2c, T, grid, nt, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_row_c2r(const RowC2RArgs& a, int nt, hipStream_t s)
{
    const int npairs = (a.nrows + 1) / 2;
    const int grid = (npairs + a.lines_per_wg - 1) / a.lines_per_wg;
    if (grid <= 0) return hipSuccess;
    MM_LAUNCH_NT(k_row_c2r, T, grid, nt, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_col_fft(const ColArgs& a, int nt, hipStream_t s)
{
    const int grid = a.nplanes * ((a.ncols + a.tw_cols - 1) / a.tw_cols);
    if (grid <= 0) return hipSuccess;
    MM_LAUNCH_NT(k_col_fft, T, grid, nt, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_kspace(const KspArgs& a, int nt, hipStream_t s)
{
    const int grid = (a.ncols + a.tw_cols - 1) / a.tw_cols;
    if (grid <= 0) return hipSuccess;
    MM_LAUNCH_NT(k_kspace, T, grid, nt, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_kspace_yz(const KyzArgs& a, int nt, hipStream_t s)
{
    if (a.hx <= 0) return hipSuccess;
    MM_LAUNCH_NT(k_kspace_yz, T, a.hx, nt, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_demag_1wg(const Demag1Args& a, int nt, hipStream_t s)
{
    // the padded volume of the three components must fit the work-group's LDS
    if (3LL * a.Px * a.Py * a.Pz > (int64_t)kElemsPerThread * nt) return hipErrorInvalidValue;
    MM_LAUNCH_NT(k_demag_1wg, T, 1, nt, s, a);
    return hipGetLastError();
}

template hipError_t launch_row_r2c<float>(const RowR2CArgs&, int, hipStream_t);
template hipError_t launch_row_r2c<double>(const RowR2CArgs&, int, hipStream_t);
template hipError_t launch_row_c2r<float>(const RowC2RArgs&, int, hipStream_t);
template hipError_t launch_row_c2r<double>(const RowC2RArgs&, int, hipStream_t);
template hipError_t launch_col_fft<float>(const ColArgs&, int, hipStream_t);
template hipError_t launch_col_fft<double>(const ColArgs&, int, hipStream_t);
template bool launch_kspace_fixed<float>(const KspArgs&, int, hipStream_t);
template bool launch_kspace_fixed<double>(const KspArgs&, int, hipStream_t);
template hipError_t launch_kspace<float>(const KspArgs&, int, hipStream_t);
template hipError_t launch_kspace<double>(const KspArgs&, int, hipStream_t);
template hipError_t launch_kspace_yz<float>(const KyzArgs&, int, hipStream_t);
template hipError_t launch_kspace_yz<double>(const KyzArgs&, int, hipStream_t);
template hipError_t launch_demag_1wg<float>(const Demag1Args&, int, hipStream_t);
template hipError_t launch_demag_1wg<double>(const Demag1Args&, int, hipStream_t);

}  // namespace mm
