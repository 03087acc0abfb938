// mm_fast.hip -- single-grid kernels of the size-specialised FFT passes (bodies
// in mm_fast.hpp) and their dispatch by padded size.
#include "mm_fast.hpp"

namespace mm {

// FULL: whole lines (a periodic axis, n = P); otherwise the padding half is pruned
template <typename T, int P, bool INV, bool FULL>
__global__ __launch_bounds__(256) void k_yline(YLineArgs a)
{
    __shared__ cpx<T> lds[yline_lds_elems<P>()];
    body_yline<T, P, INV, FULL>(a, xcd_tile(blockIdx.x, gridDim.x), lds);
}

template <typename T, int P, int L, bool FULL>
__global__ __launch_bounds__(L * (P / Sched<P>::R0)) void k_xfwd(XLineArgs a)
{
    __shared__ cpx<T> lds[xfwd_lds_elems<P, L>()];
    body_xfwd<T, P, L, FULL>(a, xcd_tile(blockIdx.x, gridDim.x), lds);
}

template <typename T, int P, int C>
__global__ __launch_bounds__(3 * C * (P / Sched<P>::R0)) void k_kspace_zl(KzArgs a)
{
    __shared__ cpx<T> lds[3 * C * padded_len<P>()];
    body_kspace_zl<T, P, C>(a, xcd_tile(blockIdx.x, gridDim.x), lds);
}

template <typename T, int P, int L, bool FULL>
__global__ __launch_bounds__(L * (P / Sched<P>::R0)) void k_xinv(XLineArgs a)
{
    __shared__ cpx<T> lds[xinv_lds_elems<P, L>()];
    body_xinv<T, P, L, FULL>(a, xcd_tile(blockIdx.x, gridDim.x), lds);
}

template <typename T, int PZ>
__global__ __launch_bounds__(3 * kspace_z_cols<T>()) void k_kspace_z(KzArgs a)
{
    __shared__ cpx<T> sh[kspace_z_lds_elems<T, PZ>()];
    body_kspace_z<T, PZ>(a, xcd_tile(blockIdx.x, gridDim.x), sh);
}

template <typename T, int PZ>
__global__ __launch_bounds__(6 * kspace_z_split_cols()) void k_kspace_z_split(KzArgs a)
{
    __shared__ cpx<T> sh[3 * PZ * kspace_z_split_cols()];
    body_kspace_z_split<T, PZ>(a, xcd_tile(blockIdx.x, gridDim.x), sh);
}

template <typename T, int P, bool FULL, int L>
__global__ __launch_bounds__(3 * L * (P / Sched<P>::R0)) void k_kspace_y(KyArgs a)
{
    __shared__ cpx<T> lds[kspace_y_lds_elems<P, L>()];
    body_kspace_y<T, P, FULL, L>(a, xcd_tile(blockIdx.x, gridDim.x), lds);
}

template <typename T, int P, bool FULL>
__global__ __launch_bounds__(6 * ky2_lines<P>() * (P / Sched<P>::R0)) void k_kspace_y2(Ky2Args a)
{
    __shared__ cpx<T> lds[kspace_y2_lds_elems<P>()];
    body_kspace_y2<T, P, FULL>(a, xcd_tile(blockIdx.x, gridDim.x), lds);
}

// ------------------------------------------------------------------ dispatch
template <typename T, bool INV, bool FULL>
static bool yline_dispatch(const YLineArgs& a, int P, hipStream_t s)
{
    auto go = [&](auto kern, int L, int tl) {
        const int grid = (a.nlines + L - 1) / L;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(L * tl), 0, s, a);
        return true;
    };
#define MM_YCASE(PP) \
    case PP: return go(k_yline<T, PP, INV, FULL>, yline_lines<PP>(), PP / Sched<PP>::R0);
    switch (P) {
        MM_YCASE(16)
        MM_YCASE(32)
        MM_YCASE(64)
        MM_YCASE(96)
        MM_YCASE(128)
        MM_YCASE(160)
        MM_YCASE(192)
        MM_YCASE(224)
        MM_YCASE(256)
        MM_YCASE(512)
        MM_YCASE(1024)
        MM_YCASE(2048)
    default: return false;
    }
#undef MM_YCASE
}

template <typename T>
bool launch_yline(const YLineArgs& a, int P, int inverse, hipStream_t s)
{
    if (a.nlines <= 0) return true;
    // the bodies prune the zero half of a forward line and the unused half of an
    // inverse one when the valid samples fit the first half; whole lines (a
    // periodic axis) take the FULL instantiation
    const int n = inverse ? a.nout : a.nin;
    if (n > P) return false;
    if (2 * n > P)
        return inverse ? yline_dispatch<T, true, true>(a, P, s) : yline_dispatch<T, false, true>(a, P, s);
    return inverse ? yline_dispatch<T, true, false>(a, P, s) : yline_dispatch<T, false, false>(a, P, s);
}

template <typename T, bool INV, int L, bool FULL>
static bool xline_dispatch(const XLineArgs& a, int P, hipStream_t s)
{
    auto go = [&](auto kern, int tl) {
        const int rows = 2 * L;
        const int grid = a.nplanes * ((a.ny + rows - 1) / rows);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(L * tl), 0, s, a);
        return true;
    };
#define MM_XCASE(PP)                                                                  \
    case PP:                                                                          \
        if constexpr (x_lds_bytes<T, PP, L>() <= kLdsBudget &&                        \
                      L * (PP / Sched<PP>::R0) <= 1024)                               \
            return INV ? go(k_xinv<T, PP, L, FULL>, PP / Sched<PP>::R0)               \
                       : go(k_xfwd<T, PP, L, FULL>, PP / Sched<PP>::R0);              \
        return false;
    switch (P) {
        MM_XCASE(16)
        MM_XCASE(32)
        MM_XCASE(64)
        MM_XCASE(96)
        MM_XCASE(128)
        MM_XCASE(160)
        MM_XCASE(192)
        MM_XCASE(224)
        MM_XCASE(256)
        MM_XCASE(512)
        MM_XCASE(1024)
        MM_XCASE(2048)
    default: return false;
    }
#undef MM_XCASE
}

template <typename T, bool FULL>
static bool xline_lines(const XLineArgs& a, int P, int inverse, hipStream_t s)
{
    if (a.lines == 4)
        return inverse ? xline_dispatch<T, true, 4, FULL>(a, P, s) : xline_dispatch<T, false, 4, FULL>(a, P, s);
    if (a.lines == 16)
        return inverse ? xline_dispatch<T, true, 16, FULL>(a, P, s)
                       : xline_dispatch<T, false, 16, FULL>(a, P, s);
    return inverse ? xline_dispatch<T, true, 8, FULL>(a, P, s) : xline_dispatch<T, false, 8, FULL>(a, P, s);
}

template <typename T>
bool launch_xline(const XLineArgs& a, int P, int inverse, hipStream_t s)
{
    if (a.nplanes <= 0 || a.ny <= 0) return true;
    if (a.nx > P) return false;
    // valid samples in the first half: pruned bodies; whole lines (periodic x): FULL
    return 2 * a.nx > P ? xline_lines<T, true>(a, P, inverse, s) : xline_lines<T, false>(a, P, inverse, s);
}

template <typename T>
bool launch_kspace_z(const KzArgs& a, int PZ, hipStream_t s)
{
    constexpr int ZC = kspace_z_cols<T>();
    const int grid = (a.ncols + ZC - 1) / ZC;
    if (grid <= 0) return true;
    // the body indexes the spectrum and the octant with 32-bit offsets: larger
    // grids take the k-space pass with 64-bit offsets
    if (3 * a.comp_stride > INT32_MAX || 6 * a.k_cs > INT32_MAX) return false;
    if constexpr (sizeof(T) == 8) {
        // FP64 with the upper half of each z line zero: two lanes per line
        if ((PZ == 16 || PZ == 32) && 2 * a.nz <= PZ) {
            constexpr int SC = kspace_z_split_cols();
            const int sgrid = (a.ncols + SC - 1) / SC;
            if (PZ == 16)
                hipLaunchKernelGGL((k_kspace_z_split<T, 16>), dim3(sgrid), dim3(6 * SC), 0, s, a);
            else
                hipLaunchKernelGGL((k_kspace_z_split<T, 32>), dim3(sgrid), dim3(6 * SC), 0, s, a);
            return true;
        }
    }
    // lines of 128 points or more: C columns a work-group, register radix stages (FP64
    // lines of 1024 points take the LDS-staged pass, launch_kspace_fixed)
    auto zl = [&](auto kern, int C, int tl) {
        const int zgrid = (a.ncols + C - 1) / C;
        hipLaunchKernelGGL(kern, dim3(zgrid), dim3(3 * C * tl), 0, s, a);
        return true;
    };
    if (PZ >= 128 && 2 * a.nz <= PZ) {
        switch (PZ) {
        case 128: return zl(k_kspace_zl<T, 128, kzl_cols<T, 128>()>, kzl_cols<T, 128>(), 128 / Sched<128>::R0);
        case 256: return zl(k_kspace_zl<T, 256, kzl_cols<T, 256>()>, kzl_cols<T, 256>(), 256 / Sched<256>::R0);
        case 512: return zl(k_kspace_zl<T, 512, kzl_cols<T, 512>()>, kzl_cols<T, 512>(), 512 / Sched<512>::R0);
        case 1024:
            if constexpr (sizeof(T) == 4)
                return zl(k_kspace_zl<T, 1024, kzl_cols<T, 1024>()>, kzl_cols<T, 1024>(), 1024 / Sched<1024>::R0);
            return false;
        default: return false;
        }
    }
    switch (PZ) {
    case 2: hipLaunchKernelGGL((k_kspace_z<T, 2>), dim3(grid), dim3(3 * ZC), 0, s, a); return true;
    case 4: hipLaunchKernelGGL((k_kspace_z<T, 4>), dim3(grid), dim3(3 * ZC), 0, s, a); return true;
    case 8: hipLaunchKernelGGL((k_kspace_z<T, 8>), dim3(grid), dim3(3 * ZC), 0, s, a); return true;
    case 16: hipLaunchKernelGGL((k_kspace_z<T, 16>), dim3(grid), dim3(3 * ZC), 0, s, a); return true;
    case 32: hipLaunchKernelGGL((k_kspace_z<T, 32>), dim3(grid), dim3(3 * ZC), 0, s, a); return true;
    case 64:
        if constexpr (sizeof(T) == 4) {
            hipLaunchKernelGGL((k_kspace_z<T, 64>), dim3(grid), dim3(3 * ZC), 0, s, a);
            return true;
        }
        return false;
    default: return false;
    }
}

// Grids of 64 to 256 x bins (small, latency-bound ones) take one bin per
// work-group: more work-groups, each a single wave or two (128x128x1, 129 bins,
// FP32 RK4: 65.9 -> 62.7 us per step; 32x8x1, 33 bins: 40.6 -> 42.0, so not there).
constexpr int kKySingleBinMinBins = 64, kKySingleBinMaxBins = 256;

template <typename T, bool FULL>
static bool kspace_y_dispatch(const KyArgs& a, int P, hipStream_t s)
{
    auto go = [&](auto kern, int L, int nt) {
        const int grid = (a.hx + L - 1) / L;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(nt), 0, s, a);
        return true;
    };
#define MM_KYCASE(PP)                                                                          \
    case PP:                                                                                   \
        if (a.hx >= kKySingleBinMinBins && a.hx <= kKySingleBinMaxBins)                        \
            return go(k_kspace_y<T, PP, FULL, 1>, 1, 3 * (PP / Sched<PP>::R0));                \
        return go(k_kspace_y<T, PP, FULL, ky_lines<PP>()>, ky_lines<PP>(),                      \
                  3 * ky_lines<PP>() * (PP / Sched<PP>::R0));
    switch (P) {
        MM_KYCASE(16)
        MM_KYCASE(32)
        MM_KYCASE(64)
        MM_KYCASE(96)
        MM_KYCASE(128)
        MM_KYCASE(160)
        MM_KYCASE(192)
        MM_KYCASE(224)
        MM_KYCASE(256)
        MM_KYCASE(512)
        MM_KYCASE(1024)
    default: return false;
    }
#undef MM_KYCASE
}

template <typename T>
bool launch_kspace_y(const KyArgs& a, int P, hipStream_t s)
{
    if (a.hx <= 0) return true;
    if (a.ny > P) return false;
    // valid samples in the first half: pruned body; whole lines (periodic y): FULL
    if (2 * a.ny > P) return kspace_y_dispatch<T, true>(a, P, s);
    return kspace_y_dispatch<T, false>(a, P, s);
}

template <typename T, bool FULL>
static bool kspace_y2_dispatch(const Ky2Args& a, int P, hipStream_t s)
{
    auto go = [&](auto kern, int L, int nt) {
        const int grid = (a.hx + L - 1) / L;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(nt), 0, s, a);
        return true;
    };
#define MM_KY2CASE(PP)                                                                          \
    case PP:                                                                                    \
        if constexpr (kspace_y2_lds_elems<PP>() * (int)sizeof(cpx<T>) <= kLdsBudget)           \
            return go(k_kspace_y2<T, PP, FULL>, ky2_lines<PP>(), 6 * ky2_lines<PP>() * (PP / Sched<PP>::R0)); \
        return false;
    switch (P) {
        MM_KY2CASE(16)
        MM_KY2CASE(32)
        MM_KY2CASE(64)
        MM_KY2CASE(96)
        MM_KY2CASE(128)
        MM_KY2CASE(160)
        MM_KY2CASE(192)
        MM_KY2CASE(224)
        MM_KY2CASE(256)
        MM_KY2CASE(512)
        MM_KY2CASE(1024)
    default: return false;
    }
#undef MM_KY2CASE
}

template <typename T>
bool launch_kspace_y2(const Ky2Args& a, int P, hipStream_t s)
{
    if (a.hx <= 0) return true;
    if (a.ny > P) return false;
    // valid samples in the first half: pruned body; whole lines (periodic y): FULL
    if (2 * a.ny > P) return kspace_y2_dispatch<T, true>(a, P, s);
    return kspace_y2_dispatch<T, false>(a, P, s);
}

int fast_ky2_lines(int P)
{
    switch (P) {
    case 16: return ky2_lines<16>();
    case 32: return ky2_lines<32>();
    case 64: return ky2_lines<64>();
    case 96: return ky2_lines<96>();
    case 128: return ky2_lines<128>();
    case 160: return ky2_lines<160>();
    case 192: return ky2_lines<192>();
    case 224: return ky2_lines<224>();
    case 256: return ky2_lines<256>();
    case 512: return ky2_lines<512>();
    case 1024: return ky2_lines<1024>();
    default: return 0;
    }
}

int fast_first_radix(int P)
{
    switch (P) {
    case 2: return Sched<2>::R0;
    case 4: return Sched<4>::R0;
    case 8: return Sched<8>::R0;
    case 16: return Sched<16>::R0;
    case 32: return Sched<32>::R0;
    case 64: return Sched<64>::R0;
    case 96: return Sched<96>::R0;
    case 128: return Sched<128>::R0;
    case 160: return Sched<160>::R0;
    case 192: return Sched<192>::R0;
    case 224: return Sched<224>::R0;
    case 256: return Sched<256>::R0;
    case 512: return Sched<512>::R0;
    case 1024: return Sched<1024>::R0;
    case 2048: return Sched<2048>::R0;
    default: return 0;
    }
}

int fast_ky_lines(int P)
{
    switch (P) {
    case 16: return ky_lines<16>();
    case 32: return ky_lines<32>();
    case 64: return ky_lines<64>();
    case 96: return ky_lines<96>();
    case 128: return ky_lines<128>();
    case 160: return ky_lines<160>();
    case 192: return ky_lines<192>();
    case 224: return ky_lines<224>();
    case 256: return ky_lines<256>();
    case 512: return ky_lines<512>();
    case 1024: return ky_lines<1024>();
    default: return 0;
    }
}

template bool launch_kspace_y2<float>(const Ky2Args&, int, hipStream_t);
template bool launch_kspace_y2<double>(const Ky2Args&, int, hipStream_t);
template bool launch_kspace_y<float>(const KyArgs&, int, hipStream_t);
template bool launch_kspace_y<double>(const KyArgs&, int, hipStream_t);
template bool launch_yline<float>(const YLineArgs&, int, int, hipStream_t);
template bool launch_yline<double>(const YLineArgs&, int, int, hipStream_t);
template bool launch_xline<float>(const XLineArgs&, int, int, hipStream_t);
template bool launch_xline<double>(const XLineArgs&, int, int, hipStream_t);
template bool launch_kspace_z<float>(const KzArgs&, int, hipStream_t);
template bool launch_kspace_z<double>(const KzArgs&, int, hipStream_t);

}  // namespace mm
