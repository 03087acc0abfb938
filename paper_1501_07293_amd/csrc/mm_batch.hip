// mm_batch.hip -- the batched form: many independent grids of uneven sizes
// advanced together.  Every pass of a field evaluation (and the LLG stage) is
// ONE kernel launch over all grids: the launch's tiles are the concatenation
// of every grid's tiles, and a work-group finds its grid by binary search in
// the per-pass tile prefix sums, then runs the same device body as the
// single-grid runtime-radix kernels with that grid's descriptor.
#include "mm_fast.hpp"
#include "mm_generic.hpp"
#include "mm_llg_body.hpp"

namespace mm {

constexpr int kBatchNT = 256;
static_assert(kBatchNT == kLlgNT, "the batched LLG pass launches kLlgNT threads per work-group");

__device__ inline int find_sample(const int* prefix, int n, int tile)
{
    int lo = 0, hi = n;  // prefix[lo] <= tile < prefix[hi]; empty grids are skipped
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= tile)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

template <typename T>
__global__ __launch_bounds__(kBatchNT) void kb_xfwd(BatchPass<T> p)
{
    __shared__ cpx<T> lds[lds_elems(kBatchNT)];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int s = find_sample(p.prefix, p.n, tile);
    const BatchDesc& d = p.d[s];
    RowR2CArgs a{};
    a.in = p.in + d.moff;
    a.in_row_stride = d.nx;
    a.nrows = 3 * d.nz * d.ny;
    a.nvalid = d.nx;
    a.out = p.S + d.soff;
    a.rows_per_plane = d.ny;
    a.out_plane_stride = (int64_t)d.hx * d.Sy;
    a.rstride = 1;
    a.kstride = d.Sy;
    a.hx = d.hx;
    a.lines_per_wg = d.x_lines;
    a.tw = p.tw + d.twx;
    body_row_r2c<T, kBatchNT>(a, d.fx, tile - p.prefix[s], lds);
}

template <typename T>
__global__ __launch_bounds__(kBatchNT) void kb_y(BatchPass<T> p, int inverse)
{
    __shared__ cpx<T> lds[lds_elems(kBatchNT)];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int s = find_sample(p.prefix, p.n, tile);
    const BatchDesc& d = p.d[s];
    LineArgs a{};
    a.buf = p.S + d.soff;
    a.nlines = 3 * d.nz * d.hx;
    a.line_stride = d.Sy;
    a.nin = inverse ? d.Py : d.ny;
    a.nout = inverse ? d.ny : d.Py;
    a.inverse = inverse;
    a.lines_per_wg = d.y_lines;
    a.tw = p.tw + d.twy;
    body_line_c2c<T, kBatchNT>(a, d.fy, tile - p.prefix[s], lds);
}

template <typename T>
__global__ __launch_bounds__(kBatchNT) void kb_kspace(BatchPass<T> p)
{
    __shared__ cpx<T> lds[lds_elems(kBatchNT)];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int s = find_sample(p.prefix, p.n, tile);
    const BatchDesc& d = p.d[s];
    const int64_t plane = (int64_t)d.hx * d.Sy;
    KspArgs a{};
    a.buf = p.S + d.soff;
    a.kern = p.kern + d.koff;
    a.hx = d.hx;
    a.Py = d.Py;
    a.Pz = d.Pz;
    a.k_cs = d.oct;
    a.k_zs = (int64_t)d.hx * (d.Py / 2 + 1);
    a.k_xs = d.Py / 2 + 1;
    a.tw_cols = d.k_tw;
    if (d.three_d) {
        a.ncomp = 6;
        a.comp_stride = (int64_t)d.nz * plane;
        a.ncols = (int)plane;
        a.cols_per_row = (int)plane;
        a.row2_stride = 0;
        a.es = plane;
        a.nvalid = d.nz;
        a.axis_is_z = 1;
        a.tw = p.tw + d.twz;
        body_kspace<T, kBatchNT>(a, d.fz, tile - p.prefix[s], lds);
    } else {
        a.ncomp = 4;
        a.comp_stride = plane;
        a.ncols = d.hx;
        a.cols_per_row = 1;
        a.row2_stride = d.Sy;
        a.es = 1;
        a.nvalid = d.ny;
        a.axis_is_z = 0;
        a.tw = p.tw + d.twy;
        body_kspace<T, kBatchNT>(a, d.fy, tile - p.prefix[s], lds);
    }
}

template <typename T>
__global__ __launch_bounds__(kBatchNT) void kb_xinv(BatchPass<T> p)
{
    __shared__ cpx<T> lds[lds_elems(kBatchNT)];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int s = find_sample(p.prefix, p.n, tile);
    const BatchDesc& d = p.d[s];
    RowC2RArgs a{};
    a.in = p.S + d.soff;
    a.rows_per_plane = d.ny;
    a.in_plane_stride = (int64_t)d.hx * d.Sy;
    a.rstride = 1;
    a.kstride = d.Sy;
    a.hx = d.hx;
    a.nrows = 3 * d.nz * d.ny;
    a.out = p.out + d.moff;
    a.out_row_stride = d.nx;
    a.nvalid = d.nx;
    a.lines_per_wg = d.x_lines;
    a.tw = p.tw + d.twx;
    body_row_c2r<T, kBatchNT>(a, d.fx, tile - p.prefix[s], lds);
}

// One launch per LLG class: the grids whose planes per thread are KZ.
template <typename T, int KZ>
__global__ __launch_bounds__(kBatchNT) void kbf_llg(BatchClass<T> c, BatchLlg<T> g)
{
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int q = find_sample(c.prefix, c.nmem, tile);
    const BatchDesc& d = c.d[c.members[q]];
    LlgArgs<T> a{};
    a.ms = g.ms + d.moff;
    a.mn = g.mn + d.moff;
    a.acc = g.acc + d.moff;
    a.out = g.out + d.moff;
    a.hd = g.hd ? g.hd + d.moff : nullptr;
    a.ku = nullptr;
    a.nx = d.nx;
    a.ny = d.ny;
    a.nz = d.nz;
    a.N = (int64_t)d.nx * d.ny * d.nz;
    a.cex = (T)d.cex;
    a.can = (T)d.can;
    a.hx = (T)d.hred[0];
    a.hy = (T)d.hred[1];
    a.hz = (T)d.hred[2];
    a.alpha = (T)d.alpha;
    a.gdt = (T)d.gdt;
    a.stage = g.stage;
    body_llg_stage<T, KZ>(a, tile - c.prefix[q], threadIdx.x);
}

template <typename T>
hipError_t launch_batch_llg(int kz, const BatchClass<T>& c, int tiles, const BatchLlg<T>& g, hipStream_t s)
{
    if (tiles <= 0) return hipSuccess;
    switch (kz) {
    case 1: hipLaunchKernelGGL((kbf_llg<T, 1>), dim3(tiles), dim3(kBatchNT), 0, s, c, g); break;
    case kLlgZ: hipLaunchKernelGGL((kbf_llg<T, kLlgZ>), dim3(tiles), dim3(kBatchNT), 0, s, c, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t launch_batch_llg<float>(int, const BatchClass<float>&, int, const BatchLlg<float>&,
                                            hipStream_t);
template hipError_t launch_batch_llg<double>(int, const BatchClass<double>&, int, const BatchLlg<double>&,
                                             hipStream_t);

// ---- size classes: the specialised bodies, one launch per padded length
template <typename T, int P, int L>
__global__ __launch_bounds__(L * (P / Sched<P>::R0)) void kbf_xfwd(BatchClass<T> c)
{
    __shared__ cpx<T> lds[xfwd_lds_elems<P, L>()];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int q = find_sample(c.prefix, c.nmem, tile);
    const BatchDesc& d = c.d[c.members[q]];
    const XLineArgs a{c.in + d.moff, c.S + d.soff, 3 * d.nz, d.ny, d.nx, d.Sy, c.tw + d.twx, L};
    body_xfwd<T, P, L>(a, tile - c.prefix[q], lds);
}

template <typename T, int P, int L>
__global__ __launch_bounds__(L * (P / Sched<P>::R0)) void kbf_xinv(BatchClass<T> c)
{
    __shared__ cpx<T> lds[xinv_lds_elems<P, L>()];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int q = find_sample(c.prefix, c.nmem, tile);
    const BatchDesc& d = c.d[c.members[q]];
    const XLineArgs a{c.S + d.soff, c.out + d.moff, 3 * d.nz, d.ny, d.nx, d.Sy, c.tw + d.twx, L};
    body_xinv<T, P, L>(a, tile - c.prefix[q], lds);
}

template <typename T, int P, bool INV>
__global__ __launch_bounds__(yline_lines<P>() * (P / Sched<P>::R0)) void kbf_yline(BatchClass<T> c)
{
    __shared__ cpx<T> lds[yline_lds_elems<P>()];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int q = find_sample(c.prefix, c.nmem, tile);
    const BatchDesc& d = c.d[c.members[q]];
    const YLineArgs a{c.S + d.soff, 3 * d.nz * d.hx, d.Sy, INV ? d.Py : d.ny, INV ? d.ny : d.Py,
                      c.tw + d.twy};
    body_yline<T, P, INV>(a, tile - c.prefix[q], lds);
}

template <typename T, int PZ>
__global__ __launch_bounds__(3 * kspace_z_cols<T>()) void kbf_kspace_z(BatchClass<T> c)
{
    __shared__ cpx<T> sh[kspace_z_lds_elems<T, PZ>()];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int q = find_sample(c.prefix, c.nmem, tile);
    const BatchDesc& d = c.d[c.members[q]];
    const int64_t plane = (int64_t)d.hx * d.Py;
    const KzArgs a{c.S + d.soff, d.nz * plane, (int)plane, d.nz, d.Py, c.tw + d.twz, c.kern + d.koff,
                   d.oct, (int64_t)d.hx * (d.Py / 2 + 1), d.Py / 2 + 1};
    body_kspace_z<T, PZ>(a, tile - c.prefix[q], sh);
}

template <typename T, int P>
__global__ __launch_bounds__(3 * ky_lines<P>() * (P / Sched<P>::R0)) void kbf_kspace_y(BatchClass<T> c)
{
    __shared__ cpx<T> lds[kspace_y_lds_elems<P>()];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int q = find_sample(c.prefix, c.nmem, tile);
    const BatchDesc& d = c.d[c.members[q]];
    const KyArgs a{c.S + d.soff, (int64_t)d.hx * d.ny, d.ny, d.hx, d.ny, c.tw + d.twy, c.kern + d.koff,
                   d.oct, d.Py / 2 + 1};
    body_kspace_y<T, P>(a, tile - c.prefix[q], lds);
}

template <typename T, int P>
__global__ __launch_bounds__(6 * ky2_lines<P>() * (P / Sched<P>::R0)) void kbf_kspace_y2(BatchClass<T> c)
{
    __shared__ cpx<T> lds[kspace_y2_lds_elems<P>()];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int q = find_sample(c.prefix, c.nmem, tile);
    const BatchDesc& d = c.d[c.members[q]];
    const int64_t plane = (int64_t)d.hx * d.ny;
    const Ky2Args a{c.S + d.soff, 2 * plane, plane, d.ny, d.hx, d.ny, c.tw + d.twy, c.kern + d.koff,
                    d.oct, d.Py / 2 + 1};
    body_kspace_y2<T, P>(a, tile - c.prefix[q], lds);
}

template <typename T, int P>
static bool class_launch(int kind, const BatchClass<T>& c, int tiles, int inverse, hipStream_t s)
{
    constexpr int TL = P / Sched<P>::R0;
    switch (kind) {
    case 0:
        if constexpr (P >= 16 && xfwd_lds_elems<P, 8>() * (int)sizeof(cpx<T>) <= 160 * 1024) {
            hipLaunchKernelGGL((kbf_xfwd<T, P, 8>), dim3(tiles), dim3(8 * TL), 0, s, c);
            return true;
        }
        return false;
    case 4:
        if constexpr (P >= 16 && xinv_lds_elems<P, 8>() * (int)sizeof(cpx<T>) <= 160 * 1024) {
            hipLaunchKernelGGL((kbf_xinv<T, P, 8>), dim3(tiles), dim3(8 * TL), 0, s, c);
            return true;
        }
        return false;
    case 1:
        if constexpr (P >= 16) {
            if (inverse)
                hipLaunchKernelGGL((kbf_yline<T, P, true>), dim3(tiles), dim3(yline_lines<P>() * TL), 0, s, c);
            else
                hipLaunchKernelGGL((kbf_yline<T, P, false>), dim3(tiles), dim3(yline_lines<P>() * TL), 0, s, c);
            return true;
        }
        return false;
    case 2:
        if constexpr (P <= 64 && kspace_z_lds_elems<T, P>() * (int)sizeof(cpx<T>) <= 160 * 1024) {
            hipLaunchKernelGGL((kbf_kspace_z<T, P>), dim3(tiles), dim3(3 * kspace_z_cols<T>()), 0, s, c);
            return true;
        }
        return false;
    case 5:
        if constexpr (P >= 16 && P <= 1024 && kspace_y2_lds_elems<P>() * (int)sizeof(cpx<T>) <= kLdsBudget) {
            hipLaunchKernelGGL((kbf_kspace_y2<T, P>), dim3(tiles), dim3(6 * ky2_lines<P>() * TL), 0, s, c);
            return true;
        }
        return false;
    default:
        if constexpr (P >= 16 && P <= 1024) {
            hipLaunchKernelGGL((kbf_kspace_y<T, P>), dim3(tiles), dim3(3 * ky_lines<P>() * TL), 0, s, c);
            return true;
        }
        return false;
    }
}

template <typename T>
bool launch_batch_class(int kind, int P, const BatchClass<T>& c, int tiles, int inverse, hipStream_t s)
{
    if (tiles <= 0) return true;
    switch (P) {
    case 2: return class_launch<T, 2>(kind, c, tiles, inverse, s);
    case 4: return class_launch<T, 4>(kind, c, tiles, inverse, s);
    case 8: return class_launch<T, 8>(kind, c, tiles, inverse, s);
    case 16: return class_launch<T, 16>(kind, c, tiles, inverse, s);
    case 32: return class_launch<T, 32>(kind, c, tiles, inverse, s);
    case 64: return class_launch<T, 64>(kind, c, tiles, inverse, s);
    case 96: return class_launch<T, 96>(kind, c, tiles, inverse, s);
    case 128: return class_launch<T, 128>(kind, c, tiles, inverse, s);
    case 160: return class_launch<T, 160>(kind, c, tiles, inverse, s);
    case 192: return class_launch<T, 192>(kind, c, tiles, inverse, s);
    case 224: return class_launch<T, 224>(kind, c, tiles, inverse, s);
    case 256: return class_launch<T, 256>(kind, c, tiles, inverse, s);
    case 512: return class_launch<T, 512>(kind, c, tiles, inverse, s);
    case 1024: return class_launch<T, 1024>(kind, c, tiles, inverse, s);
    case 2048: return class_launch<T, 2048>(kind, c, tiles, inverse, s);
    default: return false;
    }
}

template bool launch_batch_class<float>(int, int, const BatchClass<float>&, int, int, hipStream_t);
template bool launch_batch_class<double>(int, int, const BatchClass<double>&, int, int, hipStream_t);

template <typename T>
hipError_t launch_batch_pass(int which, const BatchPass<T>& p, int total_tiles, int inverse, hipStream_t s)
{
    if (total_tiles <= 0) return hipSuccess;
    const dim3 grid(total_tiles), block(kBatchNT);
    switch (which) {
    case 0: hipLaunchKernelGGL(kb_xfwd<T>, grid, block, 0, s, p); break;
    case 1: hipLaunchKernelGGL(kb_y<T>, grid, block, 0, s, p, inverse); break;
    case 2: hipLaunchKernelGGL(kb_kspace<T>, grid, block, 0, s, p); break;
    default: hipLaunchKernelGGL(kb_xinv<T>, grid, block, 0, s, p); break;
    }
    return hipGetLastError();
}

template hipError_t launch_batch_pass<float>(int, const BatchPass<float>&, int, int, hipStream_t);
template hipError_t launch_batch_pass<double>(int, const BatchPass<double>&, int, int, hipStream_t);

}  // namespace mm
