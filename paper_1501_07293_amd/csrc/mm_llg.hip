// mm_llg.hip -- the fused local-field + LLG + RK4-stage kernel, per-term
// field output, FP64 reductions and the normalisation of m.
//
// Local field (reduced units h = H / Ms) of cell c with unit vector m:
//   exchange   Sec. 2.1 Eq. 5 with the Neumann rule of Eqs. 6-7: a missing
//              neighbour equals the cell itself and adds nothing (along a
//              periodic axis the first and last cells are neighbours);
//   anisotropy Sec. 2.2 Eq. 8, easy axis x, x component only;
//   applied    H_ext / Ms;   demag  the FFT result (already reduced).
// LLG right-hand side, Eq. 2 in Landau-Lifshitz form for unit m:
//   dm/dt = -gamma Ms / (1 + alpha^2) [ m x h + alpha m x (m x h) ].
// Classical RK4 with F_s = dt f(m_s):
//   stage 1: acc = F1,      out = m_n + F1/2
//   stage 2: acc += 2 F2,   out = m_n + F2/2
//   stage 3: acc += 2 F3,   out = m_n + F3
//   stage 4: m_n <- normalise(m_n + (acc + F4) / 6)   (the per-step renormalisation)
#include "mm_common.hpp"
#include "mm_kernels.hpp"
#include "mm_llg_body.hpp"

namespace mm {

template <typename T>
struct Cell {
    T m[3];
    T hex[3];
};

template <typename T>
__device__ inline void exchange_at(const LlgArgs<T>& a, int64_t c, int i, int j, int k, Cell<T>& o)
{
    const int64_t N = a.N, sy = a.nx, sz = (int64_t)a.nx * a.ny;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T* u = a.ms + d * N;
        const T mc = u[c];
        T acc = (T)0;
        if (i > 0) acc += u[c - 1] - mc;
        else if (a.per & 1) acc += u[c + (a.nx - 1)] - mc;
        if (i < a.nx - 1) acc += u[c + 1] - mc;
        else if (a.per & 1) acc += u[c - (a.nx - 1)] - mc;
        if (j > 0) acc += u[c - sy] - mc;
        else if (a.per & 2) acc += u[c + (a.ny - 1) * sy] - mc;
        if (j < a.ny - 1) acc += u[c + sy] - mc;
        else if (a.per & 2) acc += u[c - (a.ny - 1) * sy] - mc;
        if (k > 0) acc += u[c - sz] - mc;
        else if (a.per & 4) acc += u[c + (a.nz - 1) * sz] - mc;
        if (k < a.nz - 1) acc += u[c + sz] - mc;
        else if (a.per & 4) acc += u[c - (a.nz - 1) * sz] - mc;
        o.m[d] = mc;
        o.hex[d] = a.cex * acc;
    }
}

template <typename T>
__device__ inline void heff_at(const LlgArgs<T>& a, int64_t c, const Cell<T>& o, T h[3])
{
    const T kan = a.ku ? a.ku[c] : a.can;
    h[0] = o.hex[0] + kan * o.m[0] + a.hx;
    h[1] = o.hex[1] + a.hy;
    h[2] = o.hex[2] + a.hz;
    if (a.hd) {
        h[0] += a.hd[c];
        h[1] += a.hd[a.N + c];
        h[2] += a.hd[2 * a.N + c];
    }
}

// Row-major columns (TY = 1) are XCD-aware: consecutive tiles (neighbouring rows
// of a plane) run on the same XCD, so the y-neighbour rows one work-group reads
// are in that XCD's L2.  Two-row tiles, which hold half their y neighbours
// themselves, run in dispatch order (tile b on XCD b % 8, the whole chip sweeping
// the grid front to back): the update itself takes about 1 us longer, the RK4
// step on the 512x512x16 film 0.5% less (FP32 1.3155 -> 1.3091 ms, FP64 2.909 ->
// 2.897 ms, twice each in one run).
template <typename T, int KZ, int TY>
__global__ __launch_bounds__(kLlgNT) void k_llg_stage(LlgArgs<T> a)
{
    body_llg_stage<T, KZ, TY>(a, TY > 1 ? (int)blockIdx.x : xcd_tile(blockIdx.x, gridDim.x), threadIdx.x);
}

template <typename T>
__global__ __launch_bounds__(256) void k_field_term(LlgArgs<T> a, int term, T Ms, T* out)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= a.N) return;
    const int i = (int)(c % a.nx);
    const int j = (int)((c / a.nx) % a.ny);
    const int k = (int)(c / ((int64_t)a.nx * a.ny));
    Cell<T> o;
    exchange_at(a, c, i, j, k, o);
    T h[3];
    switch (term) {
    case 0:
        h[0] = o.hex[0];
        h[1] = o.hex[1];
        h[2] = o.hex[2];
        break;
    case 1:
        h[0] = (a.ku ? a.ku[c] : a.can) * o.m[0];
        h[1] = (T)0;
        h[2] = (T)0;
        break;
    case 2:
        h[0] = a.hd ? a.hd[c] : (T)0;
        h[1] = a.hd ? a.hd[a.N + c] : (T)0;
        h[2] = a.hd ? a.hd[2 * a.N + c] : (T)0;
        break;
    case 3:
        h[0] = a.hx;
        h[1] = a.hy;
        h[2] = a.hz;
        break;
    default:
        heff_at(a, c, o, h);
        break;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) out[d * a.N + c] = Ms * h[d];
}

constexpr int kRedThreads = 256;

// One thread block's partial sums over its cells (grid-stride loop), FP64 from
// working-precision inputs: slots 0-3 the energy sums of Eq. 1 (exchange pairs,
// anisotropy, demag, applied), 4-6 the sum of m, 7 the count of non-finite
// cells, and slot 8 the largest torque |m x h| over the cells, h the reduced
// effective field of Eq. 3 (a maximum, not a sum).
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_reduce_partial(LlgArgs<T> a, double* partial)
{
    __shared__ double sh[kRedSlots][kRedThreads];
    double acc[kRedSlots] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t N = a.N, sy = a.nx, sz = (int64_t)a.nx * a.ny;
    const double cex = (double)a.cex;
    for (int64_t c = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; c < N;
         c += (int64_t)gridDim.x * kRedThreads) {
        const int i = (int)(c % a.nx);
        const int j = (int)((c / a.nx) % a.ny);
        const int k = (int)(c / ((int64_t)a.nx * a.ny));
        double m[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) m[d] = (double)a.ms[d * N + c];
        // exchange: each neighbour pair once (towards +x, +y, +z; across the
        // boundary of a periodic axis towards its first cell)
        const int64_t nb[3] = {i < a.nx - 1 ? c + 1 : ((a.per & 1) ? c - (a.nx - 1) : -1),
                               j < a.ny - 1 ? c + sy : ((a.per & 2) ? c - (int64_t)(a.ny - 1) * sy : -1),
                               k < a.nz - 1 ? c + sz : ((a.per & 4) ? c - (int64_t)(a.nz - 1) * sz : -1)};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (nb[q] < 0) continue;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double df = (double)a.ms[d * N + nb[q]] - m[d];
                acc[0] += df * df;
            }
        }
        const double kan = a.ku ? (double)a.ku[c] : (double)a.can;
        acc[1] += kan * (m[1] * m[1] + m[2] * m[2]);
        double hd[3] = {0.0, 0.0, 0.0};
        if (a.hd) {
#pragma unroll
            for (int d = 0; d < 3; ++d) hd[d] = (double)a.hd[d * N + c];
        }
        acc[2] += m[0] * hd[0] + m[1] * hd[1] + m[2] * hd[2];
        acc[3] += m[0] * (double)a.hx + m[1] * (double)a.hy + m[2] * (double)a.hz;
        acc[4] += m[0];
        acc[5] += m[1];
        acc[6] += m[2];
        if (!isfinite(m[0]) || !isfinite(m[1]) || !isfinite(m[2])) acc[7] += 1.0;
        // the six neighbours of Eq. 5; a missing one (Eq. 7) is the cell itself
        const int64_t six[6] = {i > 0 ? c - 1 : ((a.per & 1) ? c + (a.nx - 1) : c),
                                i < a.nx - 1 ? c + 1 : ((a.per & 1) ? c - (a.nx - 1) : c),
                                j > 0 ? c - sy : ((a.per & 2) ? c + (int64_t)(a.ny - 1) * sy : c),
                                j < a.ny - 1 ? c + sy : ((a.per & 2) ? c - (int64_t)(a.ny - 1) * sy : c),
                                k > 0 ? c - sz : ((a.per & 4) ? c + (int64_t)(a.nz - 1) * sz : c),
                                k < a.nz - 1 ? c + sz : ((a.per & 4) ? c - (int64_t)(a.nz - 1) * sz : c)};
        double h[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double lap = 0.0;
#pragma unroll
            for (int q = 0; q < 6; ++q) lap += (double)a.ms[d * N + six[q]] - m[d];
            h[d] = cex * lap + hd[d];
        }
        h[0] += kan * m[0] + (double)a.hx;
        h[1] += (double)a.hy;
        h[2] += (double)a.hz;
        const double tx = m[1] * h[2] - m[2] * h[1];
        const double ty = m[2] * h[0] - m[0] * h[2];
        const double tz = m[0] * h[1] - m[1] * h[0];
        acc[8] = fmax(acc[8], sqrt(tx * tx + ty * ty + tz * tz));
    }
#pragma unroll
    for (int q = 0; q < kRedSlots; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int q = 0; q < kRedSlots - 1; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
            sh[kRedSlots - 1][threadIdx.x] = fmax(sh[kRedSlots - 1][threadIdx.x],
                                                  sh[kRedSlots - 1][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < kRedSlots) partial[blockIdx.x * kRedSlots + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_final(const double* partial, int nb,
                                                              double* out)
{
    __shared__ double sh[kRedSlots][kRedThreads];
    double acc[kRedSlots] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += kRedThreads) {
#pragma unroll
        for (int q = 0; q < kRedSlots - 1; ++q) acc[q] += partial[b * kRedSlots + q];
        acc[kRedSlots - 1] = fmax(acc[kRedSlots - 1], partial[b * kRedSlots + kRedSlots - 1]);
    }
#pragma unroll
    for (int q = 0; q < kRedSlots; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int q = 0; q < kRedSlots - 1; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
            sh[kRedSlots - 1][threadIdx.x] = fmax(sh[kRedSlots - 1][threadIdx.x],
                                                  sh[kRedSlots - 1][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < kRedSlots) out[threadIdx.x] = sh[threadIdx.x][0];
}

template <typename T>
__global__ void k_normalize(T* m, int64_t N, unsigned int* bad)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= N) return;
    const T x = m[c], y = m[N + c], z = m[2 * N + c];
    const T n2 = x * x + y * y + z * z;
    if (!(n2 > (T)0) || !isfinite(n2)) {
        atomicAdd(bad, 1u);
        return;
    }
    const T inv = (T)1 / sqrt(n2);
    m[c] = x * inv;
    m[N + c] = y * inv;
    m[2 * N + c] = z * inv;
}

static int blocks_for(int64_t n) { return (int)((n + 255) / 256); }

// Rows per LLG work-group tile where the plane divides into tiles of kLlgNT / 2
// columns by 2 rows: on the 512x512x16 film FP32 the stage update measured
// 57.0 -> 55.9 us a launch (1.320 -> 1.316 ms per RK4 step); 4 rows of 64
// columns gained less (1.319), 8 rows of 32 lost (1.334).
constexpr int kLlgTileRows = 2;

template <typename T>
hipError_t launch_llg_stage(const LlgArgs<T>& a, hipStream_t s)
{
    const dim3 grid((int)llg_blocks(a.nx, a.ny, a.nz));
    constexpr int TY = kLlgTileRows;
    const bool tile = a.nx % (kLlgNT / TY) == 0 && a.ny % TY == 0;
    switch (llg_z_for(a.nz) * 2 + (tile ? 1 : 0)) {
    case 2: hipLaunchKernelGGL((k_llg_stage<T, 1, 1>), grid, dim3(kLlgNT), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_llg_stage<T, 1, TY>), grid, dim3(kLlgNT), 0, s, a); break;
    case 2 * kLlgZ + 1: hipLaunchKernelGGL((k_llg_stage<T, kLlgZ, TY>), grid, dim3(kLlgNT), 0, s, a); break;
    default: hipLaunchKernelGGL((k_llg_stage<T, kLlgZ, 1>), grid, dim3(kLlgNT), 0, s, a); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_field_term(const LlgArgs<T>& a, int term, T Ms, T* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_field_term<T>, dim3(blocks_for(a.N)), dim3(256), 0, s, a, term, Ms, out);
    return hipGetLastError();
}

int reduce_blocks(int64_t N)
{
    int64_t b = (N + kRedThreads - 1) / kRedThreads;
    if (b > 1024) b = 1024;
    return (int)(b < 1 ? 1 : b);
}

__global__ void k_trace_row(const double* sums, double inv_n, double t, double* row)
{
    if (threadIdx.x == 0) row[0] = t;
    else if (threadIdx.x < 4) row[threadIdx.x] = sums[3 + threadIdx.x] * inv_n;
}

hipError_t launch_trace_row(const double* sums, double inv_n, double t, double* row, hipStream_t s)
{
    hipLaunchKernelGGL(k_trace_row, dim3(1), dim3(64), 0, s, sums, inv_n, t, row);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce(const LlgArgs<T>& a, double* partial, int nblocks, double* out,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_partial<T>, dim3(nblocks), dim3(kRedThreads), 0, s, a, partial);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedThreads), 0, s, partial, nblocks, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_normalize(T* m, int64_t N, unsigned int* bad, hipStream_t s)
{
    hipLaunchKernelGGL(k_normalize<T>, dim3(blocks_for(N)), dim3(256), 0, s, m, N, bad);
    return hipGetLastError();
}

template hipError_t launch_llg_stage<float>(const LlgArgs<float>&, hipStream_t);
template hipError_t launch_llg_stage<double>(const LlgArgs<double>&, hipStream_t);
template hipError_t launch_field_term<float>(const LlgArgs<float>&, int, float, float*, hipStream_t);
template hipError_t launch_field_term<double>(const LlgArgs<double>&, int, double, double*,
                                              hipStream_t);
template hipError_t launch_reduce<float>(const LlgArgs<float>&, double*, int, double*, hipStream_t);
template hipError_t launch_reduce<double>(const LlgArgs<double>&, double*, int, double*,
                                          hipStream_t);
template hipError_t launch_normalize<float>(float*, int64_t, unsigned int*, hipStream_t);
template hipError_t launch_normalize<double>(double*, int64_t, unsigned int*, hipStream_t);

}  // namespace mm
