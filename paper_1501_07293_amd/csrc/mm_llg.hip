// mm_llg.hip -- the fused local-field + LLG + RK4-stage kernel, per-term
// field output, FP64 reductions and the normalisation of m.
//
// Local field (reduced units h = H / Ms) of cell c with unit vector m:
//   exchange   Sec. 2.1 Eq. 5 with the Neumann rule of Eqs. 6-7: a missing
//              neighbour equals the cell itself and adds nothing;
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
        if (i < a.nx - 1) acc += u[c + 1] - mc;
        if (j > 0) acc += u[c - sy] - mc;
        if (j < a.ny - 1) acc += u[c + sy] - mc;
        if (k > 0) acc += u[c - sz] - mc;
        if (k < a.nz - 1) acc += u[c + sz] - mc;
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

// One thread per (x, y) column and chunk of kLlgZ planes.  Every load of the
// chunk (m of planes k0-1 .. k0+kLlgZ, in-plane neighbours, H_d, Ku, m_n, acc)
// is issued before the first store, so a thread keeps many loads in flight;
// the z neighbours come from registers, the x and y neighbours from rows that
// neighbouring threads load anyway (L1/L2 hits).
constexpr int kLlgZ = 4;

template <typename T>
__global__ __launch_bounds__(256) void k_llg_stage(LlgArgs<T> a)
{
    constexpr int KZ = kLlgZ;
    const int64_t plane = (int64_t)a.nx * a.ny;
    const int nzc = (a.nz + KZ - 1) / KZ;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= plane * nzc) return;
    const int kc = (int)(t / plane);
    const int64_t pc = t - (int64_t)kc * plane;
    const int i = (int)(pc % a.nx), j = (int)(pc / a.nx);
    const int k0 = kc * KZ;
    const int64_t N = a.N, sy = a.nx;
    const T* __restrict__ ms = a.ms;
    T col[KZ + 2][3];
#pragma unroll
    for (int q = 0; q < KZ + 2; ++q) {
        const int k = k0 - 1 + q;
        const bool in = k >= 0 && k < a.nz;
#pragma unroll
        for (int d = 0; d < 3; ++d) col[q][d] = in ? ms[d * N + pc + k * plane] : (T)0;
    }
    T lap[KZ][3], hd[KZ][3], mn[KZ][3], ac[KZ][3], kan[KZ];
#pragma unroll
    for (int q = 0; q < KZ; ++q) {
        const int k = k0 + q;
        const bool in = k < a.nz;
        const int64_t c = pc + (int64_t)(in ? k : 0) * plane;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T* u = ms + d * N;
            const T mc = col[q + 1][d];
            T acc = (T)0;
            if (in) {
                if (i > 0) acc += u[c - 1] - mc;
                if (i < a.nx - 1) acc += u[c + 1] - mc;
                if (j > 0) acc += u[c - sy] - mc;
                if (j < a.ny - 1) acc += u[c + sy] - mc;
                if (k > 0) acc += col[q][d] - mc;
                if (k < a.nz - 1) acc += col[q + 2][d] - mc;
            }
            lap[q][d] = acc;
            hd[q][d] = (in && a.hd) ? a.hd[d * N + c] : (T)0;
            mn[q][d] = (in && a.stage > 1) ? a.mn[d * N + c] : (T)0;
            ac[q][d] = (in && a.stage > 1) ? a.acc[d * N + c] : (T)0;
        }
        kan[q] = (in && a.ku) ? a.ku[c] : a.can;
    }
#pragma unroll
    for (int q = 0; q < KZ; ++q) {
        const int k = k0 + q;
        if (k >= a.nz) break;
        const int64_t c = pc + (int64_t)k * plane;
        const T* m = col[q + 1];
        const T h[3] = {a.cex * lap[q][0] + kan[q] * m[0] + a.hx + hd[q][0],
                        a.cex * lap[q][1] + a.hy + hd[q][1], a.cex * lap[q][2] + a.hz + hd[q][2]};
        const T tx = m[1] * h[2] - m[2] * h[1];
        const T ty = m[2] * h[0] - m[0] * h[2];
        const T tz = m[0] * h[1] - m[1] * h[0];
        const T dx = m[1] * tz - m[2] * ty;
        const T dy = m[2] * tx - m[0] * tz;
        const T dz = m[0] * ty - m[1] * tx;
        const T F[3] = {-a.gdt * (tx + a.alpha * dx), -a.gdt * (ty + a.alpha * dy),
                        -a.gdt * (tz + a.alpha * dz)};
        if (a.stage == 1) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                a.acc[d * N + c] = F[d];
                a.out[d * N + c] = m[d] + (T)0.5 * F[d];
            }
        } else if (a.stage == 2 || a.stage == 3) {
            const T w = a.stage == 2 ? (T)0.5 : (T)1;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                a.acc[d * N + c] = ac[q][d] + (T)2 * F[d];
                a.out[d * N + c] = mn[q][d] + w * F[d];
            }
        } else {
            T v[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) v[d] = mn[q][d] + (ac[q][d] + F[d]) / (T)6;
            const T inv = (T)1 / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
#pragma unroll
            for (int d = 0; d < 3; ++d) a.out[d * N + c] = v[d] * inv;
        }
    }
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

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_reduce_partial(LlgArgs<T> a, double* partial)
{
    __shared__ double sh[8][kRedThreads];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t N = a.N, sy = a.nx, sz = (int64_t)a.nx * a.ny;
    for (int64_t c = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; c < N;
         c += (int64_t)gridDim.x * kRedThreads) {
        const int i = (int)(c % a.nx);
        const int j = (int)((c / a.nx) % a.ny);
        const int k = (int)(c / ((int64_t)a.nx * a.ny));
        double m[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) m[d] = (double)a.ms[d * N + c];
        // exchange: each neighbour pair once (towards +x, +y, +z)
        const int64_t nb[3] = {i < a.nx - 1 ? c + 1 : -1, j < a.ny - 1 ? c + sy : -1,
                               k < a.nz - 1 ? c + sz : -1};
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
        if (a.hd)
            acc[2] += m[0] * (double)a.hd[c] + m[1] * (double)a.hd[N + c] + m[2] * (double)a.hd[2 * N + c];
        acc[3] += m[0] * (double)a.hx + m[1] * (double)a.hy + m[2] * (double)a.hz;
        acc[4] += m[0];
        acc[5] += m[1];
        acc[6] += m[2];
        if (!isfinite(m[0]) || !isfinite(m[1]) || !isfinite(m[2])) acc[7] += 1.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int q = 0; q < 8; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 8) partial[blockIdx.x * 8 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_final(const double* partial, int nb,
                                                              double* out)
{
    __shared__ double sh[8][kRedThreads];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += kRedThreads)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] += partial[b * 8 + q];
#pragma unroll
    for (int q = 0; q < 8; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int q = 0; q < 8; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 8) out[threadIdx.x] = sh[threadIdx.x][0];
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

template <typename T>
hipError_t launch_llg_stage(const LlgArgs<T>& a, hipStream_t s)
{
    const int64_t threads = (int64_t)a.nx * a.ny * ((a.nz + kLlgZ - 1) / kLlgZ);
    hipLaunchKernelGGL(k_llg_stage<T>, dim3(blocks_for(threads)), dim3(256), 0, s, a);
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
