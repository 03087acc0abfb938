// mm_adjoint.hip -- vector-Jacobian products of the RK4 step with
// renormalisation, for gradients of a loss of the final state.
//
// Reduced units (h = H/Ms).  One stage computes F(m) = -G [ m x h + a m x (m x h) ]
// with G = gamma Ms dt / (1 + a^2) and h = Lop m + h_ext, where Lop (exchange
// Laplacian with the Neumann rule, diagonal anisotropy, demag convolution) is
// symmetric.  For a covector dF:
//   nu  = -G [ dF x m + a (dF x m) x m ]                 ((dF/dh)^T dF)
//   loc = -G [ h x dF + a ((m x h) x dF + h x (dF x m)) ] ((dF/dm)^T at fixed h)
//   (dF/dm)^T dF = loc + Lop nu
// and the anisotropy map enters h_x = can(c) m_x with can = 2 Ku/(mu0 Ms^2),
// so dLoss/dKu(c) gathers nu_x(c) m_x(c) 2/(mu0 Ms^2) from every stage.
#include "mm_common.hpp"
#include "mm_kernels.hpp"
#include "mm_adjoint_body.hpp"

namespace mm {

// Renormalisation step: m' = m* / |m*| with m* = m_n + (F1 + 2F2 + 2F3 + F4)/6.
// mu = (lam - (lam . m') m') / |m*|;  dF = mu / 6;  accl = mu.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_renorm(AdjArgs<T> a)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= a.N) return;
    const int64_t N = a.N;
    T ms[4][3], hs[4][3];
    ld3(a.mn, N, c, ms[0]);
    ld3(a.m2, N, c, ms[1]);
    ld3(a.m3, N, c, ms[2]);
    ld3(a.m4, N, c, ms[3]);
    ld3(a.h1, N, c, hs[0]);
    ld3(a.h2, N, c, hs[1]);
    ld3(a.h3, N, c, hs[2]);
    ld3(a.h4, N, c, hs[3]);
    T lam[3], mu[3];
    ld3(a.lam, N, c, lam);
    adj_renorm_cell(ms, hs, lam, a.G, a.alpha, mu);
    st3(a.mu, N, c, mu);
    st3(a.accl, N, c, mu);
    const T df[3] = {mu[0] / (T)6, mu[1] / (T)6, mu[2] / (T)6};
    st3(a.dF, N, c, df);
}

// nu and loc of one stage at (m_s, h_s); dku += nu_x m_x * kfac (FP64).
template <typename T>
__global__ __launch_bounds__(256) void k_adj_nu(AdjArgs<T> a, const T* ms, const T* hs)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= a.N) return;
    const int64_t N = a.N;
    T m[3], h[3], l[3];
    ld3(ms, N, c, m);
    ld3(hs, N, c, h);
    ld3(a.dF, N, c, l);
    T nu[3], loc[3];
    adj_nu_cell(m, h, l, a.G, a.alpha, nu, loc);
    st3(a.nu, N, c, nu);
    st3(a.loc, N, c, loc);
    if (a.dku) a.dku[c] += (double)nu[0] * (double)m[0] * a.kfac;
}

// a = loc + Lop nu  (Lop nu = cex Lap nu + can nu_x x + hd_nu);
// accl += a;  dF = cmu mu + ca a.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_apply(AdjArgs<T> a, T cmu, T ca)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= a.N) return;
    const int64_t N = a.N, sy = a.nx, sz = (int64_t)a.nx * a.ny;
    const int i = (int)(c % a.nx);
    const int j = (int)((c / a.nx) % a.ny);
    const int k = (int)(c / sz);
    // a neighbour missing at the boundary is the cell itself (Eq. 7): clamped
    // offsets add uc - uc = 0 and keep every load unconditional; along a
    // periodic axis the neighbour across the boundary is the cell at the other end
    const bool px = a.per & 1, py = a.per & 2, pz = a.per & 4;
    const int64_t dxm = i > 0 ? -1 : (px ? a.nx - 1 : 0), dxp = i < a.nx - 1 ? 1 : (px ? 1 - a.nx : 0);
    const int64_t dym = j > 0 ? -sy : (py ? (a.ny - 1) * sy : 0);
    const int64_t dyp = j < a.ny - 1 ? sy : (py ? (1 - a.ny) * sy : 0);
    const int64_t dzm = k > 0 ? -sz : (pz ? (a.nz - 1) * sz : 0);
    const int64_t dzp = k < a.nz - 1 ? sz : (pz ? (1 - a.nz) * sz : 0);
    T out[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T* u = a.nu + d * N + c;
        const T uc = u[0];
        T acc = (T)0;
        acc += u[dxm] - uc;
        acc += u[dxp] - uc;
        acc += u[dym] - uc;
        acc += u[dyp] - uc;
        acc += u[dzm] - uc;
        acc += u[dzp] - uc;
        T v = a.loc[d * N + c] + a.cex * acc;
        if (a.hd) v += a.hd[d * N + c];
        out[d] = v;
    }
    out[0] += (a.ku ? a.ku[c] : a.can) * a.nu[c];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        a.accl[d * N + c] += out[d];
        a.dF[d * N + c] = cmu * a.mu[d * N + c] + ca * out[d];
    }
}

static int nblk(int64_t n) { return (int)((n + 255) / 256); }

template <typename T>
hipError_t launch_adj_renorm(const AdjArgs<T>& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_renorm<T>, dim3(nblk(a.N)), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_nu(const AdjArgs<T>& a, const T* ms, const T* hs, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_nu<T>, dim3(nblk(a.N)), dim3(256), 0, s, a, ms, hs);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_apply(const AdjArgs<T>& a, T cmu, T ca, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_apply<T>, dim3(nblk(a.N)), dim3(256), 0, s, a, cmu, ca);
    return hipGetLastError();
}

// Vector-Jacobian product of the normalisation u = v / |v| applied when m is set:
// g_v = (g_u - u (u . g_u)) / |v|, per cell.
template <typename T>
__global__ __launch_bounds__(256) void k_normalize_vjp(const T* v, const T* gu, T* gv, int64_t N)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= N) return;
    T x[3], g[3];
    ld3(v, N, c, x);
    ld3(gu, N, c, g);
    const T inv = (T)1 / sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    const T u[3] = {x[0] * inv, x[1] * inv, x[2] * inv};
    const T ug = u[0] * g[0] + u[1] * g[1] + u[2] * g[2];
    const T o[3] = {(g[0] - u[0] * ug) * inv, (g[1] - u[1] * ug) * inv, (g[2] - u[2] * ug) * inv};
    st3(gv, N, c, o);
}

template <typename T>
hipError_t launch_normalize_vjp(const T* v, const T* gu, T* gv, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL(k_normalize_vjp<T>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, v, gu, gv, N);
    return hipGetLastError();
}

// Clears n doubles (a kernel, not a memset node, so that a caller may capture it).
__global__ __launch_bounds__(256) void k_zero_f64(double* p, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

template hipError_t launch_normalize_vjp<float>(const float*, const float*, float*, int64_t, hipStream_t);
template hipError_t launch_normalize_vjp<double>(const double*, const double*, double*, int64_t,
                                                 hipStream_t);
template hipError_t launch_adj_renorm<float>(const AdjArgs<float>&, hipStream_t);
template hipError_t launch_adj_renorm<double>(const AdjArgs<double>&, hipStream_t);
template hipError_t launch_adj_nu<float>(const AdjArgs<float>&, const float*, const float*, hipStream_t);
template hipError_t launch_adj_nu<double>(const AdjArgs<double>&, const double*, const double*,
                                          hipStream_t);
template hipError_t launch_adj_apply<float>(const AdjArgs<float>&, float, float, hipStream_t);
template hipError_t launch_adj_apply<double>(const AdjArgs<double>&, double, double, hipStream_t);

}  // namespace mm
