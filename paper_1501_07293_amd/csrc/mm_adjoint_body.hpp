// mm_adjoint_body.hpp -- per-cell pieces of the RK4 step's vector-Jacobian
// products, shared by the adjoint kernels (mm_adjoint.hip, where the equations
// are written out) and the fused adjoint stage pass (mm_fused.hpp).
#pragma once
#include "mm_common.hpp"

namespace mm {

template <typename T>
__device__ inline void xprod(const T a[3], const T b[3], T o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

template <typename T>
__device__ inline void ld3(const T* p, int64_t N, int64_t c, T v[3])
{
    v[0] = p[c];
    v[1] = p[N + c];
    v[2] = p[2 * N + c];
}

template <typename T>
__device__ inline void st3(T* p, int64_t N, int64_t c, const T v[3])
{
    p[c] = v[0];
    p[N + c] = v[1];
    p[2 * N + c] = v[2];
}

// F(m, h) for one cell
template <typename T>
__device__ inline void stage_F(const T m[3], const T h[3], T G, T alpha, T F[3])
{
    T t[3], d[3];
    xprod(m, h, t);
    xprod(m, t, d);
#pragma unroll
    for (int q = 0; q < 3; ++q) F[q] = -G * (t[q] + alpha * d[q]);
}

// Renormalisation: m' = m* / |m*|, m* = m_n + (F1 + 2F2 + 2F3 + F4)/6 from the
// step's stage states ms and fields hs; mu = (lam - (lam . m') m') / |m*|.
template <typename T>
__device__ inline void adj_renorm_cell(const T ms[4][3], const T hs[4][3], const T lam[3], T G, T alpha, T mu[3])
{
    T F[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s) stage_F(ms[s], hs[s], G, alpha, F[s]);
    T mstar[3];
#pragma unroll
    for (int q = 0; q < 3; ++q)
        mstar[q] = ms[0][q] + (F[0][q] + (T)2 * F[1][q] + (T)2 * F[2][q] + F[3][q]) / (T)6;
    const T nrm = sqrt(mstar[0] * mstar[0] + mstar[1] * mstar[1] + mstar[2] * mstar[2]);
    const T mp[3] = {mstar[0] / nrm, mstar[1] / nrm, mstar[2] / nrm};
    const T dot = lam[0] * mp[0] + lam[1] * mp[1] + lam[2] * mp[2];
#pragma unroll
    for (int q = 0; q < 3; ++q) mu[q] = (lam[q] - dot * mp[q]) / nrm;
}

// nu = (dF/dh)^T l and loc = (dF/dm)^T l at fixed h, for one stage at (m, h)
template <typename T>
__device__ inline void adj_nu_cell(const T m[3], const T h[3], const T l[3], T G, T alpha, T nu[3], T loc[3])
{
    T lxm[3], t4[3], t1[3], mxh[3], t2[3], t3[3];
    xprod(l, m, lxm);    // dF x m
    xprod(lxm, m, t4);   // (dF x m) x m
    xprod(h, l, t1);     // h x dF
    xprod(m, h, mxh);    // m x h
    xprod(mxh, l, t2);   // (m x h) x dF
    xprod(h, lxm, t3);   // h x (dF x m)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        nu[q] = -G * (lxm[q] + alpha * t4[q]);
        loc[q] = -G * (t1[q] + alpha * (t2[q] + t3[q]));
    }
}

}  // namespace mm
