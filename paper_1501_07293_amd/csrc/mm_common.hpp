// mm_common.hpp -- shared types of the MI355X micromagnetic library.
//
// Conventions used by every kernel:
//   * m, fields: planar [3][nz][ny][nx] arrays, x fastest, in the working
//     precision T (float or double).  m holds unit vectors; internal fields are
//     reduced, h = H / Ms.
//   * spectral buffer S: complex T, [3][planes][rows][sx] where a row is the
//     half spectrum along x (hx = Px/2 + 1 used entries, sx >= hx stride).
//   * kernel spectrum: real T octant [ncomp][Pz/2+1][Py/2+1][hx], the DFT of
//     the demag tensor laid out with wrapped offsets, pre-scaled by 1/(Px Py Pz).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mm {

template <typename T>
struct cpx {
    T re, im;
};

// two adjacent complex values, written by one aligned store
template <typename T>
struct alignas(4 * sizeof(T)) cpx2 {
    cpx<T> a, b;
};

template <typename T>
__host__ __device__ inline cpx<T> mk(T a, T b) { return cpx<T>{a, b}; }
template <typename T>
__device__ inline cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ inline cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ inline cpx<T> cmul(cpx<T> a, cpx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ inline cpx<T> conj(cpx<T> a) { return {a.re, -a.im}; }
template <typename T>
__device__ inline cpx<T> scale(cpx<T> a, T s) { return {a.re * s, a.im * s}; }
// multiply by -i
template <typename T>
__device__ inline cpx<T> mul_mi(cpx<T> a) { return {a.im, -a.re}; }

// Cache hints for data that the next passes do not read: a load of a value read
// for the last time until the caches have turned over, and a store of a value
// that only a later stage reads.  Marked non-temporal, they do not displace what
// the following passes read from the last-level cache.  (The stage update's
// demag field, m_n and accumulator: 1.386 -> 1.347 ms per RK4 step on the
// 512x512x16 film in FP32, the y forward pass after it running 62 -> 57 us.)
template <typename T>
__device__ inline T ld_last(const T* p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ inline void st_later(T v, T* p) { __builtin_nontemporal_store(v, p); }

// Radix schedule of one transform length.  tstride[s] = P / (p_s * R_s) where
// p_s is the product of the radices of the earlier stages.
constexpr int kMaxStages = 12;
struct FftPlan {
    int P;
    int nst;
    int radix[kMaxStages];
    int span[kMaxStages];     // p_s
    int tstride[kMaxStages];  // index step into the length-P twiddle table
};

// Elements each thread keeps in registers per stage (times a radix rounding).
constexpr int kElemsPerThread = 16;

// Work-group to tile remap: the dispatcher places work-group b on XCD b % 8;
// give each XCD a contiguous range of tiles so neighbouring tiles share an L2.
__device__ inline int xcd_tile(int b, int nb)
{
    int xcd = b & 7, local = b >> 3;
    int per = nb >> 3, rem = nb & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
}

}  // namespace mm
