// mm_generic.hpp -- device bodies of the runtime-radix FFT passes (any
// 7-smooth length), shared by the single-grid kernels (mm_passes.hip) and the
// batched kernels (mm_batch.hip).  Each body works one tile of its pass; the
// caller supplies the tile index, the LDS buffer (lds_elems(NT) entries) and
// the radix schedule (by reference, so a schedule held in memory is indexed in
// place rather than copied into registers).
#pragma once
#include "mm_fft.hpp"
#include "mm_kernels.hpp"

namespace mm {


constexpr int lds_elems(int nt) { return kElemsPerThread * nt + 64; }

__device__ inline int64_t row_off(int r, int rpp, int64_t plane_stride, int64_t rstride)
{
    const int pl = r / rpp;
    return (int64_t)pl * plane_stride + (int64_t)(r - pl * rpp) * rstride;
}

__device__ inline int64_t col_off(int c, int cpr, int64_t row2)
{
    const int r = c / cpr;
    return (int64_t)r * row2 + (c - r * cpr);
}

// ------------------------------------------------------------------ x forward
template <typename T, int NT>
__device__ void body_row_r2c(const RowR2CArgs& a, const FftPlan& pl, int tile, cpx<T>* lds)
{
    const int P = pl.P, LS = P + 1, B = a.lines_per_wg;
    const int npairs = (a.nrows + 1) >> 1;
    const int q0 = tile * B;
    const T* in = (const T*)a.in;
    for (int idx = threadIdx.x; idx < B * P; idx += NT) {
        const int q = idx / P, x = idx - q * P, pr = q0 + q;
        cpx<T> v = {(T)0, (T)0};
        if (pr < npairs && x < a.nvalid) {
            const int r0 = 2 * pr;
            v.re = in[(int64_t)r0 * a.in_row_stride + x];
            if (r0 + 1 < a.nrows) v.im = in[(int64_t)(r0 + 1) * a.in_row_stride + x];
        }
        lds[q * LS + x] = v;
    }
    __syncthreads();
    lds_fft<T, NT, false>(lds, LdsGeom{B, B, LS, 0, 1}, pl, (const cpx<T>*)a.tw, threadIdx.x);
    cpx<T>* out = (cpx<T>*)a.out;
    for (int idx = threadIdx.x; idx < B * a.hx; idx += NT) {
        const int q = idx / a.hx, k = idx - q * a.hx, pr = q0 + q;
        if (pr >= npairs) continue;
        const cpx<T> zk = lds[q * LS + k], zm = lds[q * LS + (k == 0 ? 0 : P - k)];
        // split Z = FFT(a + i b): A = (Z_k + conj Z_-k)/2, B = (Z_k - conj Z_-k)/(2i)
        const cpx<T> A = scale(zk + conj(zm), (T)0.5);
        const cpx<T> Bv = scale(mul_mi(zk - conj(zm)), (T)0.5);
        const int r0 = 2 * pr;
        const int64_t ko = (int64_t)k * a.kstride;
        out[row_off(r0, a.rows_per_plane, a.out_plane_stride, a.rstride) + ko] = A;
        if (r0 + 1 < a.nrows)
            out[row_off(r0 + 1, a.rows_per_plane, a.out_plane_stride, a.rstride) + ko] = Bv;
    }
}


// ------------------------------------------------------------------ x inverse
template <typename T, int NT>
__device__ void body_row_c2r(const RowC2RArgs& a, const FftPlan& pl, int tile, cpx<T>* lds)
{
    const int P = pl.P, LS = P + 1, B = a.lines_per_wg;
    const int npairs = (a.nrows + 1) >> 1;
    const int q0 = tile * B;
    const bool evenP = (P & 1) == 0;
    const cpx<T>* in = (const cpx<T>*)a.in;
    for (int idx = threadIdx.x; idx < B * P; idx += NT) {
        const int q = idx / P, x = idx - q * P, pr = q0 + q;
        cpx<T> z = {(T)0, (T)0};
        if (pr < npairs) {
            const int r0 = 2 * pr;
            const bool has1 = r0 + 1 < a.nrows;
            const int64_t o0 = row_off(r0, a.rows_per_plane, a.in_plane_stride, a.rstride);
            const int64_t o1 = has1 ? row_off(r0 + 1, a.rows_per_plane, a.in_plane_stride, a.rstride) : 0;
            const int64_t ks = a.kstride;
            cpx<T> A, Bv = {(T)0, (T)0};
            if (x < a.hx) {
                A = in[o0 + x * ks];
                if (has1) Bv = in[o1 + x * ks];
                if (x == 0 || (evenP && 2 * x == P)) {  // DC and Nyquist bins are real
                    A.im = (T)0;
                    Bv.im = (T)0;
                }
            } else {
                A = conj(in[o0 + (P - x) * ks]);
                if (has1) Bv = conj(in[o1 + (P - x) * ks]);
            }
            z = {A.re - Bv.im, A.im + Bv.re};  // A + i B
        }
        lds[q * LS + x] = conj(z);
    }
    __syncthreads();
    lds_fft<T, NT, false>(lds, LdsGeom{B, B, LS, 0, 1}, pl, (const cpx<T>*)a.tw, threadIdx.x);
    T* out = (T*)a.out;
    for (int idx = threadIdx.x; idx < B * a.nvalid; idx += NT) {
        const int q = idx / a.nvalid, x = idx - q * a.nvalid, pr = q0 + q;
        if (pr >= npairs) continue;
        const cpx<T> z = lds[q * LS + x];  // result is conj(z) = a + i b
        const int r0 = 2 * pr;
        out[(int64_t)r0 * a.out_row_stride + x] = z.re;
        if (r0 + 1 < a.nrows) out[(int64_t)(r0 + 1) * a.out_row_stride + x] = -z.im;
    }
}


// ------------------------------------------------------------ strided columns
template <typename T, int NT>
__device__ void body_col_fft(const ColArgs& a, const FftPlan& pl, int tile, cpx<T>* lds)
{
    const int P = pl.P, TW = a.tw_cols;
    const int ctiles = (a.ncols + TW - 1) / TW;
    const int plane = tile / ctiles, c0 = (tile - plane * ctiles) * TW;
    cpx<T>* buf = (cpx<T>*)a.buf + (int64_t)plane * a.plane_stride;
    for (int idx = threadIdx.x; idx < P * TW; idx += NT) {
        const int e = idx / TW, t = idx - e * TW, col = c0 + t;
        cpx<T> v = {(T)0, (T)0};
        if (e < a.nin && col < a.ncols) {
            v = buf[e * a.es + col_off(col, a.cols_per_row, a.row2_stride)];
            if (a.inverse) v = conj(v);
        }
        lds[idx] = v;
    }
    __syncthreads();
    lds_fft<T, NT, true>(lds, LdsGeom{TW, TW, 1, 0, TW}, pl, (const cpx<T>*)a.tw, threadIdx.x);
    for (int idx = threadIdx.x; idx < a.nout * TW; idx += NT) {
        const int e = idx / TW, t = idx - e * TW, col = c0 + t;
        if (col >= a.ncols) continue;
        cpx<T> v = lds[idx];
        if (a.inverse) v = conj(v);
        buf[e * a.es + col_off(col, a.cols_per_row, a.row2_stride)] = v;
    }
}


// Contiguous lines (line l at buf + l * line_stride), i-fast thread mapping:
// B = lines_per_wg lines per work-group, inputs beyond nin zero, first nout
// outputs stored, inverse by conjugation.
template <typename T, int NT>
__device__ void body_line_c2c(const LineArgs& a, const FftPlan& pl, int tile, cpx<T>* lds)
{
    const int P = pl.P, LS = P + 1, B = a.lines_per_wg;
    const int l0 = tile * B;
    cpx<T>* buf = (cpx<T>*)a.buf;
    for (int idx = threadIdx.x; idx < B * P; idx += NT) {
        const int q = idx / P, e = idx - q * P, l = l0 + q;
        cpx<T> v = {(T)0, (T)0};
        if (l < a.nlines && e < a.nin) {
            v = buf[(int64_t)l * a.line_stride + e];
            if (a.inverse) v = conj(v);
        }
        lds[q * LS + e] = v;
    }
    __syncthreads();
    lds_fft<T, NT, false>(lds, LdsGeom{B, B, LS, 0, 1}, pl, (const cpx<T>*)a.tw, threadIdx.x);
    for (int idx = threadIdx.x; idx < B * a.nout; idx += NT) {
        const int q = idx / a.nout, e = idx - q * a.nout, l = l0 + q;
        if (l >= a.nlines) continue;
        cpx<T> v = lds[q * LS + e];
        if (a.inverse) v = conj(v);
        buf[(int64_t)l * a.line_stride + e] = v;
    }
}

// ------------------------------------------------------------------ k-space
template <typename T, int NT>
__device__ void body_kspace(const KspArgs& a, const FftPlan& pl, int tile, cpx<T>* lds)
{
    const int P = pl.P, TW = a.tw_cols;
    const int c0 = tile * TW;
    cpx<T>* buf = (cpx<T>*)a.buf;
    const int PT = P * TW;
    for (int idx = threadIdx.x; idx < 3 * PT; idx += NT) {
        const int c = idx / PT, rem = idx - c * PT, e = rem / TW, t = rem - e * TW, col = c0 + t;
        cpx<T> v = {(T)0, (T)0};
        if (e < a.nvalid && col < a.ncols)
            v = buf[c * a.comp_stride + e * a.es + col_off(col, a.cols_per_row, a.row2_stride)];
        lds[idx] = v;
    }
    __syncthreads();
    const LdsGeom g{3 * TW, TW, 1, PT, TW};
    lds_fft<T, NT, true>(lds, g, pl, (const cpx<T>*)a.tw, threadIdx.x);
    // Eq. 14: H~_a = sum_b K~_ab M~_b with the real, symmetric kernel spectrum.
    const T* K = (const T*)a.kern;
    for (int idx = threadIdx.x; idx < PT; idx += NT) {
        const int e = idx / TW, t = idx - e * TW, col = c0 + t;
        if (col >= a.ncols) continue;
        int kx, ky, kz;
        if (a.axis_is_z) {
            kx = col / a.Py;
            ky = col - kx * a.Py;
            kz = e;
        } else {
            kx = col;
            ky = e;
            kz = 0;
        }
        T sy = (T)1, sz = (T)1;
        if (2 * ky > a.Py) {
            ky = a.Py - ky;
            sy = (T)-1;
        }
        if (2 * kz > a.Pz) {
            kz = a.Pz - kz;
            sz = (T)-1;
        }
        const int64_t ko = kz * a.k_zs + kx * a.k_xs + ky;
        T kxx, kxy, kxz, kyy, kyz, kzz;
        if (a.ncomp == 6) {
            kxx = K[ko];
            kxy = sy * K[a.k_cs + ko];
            kxz = sz * K[2 * a.k_cs + ko];
            kyy = K[3 * a.k_cs + ko];
            kyz = sy * sz * K[4 * a.k_cs + ko];
            kzz = K[5 * a.k_cs + ko];
        } else {
            kxx = K[ko];
            kxy = sy * K[a.k_cs + ko];
            kxz = (T)0;
            kyy = K[2 * a.k_cs + ko];
            kyz = (T)0;
            kzz = K[3 * a.k_cs + ko];
        }
        const cpx<T> mx = lds[idx], my = lds[PT + idx], mz = lds[2 * PT + idx];
        const cpx<T> hx = {kxx * mx.re + kxy * my.re + kxz * mz.re, kxx * mx.im + kxy * my.im + kxz * mz.im};
        const cpx<T> hy = {kxy * mx.re + kyy * my.re + kyz * mz.re, kxy * mx.im + kyy * my.im + kyz * mz.im};
        const cpx<T> hz = {kxz * mx.re + kyz * my.re + kzz * mz.re, kxz * mx.im + kyz * my.im + kzz * mz.im};
        lds[idx] = conj(hx);  // inverse transform by conjugation
        lds[PT + idx] = conj(hy);
        lds[2 * PT + idx] = conj(hz);
    }
    __syncthreads();
    lds_fft<T, NT, true>(lds, g, pl, (const cpx<T>*)a.tw, threadIdx.x);
    const int VT = a.nvalid * TW;
    for (int idx = threadIdx.x; idx < 3 * VT; idx += NT) {
        const int c = idx / VT, rem = idx - c * VT, e = rem / TW, t = rem - e * TW, col = c0 + t;
        if (col >= a.ncols) continue;
        buf[c * a.comp_stride + e * a.es + col_off(col, a.cols_per_row, a.row2_stride)] =
            conj(lds[c * PT + e * TW + t]);
    }
}

}  // namespace mm
