// mm_generic.hpp -- device bodies of the runtime-radix FFT passes (any
// 7-smooth length), shared by the single-grid kernels (mm_passes.hip) and the
// batched kernels (mm_batch.hip).  Each body works one tile of its pass; the
// caller supplies the tile index, the LDS buffer (lds_elems(NT) entries) and
// the radix schedule (by reference, so a schedule held in memory is indexed in
// place rather than copied into registers).
#pragma once
#include "mm_demag1.hpp"
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

// Global loads of the input loops go through registers in groups of kStage per
// thread, all issued before the group's LDS stores, so a group costs one
// memory latency instead of one per element.
constexpr int kStage = 8;

// ------------------------------------------------------------------ x forward
template <typename T, int NT>
__device__ void body_row_r2c(const RowR2CArgs& a, const FftPlan& pl, int tile, cpx<T>* lds)
{
    const int P = pl.P, LS = P + 1, B = a.lines_per_wg;
    const int npairs = (a.nrows + 1) >> 1;
    const int q0 = tile * B;
    const T* in = (const T*)a.in;
    const int BP = B * P;
    for (int i0 = 0; i0 < BP; i0 += kStage * NT) {
        cpx<T> v[kStage];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int idx = i0 + (int)threadIdx.x + u * NT;
            const int q = idx / P, x = idx - q * P, pr = q0 + q;
            v[u] = cpx<T>{(T)0, (T)0};
            if (idx < BP && pr < npairs && x < a.nvalid) {
                const int r0 = 2 * pr;
                v[u].re = in[(int64_t)r0 * a.in_row_stride + x];
                if (r0 + 1 < a.nrows) v[u].im = in[(int64_t)(r0 + 1) * a.in_row_stride + x];
            }
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int idx = i0 + (int)threadIdx.x + u * NT;
            if (idx < BP) lds[(idx / P) * LS + idx % P] = v[u];
        }
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
    const int BP = B * P;
    for (int i0 = 0; i0 < BP; i0 += kStage * NT) {
        cpx<T> A[kStage], Bv[kStage];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int idx = i0 + (int)threadIdx.x + u * NT;
            const int q = idx / P, x = idx - q * P, pr = q0 + q;
            A[u] = Bv[u] = cpx<T>{(T)0, (T)0};
            if (idx < BP && pr < npairs) {
                const int r0 = 2 * pr;
                const bool has1 = r0 + 1 < a.nrows;
                const int64_t o0 = row_off(r0, a.rows_per_plane, a.in_plane_stride, a.rstride);
                const int64_t o1 = has1 ? row_off(r0 + 1, a.rows_per_plane, a.in_plane_stride, a.rstride) : 0;
                const int64_t kk = (int64_t)(x < a.hx ? x : P - x) * a.kstride;
                A[u] = in[o0 + kk];
                if (has1) Bv[u] = in[o1 + kk];
            }
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int idx = i0 + (int)threadIdx.x + u * NT;
            if (idx >= BP) continue;
            const int q = idx / P, x = idx - q * P;
            cpx<T> a0 = A[u], b0 = Bv[u];
            if (x < a.hx) {
                if (x == 0 || (evenP && 2 * x == P)) {  // DC and Nyquist bins are real
                    a0.im = (T)0;
                    b0.im = (T)0;
                }
            } else {
                a0 = conj(a0);
                b0 = conj(b0);
            }
            const cpx<T> z = {a0.re - b0.im, a0.im + b0.re};  // A + i B
            lds[q * LS + x] = conj(z);
        }
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
    const int PTW = P * TW;
    for (int i0 = 0; i0 < PTW; i0 += kStage * NT) {
        cpx<T> v[kStage];
        bool ok[kStage];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int idx = i0 + (int)threadIdx.x + u * NT;
            const int e = idx / TW, t = idx - e * TW, col = c0 + t;
            v[u] = cpx<T>{(T)0, (T)0};
            ok[u] = idx < PTW && e < a.nin && col < a.ncols;
            if (ok[u]) v[u] = buf[e * a.es + col_off(col, a.cols_per_row, a.row2_stride)];
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int idx = i0 + (int)threadIdx.x + u * NT;
            if (idx < PTW) lds[idx] = (a.inverse && ok[u]) ? conj(v[u]) : v[u];
        }
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
    const int BP = B * P;
    for (int i0 = 0; i0 < BP; i0 += kStage * NT) {
        cpx<T> v[kStage];
        bool ok[kStage];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int idx = i0 + (int)threadIdx.x + u * NT;
            const int q = idx / P, e = idx - q * P, l = l0 + q;
            v[u] = cpx<T>{(T)0, (T)0};
            ok[u] = idx < BP && l < a.nlines && e < a.nin;
            if (ok[u]) v[u] = buf[(int64_t)l * a.line_stride + e];
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int idx = i0 + (int)threadIdx.x + u * NT;
            if (idx < BP) lds[(idx / P) * LS + idx % P] = (a.inverse && ok[u]) ? conj(v[u]) : v[u];
        }
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
// PF > 0: the last-axis length is PF (a power of two), fixed at compile time.
template <typename T, int NT, int PF = 0>
__device__ void body_kspace(const KspArgs& a, const FftPlan& pl, int tile, cpx<T>* lds)
{
    const int P = PF > 0 ? PF : pl.P, TW = a.tw_cols;
    const int c0 = tile * TW;
    cpx<T>* buf = (cpx<T>*)a.buf;
    const int PT = P * TW;
    for (int i0 = 0; i0 < 3 * PT; i0 += kStage * NT) {
        cpx<T> v[kStage];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int idx = i0 + (int)threadIdx.x + u * NT;
            const int c = idx / PT, rem = idx - c * PT, e = rem / TW, t = rem - e * TW, col = c0 + t;
            v[u] = cpx<T>{(T)0, (T)0};
            if (idx < 3 * PT && e < a.nvalid && col < a.ncols)
                v[u] = buf[c * a.comp_stride + e * a.es + col_off(col, a.cols_per_row, a.row2_stride)];
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int idx = i0 + (int)threadIdx.x + u * NT;
            if (idx < 3 * PT) lds[idx] = v[u];
        }
    }
    __syncthreads();
    const LdsGeom g{3 * TW, TW, 1, PT, TW};
    if constexpr (PF > 0)
        lds_fft_fixed<T, NT, PF, true>(lds, g, (const cpx<T>*)a.tw, threadIdx.x);
    else
        lds_fft<T, NT, true>(lds, g, pl, (const cpx<T>*)a.tw, threadIdx.x);
    // Eq. 14: H~_a = sum_b K~_ab M~_b with the real, symmetric kernel spectrum.
    const T* K = (const T*)a.kern;
    constexpr int KS = kStage / 2;  // elements per thread whose spectra load together
    for (int i0 = 0; i0 < PT; i0 += KS * NT) {
        T kv[KS][6];
        bool ok[KS];
#pragma unroll
        for (int u = 0; u < KS; ++u) {
            const int idx = i0 + (int)threadIdx.x + u * NT;
            const int e = idx / TW, t = idx - e * TW, col = c0 + t;
            ok[u] = idx < PT && col < a.ncols;
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
            const int64_t ko = ok[u] ? kz * a.k_zs + kx * a.k_xs + ky : 0;
#pragma unroll
            for (int c = 0; c < 6; ++c) kv[u][c] = (T)0;
            if (ok[u]) {
                if (a.ncomp == 6) {
#pragma unroll
                    for (int c = 0; c < 6; ++c) kv[u][c] = K[c * a.k_cs + ko];
                } else {  // xx, xy, yy, zz
                    kv[u][0] = K[ko];
                    kv[u][1] = K[a.k_cs + ko];
                    kv[u][3] = K[2 * a.k_cs + ko];
                    kv[u][5] = K[3 * a.k_cs + ko];
                }
            }
            // parities of the mirrored octant: xy odd in y, xz odd in z, yz odd in both
            kv[u][1] *= sy;
            kv[u][2] *= sz;
            kv[u][4] *= sy * sz;
        }
        // Eq. 14: H~_a = sum_b K~_ab M~_b with the real, symmetric kernel spectrum.
#pragma unroll
        for (int u = 0; u < KS; ++u) {
            if (!ok[u]) continue;
            const int idx = i0 + (int)threadIdx.x + u * NT;
            const T kxx = kv[u][0], kxy = kv[u][1], kxz = kv[u][2], kyy = kv[u][3], kyz = kv[u][4],
                    kzz = kv[u][5];
            const cpx<T> mx = lds[idx], my = lds[PT + idx], mz = lds[2 * PT + idx];
            const cpx<T> hx = {kxx * mx.re + kxy * my.re + kxz * mz.re, kxx * mx.im + kxy * my.im + kxz * mz.im};
            const cpx<T> hy = {kxy * mx.re + kyy * my.re + kyz * mz.re, kxy * mx.im + kyy * my.im + kyz * mz.im};
            const cpx<T> hz = {kxz * mx.re + kyz * my.re + kzz * mz.re, kxz * mx.im + kyz * my.im + kzz * mz.im};
            lds[idx] = conj(hx);  // inverse transform by conjugation
            lds[PT + idx] = conj(hy);
            lds[2 * PT + idx] = conj(hz);
        }
    }
    __syncthreads();
    if constexpr (PF > 0)
        lds_fft_fixed<T, NT, PF, true>(lds, g, (const cpx<T>*)a.tw, threadIdx.x);
    else
        lds_fft<T, NT, true>(lds, g, pl, (const cpx<T>*)a.tw, threadIdx.x);
    const int VT = a.nvalid * TW;
    for (int idx = threadIdx.x; idx < 3 * VT; idx += NT) {
        const int c = idx / VT, rem = idx - c * VT, e = rem / TW, t = rem - e * TW, col = c0 + t;
        if (col >= a.ncols) continue;
        buf[c * a.comp_stride + e * a.es + col_off(col, a.cols_per_row, a.row2_stride)] =
            conj(lds[c * PT + e * TW + t]);
    }
}

// Fused y-z pass: x bin `tile`; LDS element (c, z, y) at c Py Pz + z Py + y.
// The y lines of the nz valid planes are transformed (the others are zero),
// then every z line; after the product (written conjugated) every z line and
// the y lines of the nz planes that are kept go back through the forward
// transform, and the conjugate of the valid window is stored.
template <typename T, int NT>
__device__ void body_kspace_yz(const KyzArgs& a, int tile, cpx<T>* lds)
{
    const int kx = tile, Py = a.Py, Pz = a.Pz, PP = Py * Pz;
    cpx<T>* buf = (cpx<T>*)a.buf;
    const int64_t col = (int64_t)kx * a.Sy;
    for (int i0 = 0; i0 < 3 * PP; i0 += kStage * NT) {
        cpx<T> v[kStage];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int idx = i0 + (int)threadIdx.x + u * NT;
            const int c = idx / PP, rem = idx - c * PP, z = rem / Py, y = rem - z * Py;
            v[u] = cpx<T>{(T)0, (T)0};
            if (idx < 3 * PP && z < a.nz && y < a.ny) v[u] = buf[c * a.comp_stride + z * a.zs + col + y];
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int idx = i0 + (int)threadIdx.x + u * NT;
            if (idx < 3 * PP) lds[idx] = v[u];
        }
    }
    __syncthreads();
    // y lines (c, z < nz): element y at c PP + z Py + y;  z lines (c, y): at c PP + y + z Py
    const LdsGeom gy{3 * a.nz, a.nz, Py, PP, 1};
    const LdsGeom gz{3 * Py, Py, 1, PP, Py};
    const cpx<T>* twy = (const cpx<T>*)a.twy;
    const cpx<T>* twz = (const cpx<T>*)a.twz;
    lds_fft<T, NT, false>(lds, gy, a.ply, twy, threadIdx.x);
    lds_fft<T, NT, true>(lds, gz, a.plz, twz, threadIdx.x);
    // Eq. 14: H~_a = sum_b K~_ab M~_b; negative ky and kz mirror into the octant
    // with the parities of the components (xy odd in y, xz odd in z, yz odd in both)
    const T* K = (const T*)a.kern;
    for (int idx = threadIdx.x; idx < PP; idx += NT) {
        int kz = idx / Py, ky = idx - kz * Py;
        T sy = (T)1, sz = (T)1;
        if (2 * ky > Py) {
            ky = Py - ky;
            sy = (T)-1;
        }
        if (2 * kz > Pz) {
            kz = Pz - kz;
            sz = (T)-1;
        }
        const int64_t ko = kz * a.k_zs + kx * a.k_xs + ky;
        const T kxx = K[ko], kxy = sy * K[a.k_cs + ko], kxz = sz * K[2 * a.k_cs + ko];
        const T kyy = K[3 * a.k_cs + ko], kyz = sy * sz * K[4 * a.k_cs + ko], kzz = K[5 * a.k_cs + ko];
        const cpx<T> mx = lds[idx], my = lds[PP + idx], mz = lds[2 * PP + idx];
        const cpx<T> hx = {kxx * mx.re + kxy * my.re + kxz * mz.re, kxx * mx.im + kxy * my.im + kxz * mz.im};
        const cpx<T> hy = {kxy * mx.re + kyy * my.re + kyz * mz.re, kxy * mx.im + kyy * my.im + kyz * mz.im};
        const cpx<T> hz = {kxz * mx.re + kyz * my.re + kzz * mz.re, kxz * mx.im + kyz * my.im + kzz * mz.im};
        lds[idx] = conj(hx);  // inverse transform by conjugation
        lds[PP + idx] = conj(hy);
        lds[2 * PP + idx] = conj(hz);
    }
    __syncthreads();
    lds_fft<T, NT, true>(lds, gz, a.plz, twz, threadIdx.x);
    lds_fft<T, NT, false>(lds, gy, a.ply, twy, threadIdx.x);
    const int VV = a.nz * a.ny;
    for (int idx = threadIdx.x; idx < 3 * VV; idx += NT) {
        const int c = idx / VV, rem = idx - c * VV, z = rem / a.ny, y = rem - z * a.ny;
        buf[c * a.comp_stride + z * a.zs + col + y] = conj(lds[c * PP + z * Py + y]);
    }
}

// Eq. 14 for a whole small grid in one work-group: the padded volume
// [3][Pz][Py][Px] (x fastest) of complex values sits in LDS; m enters as the real
// part (zero padding around it), every x, y and z line is transformed, the
// product with the real symmetric spectrum is taken at every (kx, ky, kz) with
// negative frequencies mirrored into the octant (xy odd in x and y, xz in x and z,
// yz in y and z), and the conjugated product goes back through the forward
// transforms; the real part of the valid window is the field.
template <typename T, int NT>
__device__ void body_demag_1wg(const Demag1Args& a, cpx<T>* lds)
{
    const int Px = a.Px, Py = a.Py, Pz = a.Pz;
    const int A = Px * Py, V = A * Pz;
    const T* m = (const T*)a.m;
    const int64_t N = (int64_t)a.nx * a.ny * a.nz;
    for (int idx = threadIdx.x; idx < 3 * V; idx += NT) {
        const int c = idx / V, r = idx - c * V, z = r / A, r2 = r - z * A, y = r2 / Px, x = r2 - y * Px;
        T v = (T)0;
        if (x < a.nx && y < a.ny && z < a.nz) v = m[c * N + ((int64_t)z * a.ny + y) * a.nx + x];
        lds[idx] = cpx<T>{v, (T)0};
    }
    __syncthreads();
    // x lines: 3 Pz Py of them, contiguous; y lines: (c, z, x), stride Px;
    // z lines: (c, y, x), stride Px Py
    const LdsGeom gx{3 * Pz * Py, 3 * Pz * Py, Px, 0, 1};
    const LdsGeom gy{3 * Pz * Px, Px, 1, A, Px};
    const LdsGeom gz{3 * A, A, 1, V, A};
    const cpx<T>* twx = (const cpx<T>*)a.twx;
    const cpx<T>* twy = (const cpx<T>*)a.twy;
    const cpx<T>* twz = (const cpx<T>*)a.twz;
    lds_fft<T, NT, false>(lds, gx, a.plx, twx, threadIdx.x);
    lds_fft<T, NT, true>(lds, gy, a.ply, twy, threadIdx.x);
    if (Pz > 1) lds_fft<T, NT, true>(lds, gz, a.plz, twz, threadIdx.x);
    const T* K = (const T*)a.kern;
    const bool six = a.ncomp == 6;
    for (int idx = threadIdx.x; idx < V; idx += NT) {
        int kz = idx / A;
        const int r2 = idx - kz * A;
        int ky = r2 / Px, kx = r2 - ky * Px;
        T sx = (T)1, sy = (T)1, sz = (T)1;
        if (2 * kx > Px) {
            kx = Px - kx;
            sx = (T)-1;
        }
        if (2 * ky > Py) {
            ky = Py - ky;
            sy = (T)-1;
        }
        if (2 * kz > Pz) {
            kz = Pz - kz;
            sz = (T)-1;
        }
        const int64_t ko = kz * a.k_zs + kx * a.k_xs + ky;
        const T kxx = K[ko];
        const T kxy = sx * sy * K[a.k_cs + ko];
        const T kxz = six ? sx * sz * K[2 * a.k_cs + ko] : (T)0;
        const T kyy = K[(six ? 3 : 2) * a.k_cs + ko];
        const T kyz = six ? sy * sz * K[4 * a.k_cs + ko] : (T)0;
        const T kzz = K[(six ? 5 : 3) * a.k_cs + ko];
        const cpx<T> mx = lds[idx], my = lds[V + idx], mz = lds[2 * V + idx];
        const cpx<T> hx = {kxx * mx.re + kxy * my.re + kxz * mz.re, kxx * mx.im + kxy * my.im + kxz * mz.im};
        const cpx<T> hy = {kxy * mx.re + kyy * my.re + kyz * mz.re, kxy * mx.im + kyy * my.im + kyz * mz.im};
        const cpx<T> hz = {kxz * mx.re + kyz * my.re + kzz * mz.re, kxz * mx.im + kyz * my.im + kzz * mz.im};
        lds[idx] = conj(hx);  // inverse transform by conjugation
        lds[V + idx] = conj(hy);
        lds[2 * V + idx] = conj(hz);
    }
    __syncthreads();
    if (Pz > 1) lds_fft<T, NT, true>(lds, gz, a.plz, twz, threadIdx.x);
    lds_fft<T, NT, true>(lds, gy, a.ply, twy, threadIdx.x);
    lds_fft<T, NT, false>(lds, gx, a.plx, twx, threadIdx.x);
    // Re(conj(w)) = Re(w): the real part of the valid window is the field
    T* hd = (T*)a.hd;
    for (int64_t idx = threadIdx.x; idx < 3 * N; idx += NT) {
        const int64_t c = idx / N, r = idx - c * N;
        const int x = (int)(r % a.nx), y = (int)((r / a.nx) % a.ny), z = (int)(r / ((int64_t)a.nx * a.ny));
        hd[idx] = lds[c * V + (z * Py + y) * Px + x].re;
    }
}

}  // namespace mm
