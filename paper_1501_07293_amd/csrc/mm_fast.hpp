// mm_fast.hpp -- device bodies of the FFT passes specialised at compile time
// for power-of-two padded sizes (the common case: P = 2n with n a power of
// two), shared by the single-grid kernels (mm_fast.hip) and the batched ones
// (mm_batch.hip).  Each body works one tile; the caller passes the tile index
// and an LDS buffer of the size the matching *_lds_elems() gives.
//
// Spectrum layout shared with the generic passes: S = [3][nz][hx][Sy] complex
// (Sy = Py on 3-D grids, ny on one-cell-thick grids), i.e. the x pass writes
// its half spectrum transposed so that every y line is contiguous.
//
// Line passes (x and y): a line of P points is worked by TL = P / R1 threads.
// Stage 1 of the Stockham schedule takes its R1 inputs x[u + TL r] straight
// from global memory (coalesced), stages 2.. go through LDS, and the last
// stage writes x[i + r P/R] straight to global memory (coalesced).  All
// radices, spans and strides are compile-time constants.
//
// Z pass: one thread per (column, component) holds the whole z line in
// registers; components meet in LDS for the Eq. 14 product.
//
// Pruning (line passes): a zero-padded axis has a power-of-two length
// P >= 2n - 1, so P >= 2n and the n valid samples sit in the first half of a
// line.  Forward transforms take the second half as literal zeros and inverse
// transforms never form the outputs of the second half.  A periodic axis
// (n = P) takes the FULL instantiation, which transforms whole lines; the
// launchers pick it when 2n > P.  (The z pass keeps whole lines: pruned there
// it measured slower.)
#pragma once
#include "mm_fft.hpp"
#include "mm_kernels.hpp"

namespace mm {

template <int P, int S>
constexpr int radix_of() { return S == 0 ? Sched<P>::R0 : (S == 1 ? Sched<P>::R1 : Sched<P>::R2); }
template <int P, int S>
constexpr int span_of() { return S == 0 ? 1 : (S == 1 ? Sched<P>::R0 : Sched<P>::R0 * Sched<P>::R1); }

// LDS index with one pad slot every 16 entries (breaks the stride-R1 bank pattern
// of the first-stage writes).
__device__ constexpr int pad16(int e) { return e + (e >> 4); }
// LDS line length: the in-line pad plus one slot so consecutive lines start on
// different banks.
template <int P>
constexpr int padded_len() { return P + P / 16 + 1; }

// Butterflies per thread in stage S >= 1: a line has P / R butterflies of radix
// R and TL = P / R0 threads, so R0 / R each when R divides R0 (every power-of-two
// schedule); otherwise (a stage of radix 3, 5 or 7 after a first radix of 16)
// the last round is partly idle.
template <int P, int S>
constexpr int stage_nb() { return (Sched<P>::R0 + radix_of<P, S>() - 1) / radix_of<P, S>(); }

// Twiddles of stage S >= 1 for one thread: w[q][r - 1] = tw[r k ts] for its
// q-th butterfly (k < p, so an idle butterfly's index stays inside the table).
template <typename T, int P, int S>
struct StageTw {
    static constexpr int R = radix_of<P, S>(), NB = stage_nb<P, S>();
    cpx<T> w[NB][R - 1];
    __device__ inline void load(int u, const cpx<T>* __restrict__ tw)
    {
        constexpr int TL = P / Sched<P>::R0, p = span_of<P, S>(), m = P / R, ts = m / p;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int k = (int)((unsigned)(u + TL * q) % (unsigned)p);
#pragma unroll
            for (int r = 1; r < R; ++r) w[q][r - 1] = tw[r * k * ts];
        }
    }
};

// Stage S >= 1 on one LDS line: each thread does up to NB butterflies.  Reads
// all, barrier, writes all, barrier.  act = false: a thread that only takes part
// in the barriers (a work-group with more threads than its lines need).
template <typename T, int P, int S>
__device__ inline void mid_stage(cpx<T>* ln, int u, const StageTw<T, P, S>& W, bool act = true)
{
    constexpr int R = radix_of<P, S>(), R0 = Sched<P>::R0, TL = P / R0;
    constexpr int p = span_of<P, S>(), m = P / R, NB = stage_nb<P, S>();
    constexpr bool EXACT = NB * TL == m;
    cpx<T> v[NB][R];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = u + TL * q, k = (int)((unsigned)i % (unsigned)p);
        if (act && (EXACT || i < m)) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = ln[pad16(i + r * m)];
            if (k != 0) {
#pragma unroll
                for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], W.w[q][r - 1]);
            }
            Dft<T, R>::run(v[q]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = u + TL * q, k = (int)((unsigned)i % (unsigned)p), j = (i - k) * R + k;
        if (act && (EXACT || i < m)) {
#pragma unroll
            for (int r = 0; r < R; ++r) ln[pad16(j + r * p)] = v[q][r];
        }
    }
    __syncthreads();
}

// Last stage: outputs land at natural index i + r * P/R; handed to `put`.  HALF:
// only the outputs below P / 2 are formed (r < R / 2 for an even last radix, as
// i < P / R).
template <typename T, int P, int S, bool HALF, typename Put>
__device__ inline void last_stage(const cpx<T>* ln, int u, const StageTw<T, P, S>& W, Put put)
{
    constexpr int R = radix_of<P, S>(), R0 = Sched<P>::R0, TL = P / R0;
    constexpr int p = span_of<P, S>(), m = P / R, NB = stage_nb<P, S>();
    constexpr bool EXACT = NB * TL == m;
    static_assert(p == m, "last stage spans P / R");
    static_assert(!HALF || R % 2 == 0, "pruned schedules end on an even radix");
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = u + TL * q;  // < m = p, so the twiddle index k of StageTw is i
        if (!EXACT && i >= m) break;
        cpx<T> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = ln[pad16(i + r * m)];
        if (i != 0) {
#pragma unroll
            for (int r = 1; r < R; ++r) v[r] = cmul(v[r], W.w[q][r - 1]);
        }
        Dft<T, R>::run(v);
#pragma unroll
        for (int r = 0; r < (HALF ? R / 2 : R); ++r) put(i + r * m, v[r]);
    }
}

// Twiddles of stages 1.. of one thread of a line.  They do not depend on the
// data, so the passes load them at the start, where their latency overlaps the
// loads of the line itself.
template <typename T, int P, int NS = Sched<P>::NS>
struct LineTw {
    __device__ inline void load(int, const cpx<T>* __restrict__) {}
};
template <typename T, int P>
struct LineTw<T, P, 2> {
    StageTw<T, P, 1> wl;
    __device__ inline void load(int u, const cpx<T>* __restrict__ tw) { wl.load(u, tw); }
};
template <typename T, int P>
struct LineTw<T, P, 3> {
    StageTw<T, P, 1> wm;
    StageTw<T, P, 2> wl;
    __device__ inline void load(int u, const cpx<T>* __restrict__ tw)
    {
        wm.load(u, tw);
        wl.load(u, tw);
    }
};

// Whole line after stage 1 has been computed into v (registers): write to LDS,
// run the remaining stages, deliver outputs through put (HALF: those below
// P / 2 only).  NS >= 2.
template <typename T, int P, bool HALF = false, typename Put>
__device__ inline void finish_line(cpx<T>* ln, int u, cpx<T>* v, const LineTw<T, P>& W, Put put,
                                   bool act = true)
{
    constexpr int NS = Sched<P>::NS, R0 = Sched<P>::R0;
    if (act) {
#pragma unroll
        for (int r = 0; r < R0; ++r) ln[pad16(u * R0 + r)] = v[r];
    }
    __syncthreads();
    if constexpr (NS == 3) mid_stage<T, P, 1>(ln, u, W.wm, act);
    if (act) last_stage<T, P, NS - 1, HALF>(ln, u, W.wl, put);
}

// In-register FFT of N points (N <= 64), all indices compile-time; Stockham
// order so the output is in natural order.
template <typename T, int N>
__device__ inline void fft_reg(cpx<T>* x, const cpx<T>* __restrict__ tw)
{
    constexpr int NS = Sched<N>::NS;
    if constexpr (NS == 1) {
        Dft<T, N>::run(x);
    } else {
        constexpr int R0 = Sched<N>::R0, R1 = Sched<N>::R1;
        // stage 0 (p = 1): no twiddles
        cpx<T> y[N];
        constexpr int m0 = N / R0;
#pragma unroll
        for (int i = 0; i < m0; ++i) {
            cpx<T> u[R0];
#pragma unroll
            for (int r = 0; r < R0; ++r) u[r] = x[i + r * m0];
            Dft<T, R0>::run(u);
#pragma unroll
            for (int r = 0; r < R0; ++r) y[i * R0 + r] = u[r];
        }
        // stage 1 (p = R0, last): j = i
        constexpr int m1 = N / R1, ts = m1 / R0;
        static_assert(m1 == R0, "two-stage register FFT");
#pragma unroll
        for (int i = 0; i < m1; ++i) {
            cpx<T> u[R1];
#pragma unroll
            for (int r = 0; r < R1; ++r) u[r] = y[i + r * m1];
            if (i != 0) {
#pragma unroll
                for (int r = 1; r < R1; ++r) u[r] = cmul(u[r], tw[r * i * ts]);
            }
            Dft<T, R1>::run(u);
#pragma unroll
            for (int r = 0; r < R1; ++r) x[i + r * m1] = u[r];
        }
    }
}

// ------------------------------------------------------------------ y lines
// Lines per work-group of the y passes (L * TL <= 256 threads; with a mixed-radix
// length TL = P / R0 need not divide 256, and the work-group has L * TL threads).
template <int P>
constexpr int yline_lines() { return 256 / (P / Sched<P>::R0); }

template <typename T, int P, bool INV, bool FULL = false>
__device__ inline void body_yline(const YLineArgs& a, int tile, cpx<T>* lds)
{
    constexpr int R0 = Sched<P>::R0, TL = P / R0, L = yline_lines<P>(), LP = padded_len<P>();
    const int l = threadIdx.x / TL, u = threadIdx.x % TL;
    const int line = tile * L + l;
    const bool ok = line < a.nlines;  // launched with L * TL threads
    int mline = ok ? line : 0;        // its place in memory: plane * hx + bin
    if (a.kx_major) mline = (mline % a.kx_major) * (a.nlines / a.kx_major) + mline / a.kx_major;
    cpx<T>* g = (cpx<T>*)a.buf + (int64_t)mline * a.line_stride;
    const cpx<T>* tw = (const cpx<T>*)a.tw;
    LineTw<T, P> W;
    W.load(u, tw);
    cpx<T> v[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) {
        const int e = u + TL * r;
        cpx<T> x = {(T)0, (T)0};
        if ((INV || FULL || 2 * r < R0) && ok && e < a.nin) x = g[e];  // forward: e >= P/2 is padding
        v[r] = INV ? conj(x) : x;
    }
    Dft<T, R0>::run(v);
    auto put = [&](int e, cpx<T> val) {
        if (ok && e < a.nout) g[e] = INV ? conj(val) : val;
    };
    if constexpr (Sched<P>::NS == 1) {
#pragma unroll
        for (int r = 0; r < R0; ++r) put(r, v[r]);
    } else {
        finish_line<T, P, INV && !FULL>(lds + l * LP, u, v, W, put);
    }
}

// ------------------------------------------------------------------ x forward
constexpr int kLdsBudget = 160 * 1024;
// 8 complex lines (16 consecutive real rows of one (component, z) plane) per
// work-group; the half spectrum is stored transposed, 16 rows per bin.
// A work-group of the x passes holds L complex lines = 2L consecutive rows of
// one plane (L = 8: 128-byte transposed segments in FP32; L = 4: half the LDS,
// twice the work-groups per CU).

template <typename T, int P, int L>
constexpr int x_lds_bytes()
{
    return (int)sizeof(cpx<T>) * ((L * padded_len<P>() > 2 * L * (P / 2 + 1)) ? L * padded_len<P>()
                                                                              : 2 * L * (P / 2 + 1));
}

template <typename T, int P, int L, bool FULL = false>
__device__ inline void body_xfwd(const XLineArgs& a, int tile, cpx<T>* lds)
{
    constexpr int R0 = Sched<P>::R0, TL = P / R0, NT = L * TL, LP = padded_len<P>();
    constexpr int HX = P / 2 + 1, ROWS = 2 * L;
    const int tpp = (a.ny + ROWS - 1) / ROWS;
    const int plane = tile / tpp, yb = (tile - plane * tpp) * ROWS;
    const int l = threadIdx.x / TL, u = threadIdx.x % TL;
    const int y0 = yb + 2 * l;
    const T* in = (const T*)a.in + ((int64_t)plane * a.ny + y0) * a.nx;
    const bool ok0 = y0 < a.ny, ok1 = y0 + 1 < a.ny;
    const cpx<T>* tw = (const cpx<T>*)a.tw;
    cpx<T>* ln = lds + l * LP;
    cpx<T> v[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) {
        const int e = u + TL * r;
        cpx<T> x = {(T)0, (T)0};
        if ((FULL || 2 * r < R0) && e < a.nx) {  // e >= P/2 is zero padding
            if (ok0) x.re = in[e];
            if (ok1) x.im = in[a.nx + e];
        }
        v[r] = x;
    }
    Dft<T, R0>::run(v);
    if constexpr (Sched<P>::NS == 1) {
#pragma unroll
        for (int r = 0; r < R0; ++r) ln[pad16(r)] = v[r];
    } else {
        // the last stage writes back to LDS in natural order (in place: each thread
        // rewrites exactly the slots its own butterflies read)
        // here the twiddles are loaded after the first stage (measured: loaded
        // with the row data they lengthen this pass, unlike the other line passes)
        LineTw<T, P> W;
        W.load(u, tw);
        finish_line<T, P>(ln, u, v, W, [&](int e, cpx<T> val) { ln[pad16(e)] = val; });
    }
    __syncthreads();
    cpx<T>* out = (cpx<T>*)a.out + (int64_t)plane * HX * a.srows;
    // one thread per (bin, row pair): both rows of a pair come from the same two
    // entries of its line and are adjacent in the transposed layout.  With an even
    // row stride (every 3-D grid) and a spectrum that starts on a pair boundary, the
    // pair starts at an even element (yb and 2q are even) and goes out as one
    // aligned store; otherwise as two.
    const bool paired = (a.srows & 1) == 0 &&
                        (reinterpret_cast<uintptr_t>(a.out) % sizeof(cpx2<T>)) == 0;
    for (int idx = threadIdx.x; idx < HX * L; idx += NT) {
        const int q = idx % L, kx = idx / L;
        const cpx<T> zk = lds[q * LP + pad16(kx)];
        const cpx<T> zm = lds[q * LP + pad16(kx == 0 ? 0 : P - kx)];
        // Z = FFT(a + i b): A = (Z_k + conj Z_-k)/2, B = (Z_k - conj Z_-k)/(2i)
        const cpx<T> A = scale(zk + conj(zm), (T)0.5);
        const cpx<T> B = scale(mul_mi(zk - conj(zm)), (T)0.5);
        const int y = yb + 2 * q;
        cpx<T>* o = out + (int64_t)kx * a.srows + y;
        if (paired && y + 1 < a.ny) {
            *reinterpret_cast<cpx2<T>*>(o) = cpx2<T>{A, B};
        } else {
            if (y < a.ny) o[0] = A;
            if (y + 1 < a.ny) o[1] = B;
        }
    }
}

// ------------------------------------------------------------------ x inverse
template <typename T, int P, int L, bool FULL = false>
__device__ inline void body_xinv(const XLineArgs& a, int tile, cpx<T>* lds)
{
    constexpr int R0 = Sched<P>::R0, TL = P / R0, NT = L * TL, LP = padded_len<P>();
    constexpr int HX = P / 2 + 1, ROWS = 2 * L;
    constexpr int LDSN = (L * LP > ROWS * HX) ? L * LP : ROWS * HX;
    const int tpp = (a.ny + ROWS - 1) / ROWS;
    const int plane = tile / tpp, yb = (tile - plane * tpp) * ROWS;
    const int l = threadIdx.x / TL, u = threadIdx.x % TL;
    LineTw<T, P> W;
    W.load(u, (const cpx<T>*)a.tw);
    const cpx<T>* src = (const cpx<T>*)a.in + (int64_t)plane * HX * a.srows;
    // gather the 2L half-spectrum rows of this block, raw[rr][kx]: one thread per
    // (bin, row pair), the two rows adjacent in the transposed layout (one aligned
    // 2-element load under the conditions of the forward pass's paired store);
    // every load is issued before the first LDS store, so the gather costs one
    // memory latency
    constexpr int NEL = HX * L, ITER = (NEL + NT - 1) / NT;
    const bool paired = (a.srows & 1) == 0 &&
                        (reinterpret_cast<uintptr_t>(a.in) % sizeof(cpx2<T>)) == 0;
    cpx2<T> g[ITER];
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
        const int idx = (int)threadIdx.x + it * NT;
        const int q = idx % L, kx = idx / L, y = yb + 2 * q;
        const cpx<T>* p = src + (int64_t)kx * a.srows + y;
        g[it].a = g[it].b = cpx<T>{(T)0, (T)0};
        if (idx < NEL) {
            if (paired && y + 1 < a.ny) {
                g[it] = *reinterpret_cast<const cpx2<T>*>(p);
            } else {
                if (y < a.ny) g[it].a = p[0];
                if (y + 1 < a.ny) g[it].b = p[1];
            }
        }
    }
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
        const int idx = (int)threadIdx.x + it * NT;
        if (idx < NEL) {
            const int q = idx % L, kx = idx / L;
            lds[(2 * q) * HX + kx] = g[it].a;
            lds[(2 * q + 1) * HX + kx] = g[it].b;
        }
    }
    __syncthreads();
    const cpx<T>* ra = lds + (2 * l) * HX;
    const cpx<T>* rb = lds + (2 * l + 1) * HX;
    cpx<T> v[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) {
        const int k = u + TL * r;
        cpx<T> A, B;
        if (k < HX) {
            A = ra[k];
            B = rb[k];
            if (k == 0 || 2 * k == P) {  // DC and Nyquist bins of a real row are real
                A.im = (T)0;
                B.im = (T)0;
            }
        } else {
            A = conj(ra[P - k]);
            B = conj(rb[P - k]);
        }
        v[r] = conj(cpx<T>{A.re - B.im, A.im + B.re});  // conj(A + i B): inverse by conjugation
    }
    Dft<T, R0>::run(v);
    __syncthreads();  // every raw read is done before the FFT reuses the LDS
    const int y0 = yb + 2 * l;
    T* out = (T*)a.out + ((int64_t)plane * a.ny + y0) * a.nx;
    const bool ok0 = y0 < a.ny, ok1 = y0 + 1 < a.ny;
    auto put = [&](int e, cpx<T> val) {  // result a + i b = conj(val)
        if (e < a.nx) {
            if (ok0) out[e] = val.re;
            if (ok1) out[a.nx + e] = -val.im;
        }
    };
    if constexpr (Sched<P>::NS == 1) {
#pragma unroll
        for (int r = 0; r < R0; ++r) put(r, v[r]);
    } else {
        finish_line<T, P, !FULL>(lds + l * LP, u, v, W, put);
    }
}

// ------------------------------------------------------------------ z k-space

template <typename T, int PZ>
__device__ inline void body_kspace_z(const KzArgs& a, int tile, cpx<T>* sh)
{
    constexpr int ZC = kspace_z_cols<T>();
    const int comp = threadIdx.x / ZC, t = threadIdx.x % ZC;
    const int col = tile * ZC + t;
    const bool ok = col < a.ncols;
    // 32-bit element offsets from the uniform base pointers (the spectrum and
    // the octant both stay below 2^31 elements)
    const int zs = a.ncols;  // z stride: one (kx, ky) plane
    const cpx<T>* tw = (const cpx<T>*)a.tw;
    cpx<T>* buf = (cpx<T>*)a.buf;
    const int base = comp * (int)a.comp_stride + (ok ? col : 0);
    cpx<T> v[PZ];
#pragma unroll
    for (int z = 0; z < PZ; ++z) {
        cpx<T> x = {(T)0, (T)0};
        if (ok && z < a.nz) x = buf[base + z * zs];
        v[z] = x;
    }
    // Eq. 14, row `comp` of the symmetric tensor; negative frequencies mirror with
    // the component parities (xy odd in y, xz odd in z, yz odd in y and z).  The
    // 3 x (PZ/2 + 1) spectrum values of this column do not depend on the data:
    // they are loaded before the forward transform, so their latency overlaps it.
    const int kx = (ok ? col : 0) / a.Py;
    int ky = (ok ? col : 0) - kx * a.Py;
    T sy = (T)1;
    if (2 * ky > a.Py) {
        ky = a.Py - ky;
        sy = (T)-1;
    }
    const T* K = (const T*)a.kern;
    const int ko = kx * (int)a.k_xs + ky, cs = (int)a.k_cs, kzs = (int)a.k_zs;
    // the three spectra of row `comp`
    const int c0 = comp == 0 ? 0 : (comp == 1 ? 1 : 2);
    const int c1 = comp == 0 ? 1 : (comp == 1 ? 3 : 4);
    const int c2 = comp == 0 ? 2 : (comp == 1 ? 4 : 5);
    constexpr int H = PZ / 2;
    T k0v[H + 1], k1v[H + 1], k2v[H + 1];
#pragma unroll
    for (int kz = 0; kz <= H; ++kz) {
        const int kk = ko + kz * kzs;
        k0v[kz] = K[c0 * cs + kk];
        k1v[kz] = K[c1 * cs + kk];
        k2v[kz] = K[c2 * cs + kk];
    }
    fft_reg<T, PZ>(v, tw);
#pragma unroll
    for (int z = 0; z < PZ; ++z) sh[(comp * PZ + z) * ZC + t] = v[z];
    __syncthreads();
    // parity signs in y and z (xz, c = 2, and yz, c = 4, are odd in z)
    const T y0 = comp == 1 ? sy : (T)1, y1 = comp == 0 ? sy : (comp == 2 ? sy : (T)1);
    const T y2 = comp == 1 ? sy : (T)1;
    const bool z0 = c0 == 2, z1 = c1 == 4, z2 = (c2 == 2 || c2 == 4);
#pragma unroll
    for (int z = 0; z < PZ; ++z) {
        const int kz = z <= H ? z : PZ - z;
        const T sz = (z <= H || 2 * z == PZ) ? (T)1 : (T)-1;
        const T k0 = y0 * (z0 ? sz : (T)1) * k0v[kz];
        const T k1 = y1 * (z1 ? sz : (T)1) * k1v[kz];
        const T k2 = y2 * (z2 ? sz : (T)1) * k2v[kz];
        const cpx<T> m0 = sh[(0 * PZ + z) * ZC + t];
        const cpx<T> m1 = sh[(1 * PZ + z) * ZC + t];
        const cpx<T> m2 = sh[(2 * PZ + z) * ZC + t];
        const cpx<T> h = {k0 * m0.re + k1 * m1.re + k2 * m2.re, k0 * m0.im + k1 * m1.im + k2 * m2.im};
        v[z] = conj(h);
    }
    fft_reg<T, PZ>(v, tw);
    if (ok) {
#pragma unroll
        for (int z = 0; z < PZ; ++z)
            if (z < a.nz) buf[base + z * zs] = conj(v[z]);
    }
}

// ------------------------------------------------------- z k-space, long lines
// Lines of 128 points or more (thick 3-D grids such as the cubes), whose whole
// lines do not fit a thread's registers: a work-group holds C adjacent columns
// (kx, ky), three component lines each, and transforms them with the line
// passes' register radix stages exchanged through LDS (the input's upper half is
// zero, the kept outputs are the first nz).  Lanes run column fastest, so each
// load and store of one z point covers the C columns as one contiguous segment,
// and the octant loads of the product run along ky.
// Columns per work-group: as many as 1024 threads (3 C (P / R0)) and the LDS (3 C
// padded lines) allow, up to 32: the segments are what the pass waits on (128^3
// cube, Pz = 256, FP32: 8 columns 244 us per Euler step, 16 columns 209 us).  At
// 1024 points at most 512 threads, whose 256 registers a thread hold the lines
// without spilling (FP64 spills even so and keeps the LDS-staged pass).
template <typename T, int P>
constexpr int kzl_cols()
{
    constexpr int TL = P / Sched<P>::R0, MAXT = P >= 1024 ? 512 : 1024;
    int c = 32;
    while (c > 1 && (3 * c * TL > MAXT || 3 * c * padded_len<P>() * (int)sizeof(cpx<T>) > kLdsBudget)) c /= 2;
    return c;
}

template <typename T, int P, int C>
__device__ inline void body_kspace_zl(const KzArgs& a, int tile, cpx<T>* lds)
{
    constexpr int R0 = Sched<P>::R0, TL = P / R0, NT = 3 * C * TL, LP = padded_len<P>();
    static_assert(Sched<P>::NS >= 2, "lines of 128 points or more");
    const int t = (int)threadIdx.x;
    const int l = t % C, u = (t / C) % TL, comp = t / (C * TL);
    const int col = tile * C + l;
    const bool ok = col < a.ncols;
    const int64_t zs = a.ncols;
    cpx<T>* g = (cpx<T>*)a.buf + comp * a.comp_stride + (ok ? col : 0);
    cpx<T>* ln = lds + (comp * C + l) * LP;
    LineTw<T, P> W;
    W.load(u, (const cpx<T>*)a.tw);
    cpx<T> v[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) {
        const int e = u + TL * r;
        cpx<T> x = {(T)0, (T)0};
        if (2 * r < R0 && ok && e < a.nz) x = g[e * zs];  // e >= P/2 is zero padding
        v[r] = x;
    }
    // Eq. 14 spectra of the product elements this thread takes (element idx: column
    // idx % C, kz = idx / C), loaded with the data so their latency overlaps the
    // forward transform; negative frequencies mirror with the component parities
    // (xy odd in y, xz odd in z, yz odd in y and z)
    constexpr int NI = (C * P + NT - 1) / NT;
    const T* K = (const T*)a.kern;
    T kv[NI][6];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int idx = t + it * NT;
        const int l2 = idx % C, e = idx / C, col2 = tile * C + l2;
        const bool in = idx < C * P && col2 < a.ncols;
        const int cc = in ? col2 : 0;
        const int kx = cc / a.Py;
        int ky = cc - kx * a.Py, kz = e;
        T sy = (T)1, sz = (T)1;
        if (2 * ky > a.Py) {
            ky = a.Py - ky;
            sy = (T)-1;
        }
        if (2 * kz > P) {
            kz = P - kz;
            sz = (T)-1;
        }
        const T* Kp = K + (in ? kz * a.k_zs + kx * a.k_xs + ky : 0);
#pragma unroll
        for (int c = 0; c < 6; ++c) kv[it][c] = Kp[c * a.k_cs];
        kv[it][1] *= sy;
        kv[it][2] *= sz;
        kv[it][4] *= sy * sz;
    }
    Dft<T, R0>::run(v);
    finish_line<T, P>(ln, u, v, W, [&](int e, cpx<T> val) { ln[pad16(e)] = val; });
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int idx = t + it * NT;
        const int l2 = idx % C, e = idx / C;
        if (idx >= C * P || tile * C + l2 >= a.ncols) continue;
        const T kxx = kv[it][0], kxy = kv[it][1], kxz = kv[it][2], kyy = kv[it][3], kyz = kv[it][4],
                kzz = kv[it][5];
        cpx<T>* px = lds + (0 * C + l2) * LP + pad16(e);
        cpx<T>* py = lds + (1 * C + l2) * LP + pad16(e);
        cpx<T>* pz = lds + (2 * C + l2) * LP + pad16(e);
        const cpx<T> mx = *px, my = *py, mz = *pz;
        *px = conj(cpx<T>{kxx * mx.re + kxy * my.re + kxz * mz.re, kxx * mx.im + kxy * my.im + kxz * mz.im});
        *py = conj(cpx<T>{kxy * mx.re + kyy * my.re + kyz * mz.re, kxy * mx.im + kyy * my.im + kyz * mz.im});
        *pz = conj(cpx<T>{kxz * mx.re + kyz * my.re + kzz * mz.re, kxz * mx.im + kyz * my.im + kzz * mz.im});
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R0; ++r) v[r] = ln[pad16(u + TL * r)];
    Dft<T, R0>::run(v);
    __syncthreads();  // stage-1 reads of every line are done before LDS is rewritten
    finish_line<T, P, true>(ln, u, v, W, [&](int e, cpx<T> val) {
        if (ok && e < a.nz) g[e * zs] = conj(val);  // inverse by conjugation
    });
}

// Split z lines (FP64, nz <= PZ / 2): two adjacent lanes share a (column,
// component) line, so each holds PZ / 2 values instead of PZ.  With the upper
// half of the input zero, the even outputs are FFT_{PZ/2}(x) and the odd ones
// FFT_{PZ/2}(x_n w^n) (w = exp(-2 pi i / PZ)): lane h = 0 forms the even, lane
// h = 1 the odd, from the same loaded values.  After the product (conjugated),
// the kept outputs n < PZ / 2 are x_n = A_n + w^-n B_n, A and B the inverse
// half transforms of the even and odd products; lane 0 keeps n < PZ / 4, lane 1
// the rest, trading PZ / 4 values across the lane pair.
template <typename T, int PZ>
__device__ inline void body_kspace_z_split(const KzArgs& a, int tile, cpx<T>* sh)
{
    constexpr int ZC = kspace_z_split_cols(), H2 = PZ / 2, Q = PZ / 4;
    static_assert(PZ == 16 || PZ == 32, "half lines of 8 or 16 points: one radix stage");
    const int comp = threadIdx.x / (2 * ZC), rem = threadIdx.x % (2 * ZC);
    const int t = rem >> 1, h = rem & 1;
    const int col = tile * ZC + t;
    const bool ok = col < a.ncols;
    const int zs = a.ncols;
    const cpx<T>* tw = (const cpx<T>*)a.tw;  // length PZ
    cpx<T>* buf = (cpx<T>*)a.buf;
    const int base = comp * (int)a.comp_stride + (ok ? col : 0);
    cpx<T> v[H2];
#pragma unroll
    for (int z = 0; z < H2; ++z) {
        cpx<T> x = {(T)0, (T)0};
        if (ok && z < a.nz) x = buf[base + z * zs];
        v[z] = x;
    }
    const int kx = (ok ? col : 0) / a.Py;
    int ky = (ok ? col : 0) - kx * a.Py;
    T sy = (T)1;
    if (2 * ky > a.Py) {
        ky = a.Py - ky;
        sy = (T)-1;
    }
    const T* K = (const T*)a.kern;
    const int ko = kx * (int)a.k_xs + ky, cs = (int)a.k_cs, kzs = (int)a.k_zs;
    const int c0 = comp == 0 ? 0 : (comp == 1 ? 1 : 2);
    const int c1 = comp == 0 ? 1 : (comp == 1 ? 3 : 4);
    const int c2 = comp == 0 ? 2 : (comp == 1 ? 4 : 5);
    // this lane's kz values 2k + h mirror into the octant rows j = kzm / 2 of its parity
    constexpr int NJ = H2 / 2 + 1;
    T k0v[NJ], k1v[NJ], k2v[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int kzm = 2 * j + h, kk = ko + (kzm <= H2 ? kzm : 0) * kzs;
        k0v[j] = K[c0 * cs + kk];
        k1v[j] = K[c1 * cs + kk];
        k2v[j] = K[c2 * cs + kk];
    }
    if (h) {
#pragma unroll
        for (int z = 0; z < H2; ++z) v[z] = cmul(v[z], tw[z]);
    }
    Dft<T, H2>::run(v);  // v[k] = X(2k + h)
#pragma unroll
    for (int k = 0; k < H2; ++k) sh[(comp * PZ + 2 * k + h) * ZC + t] = v[k];
    __syncthreads();
    const T y0 = comp == 1 ? sy : (T)1, y1 = comp == 0 ? sy : (comp == 2 ? sy : (T)1);
    const T y2 = comp == 1 ? sy : (T)1;
    const bool z0 = c0 == 2, z1 = c1 == 4, z2 = (c2 == 2 || c2 == 4);
#pragma unroll
    for (int k = 0; k < H2; ++k) {
        const int kz = 2 * k + h, kzm = kz <= H2 ? kz : PZ - kz, j = kzm >> 1;
        const T sz = kz <= H2 ? (T)1 : (T)-1;
        const T k0 = y0 * (z0 ? sz : (T)1) * k0v[j];
        const T k1 = y1 * (z1 ? sz : (T)1) * k1v[j];
        const T k2 = y2 * (z2 ? sz : (T)1) * k2v[j];
        const cpx<T> m0 = sh[(0 * PZ + kz) * ZC + t];
        const cpx<T> m1 = sh[(1 * PZ + kz) * ZC + t];
        const cpx<T> m2 = sh[(2 * PZ + kz) * ZC + t];
        const cpx<T> hh = {k0 * m0.re + k1 * m1.re + k2 * m2.re, k0 * m0.im + k1 * m1.im + k2 * m2.im};
        v[k] = conj(hh);  // inverse transform by conjugation
    }
    Dft<T, H2>::run(v);  // conj(A) (h = 0) or conj(B) (h = 1)
    if (h) {
#pragma unroll
        for (int n = 0; n < H2; ++n) v[n] = cmul(v[n], tw[n]);  // conj(w^-n B_n)
    }
    // lane 0 keeps n < Q and takes w^-n B_n from lane 1; lane 1 keeps n >= Q and takes A_n
    cpx<T> o[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const cpx<T> send = h ? v[q] : v[Q + q];
        cpx<T> recv;
        recv.re = __shfl_xor(send.re, 1);
        recv.im = __shfl_xor(send.im, 1);
        o[q] = h ? recv + v[Q + q] : v[q] + recv;
    }
    if (ok) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int n = h * Q + q;
            if (n < a.nz) buf[base + n * zs] = conj(o[q]);
        }
    }
}

// ------------------------------------------------------------ y k-space (2-D)
// One-cell-thick grids: the k-space pass runs along y.  A work-group holds L
// x-bins, three component lines each: forward FFT (stage 1 from global memory),
// Eq. 14 product with the four real spectra (xx, xy, yy, zz) in LDS, inverse
// FFT (stage 1 from LDS, last stage to global memory).
template <int P>
constexpr int ky_lines() { return (256 / (3 * (P / Sched<P>::R0))) > 0 ? 256 / (3 * (P / Sched<P>::R0)) : 1; }

template <typename T, int P, bool FULL = false, int L = ky_lines<P>()>
__device__ inline void body_kspace_y(const KyArgs& a, int tile, cpx<T>* lds)
{
    constexpr int R0 = Sched<P>::R0, TL = P / R0, NT = 3 * L * TL;
    constexpr int LP = padded_len<P>();
    const int line = threadIdx.x / TL, u = threadIdx.x % TL;
    const int comp = line / L, l = line - comp * L;
    const int kx = tile * L + l;
    const bool ok = kx < a.hx;
    cpx<T>* g = (cpx<T>*)a.buf + comp * a.comp_stride + (int64_t)(ok ? kx : 0) * a.line_stride;
    cpx<T>* ln = lds + line * LP;
    const cpx<T>* tw = (const cpx<T>*)a.tw;
    LineTw<T, P> W;
    W.load(u, tw);
    cpx<T> v[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) {
        const int e = u + TL * r;
        cpx<T> x = {(T)0, (T)0};
        if ((FULL || 2 * r < R0) && ok && e < a.ny) x = g[e];  // e >= P/2 is zero padding
        v[r] = x;
    }
    // the spectra of the product elements this thread takes do not depend on the
    // data: loaded here, their latency overlaps the forward transform
    constexpr int NI = (L * P + NT - 1) / NT;
    const T* K = (const T*)a.kern;
    T kv[NI][4];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int idx = (int)threadIdx.x + it * NT;
        const int l2 = idx / P, e = idx - l2 * P, kx2 = tile * L + l2;
        int ky = e;
        if (2 * ky > P) ky = P - ky;
        const bool in = idx < L * P && kx2 < a.hx;
        const T* Kp = K + (in ? (int64_t)kx2 * a.k_xs + ky : 0);
#pragma unroll
        for (int c = 0; c < 4; ++c) kv[it][c] = Kp[c * a.k_cs];
    }
    Dft<T, R0>::run(v);
    if constexpr (Sched<P>::NS == 1) {
#pragma unroll
        for (int r = 0; r < R0; ++r) ln[pad16(r)] = v[r];
    } else {
        finish_line<T, P>(ln, u, v, W, [&](int e, cpx<T> val) { ln[pad16(e)] = val; });
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int idx = (int)threadIdx.x + it * NT;
        const int l2 = idx / P, e = idx - l2 * P, kx2 = tile * L + l2;
        if (idx >= L * P || kx2 >= a.hx) continue;
        const T sy = 2 * e > P ? (T)-1 : (T)1;
        const T kxx = kv[it][0], kxy = sy * kv[it][1], kyy = kv[it][2], kzz = kv[it][3];
        cpx<T>* px = lds + (0 * L + l2) * LP + pad16(e);
        cpx<T>* py = lds + (1 * L + l2) * LP + pad16(e);
        cpx<T>* pz = lds + (2 * L + l2) * LP + pad16(e);
        const cpx<T> mx = *px, my = *py, mz = *pz;
        *px = conj(cpx<T>{kxx * mx.re + kxy * my.re, kxx * mx.im + kxy * my.im});
        *py = conj(cpx<T>{kxy * mx.re + kyy * my.re, kxy * mx.im + kyy * my.im});
        *pz = conj(cpx<T>{kzz * mz.re, kzz * mz.im});
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R0; ++r) v[r] = ln[pad16(u + TL * r)];
    Dft<T, R0>::run(v);
    auto put = [&](int e, cpx<T> val) {
        if (ok && e < a.ny) g[e] = conj(val);
    };
    if constexpr (Sched<P>::NS == 1) {
#pragma unroll
        for (int r = 0; r < R0; ++r) put(r, v[r]);
    } else {
        __syncthreads();  // stage-1 reads of every line are done before LDS is rewritten
        finish_line<T, P, !FULL>(ln, u, v, W, put);
    }
}

// ------------------------------------------------- y k-space (two cells thick)
// Grids of two cells along z (nz = 2, open z): the z coupling of the two planes
// is a 2 x 2 block sum with the tensor planes at z offsets -1, 0, 1 (the layout
// and parities of the 10 coefficient planes are given with Ky2Args), so no z
// transform, no z padding and no Py-long spectrum in HBM: a work-group holds L
// x bins, six lines each (three components of both planes), runs the forward
// y FFT (stage 1 from global memory), the block product in LDS, and the inverse
// (last stage to global memory).
template <int P>
constexpr int ky2_lines() { return (256 / (6 * (P / Sched<P>::R0))) > 0 ? 256 / (6 * (P / Sched<P>::R0)) : 1; }

template <typename T, int P, bool FULL = false>
__device__ inline void body_kspace_y2(const Ky2Args& a, int tile, cpx<T>* lds)
{
    constexpr int R0 = Sched<P>::R0, TL = P / R0, L = ky2_lines<P>(), NT = 6 * L * TL;
    constexpr int LP = padded_len<P>();
    const int line = threadIdx.x / TL, u = threadIdx.x % TL;
    const int cz = line / L, l = line - cz * L;  // cz = 2 component + plane
    const int kx = tile * L + l;
    const bool ok = kx < a.hx;
    cpx<T>* g = (cpx<T>*)a.buf + (cz >> 1) * a.comp_stride + (cz & 1) * a.plane_stride +
                (int64_t)(ok ? kx : 0) * a.line_stride;
    cpx<T>* ln = lds + line * LP;
    const cpx<T>* tw = (const cpx<T>*)a.tw;
    LineTw<T, P> W;
    W.load(u, tw);
    cpx<T> v[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) {
        const int e = u + TL * r;
        cpx<T> x = {(T)0, (T)0};
        if ((FULL || 2 * r < R0) && ok && e < a.ny) x = g[e];  // e >= P/2 is zero padding
        v[r] = x;
    }
    // the coefficients of this thread's product elements, loaded with the data
    constexpr int NI = (L * P + NT - 1) / NT;
    const T* K = (const T*)a.kern;
    const int64_t cs = a.k_cs;
    T kv[NI][kTwoPlaneTablePlanes];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int idx = (int)threadIdx.x + it * NT;
        const int l2 = idx / P, e = idx - l2 * P, kx2 = tile * L + l2;
        int ky = e;
        if (2 * ky > P) ky = P - ky;
        const bool in = idx < L * P && kx2 < a.hx;
        const T* Kp = K + (in ? (int64_t)kx2 * a.k_xs + ky : 0);
#pragma unroll
        for (int c = 0; c < kTwoPlaneTablePlanes; ++c) kv[it][c] = Kp[c * cs];
    }
    Dft<T, R0>::run(v);
    if constexpr (Sched<P>::NS == 1) {
#pragma unroll
        for (int r = 0; r < R0; ++r) ln[pad16(r)] = v[r];
    } else {
        finish_line<T, P>(ln, u, v, W, [&](int e, cpx<T> val) { ln[pad16(e)] = val; });
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int idx = (int)threadIdx.x + it * NT;
        const int l2 = idx / P, e = idx - l2 * P, kx2 = tile * L + l2;
        if (idx >= L * P || kx2 >= a.hx) continue;
        const T sy = 2 * e > P ? (T)-1 : (T)1;
        const T xx0 = kv[it][0], xx1 = kv[it][1], xy0 = sy * kv[it][2], xy1 = sy * kv[it][3];
        const T sxz = kv[it][4], yy0 = kv[it][5], yy1 = kv[it][6], syz = sy * kv[it][7];
        const T zz0 = kv[it][8], zz1 = kv[it][9];
        // line (component c, plane z) of bin l2 at LDS line (2 c + z) L + l2
        cpx<T>* p[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) p[q] = lds + (q * L + l2) * LP + pad16(e);
        const cpx<T> ax = *p[0], bx = *p[1], ay = *p[2], by = *p[3], az = *p[4], bz = *p[5];
        // plane 0 (observer z = 0): K^(0) a + K^(-1) b, with K^(-1)_xz = -i Sxz, K^(-1)_yz = -i Syz
        // plane 1 (observer z = 1): K^(1) a + K^(0) b, with K^(1)_xz = i Sxz, K^(1)_yz = i Syz
        // (-i s (u + i v) = s v - i s u; i s (u + i v) = -s v + i s u)
        const cpx<T> h0x = {xx0 * ax.re + xy0 * ay.re + xx1 * bx.re + xy1 * by.re + sxz * bz.im,
                            xx0 * ax.im + xy0 * ay.im + xx1 * bx.im + xy1 * by.im - sxz * bz.re};
        const cpx<T> h0y = {xy0 * ax.re + yy0 * ay.re + xy1 * bx.re + yy1 * by.re + syz * bz.im,
                            xy0 * ax.im + yy0 * ay.im + xy1 * bx.im + yy1 * by.im - syz * bz.re};
        const cpx<T> h0z = {zz0 * az.re + zz1 * bz.re + sxz * bx.im + syz * by.im,
                            zz0 * az.im + zz1 * bz.im - sxz * bx.re - syz * by.re};
        const cpx<T> h1x = {xx1 * ax.re + xy1 * ay.re + xx0 * bx.re + xy0 * by.re - sxz * az.im,
                            xx1 * ax.im + xy1 * ay.im + xx0 * bx.im + xy0 * by.im + sxz * az.re};
        const cpx<T> h1y = {xy1 * ax.re + yy1 * ay.re + xy0 * bx.re + yy0 * by.re - syz * az.im,
                            xy1 * ax.im + yy1 * ay.im + xy0 * bx.im + yy0 * by.im + syz * az.re};
        const cpx<T> h1z = {zz1 * az.re + zz0 * bz.re - sxz * ax.im - syz * ay.im,
                            zz1 * az.im + zz0 * bz.im + sxz * ax.re + syz * ay.re};
        // stored conjugated: the inverse transform runs as a forward one
        *p[0] = conj(h0x);
        *p[1] = conj(h1x);
        *p[2] = conj(h0y);
        *p[3] = conj(h1y);
        *p[4] = conj(h0z);
        *p[5] = conj(h1z);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R0; ++r) v[r] = ln[pad16(u + TL * r)];
    Dft<T, R0>::run(v);
    auto put = [&](int e, cpx<T> val) {
        if (ok && e < a.ny) g[e] = conj(val);
    };
    if constexpr (Sched<P>::NS == 1) {
#pragma unroll
        for (int r = 0; r < R0; ++r) put(r, v[r]);
    } else {
        __syncthreads();  // stage-1 reads of every line are done before LDS is rewritten
        finish_line<T, P, !FULL>(ln, u, v, W, put);
    }
}

// LDS entries (complex) each body needs.
template <int P>
constexpr int yline_lds_elems() { return yline_lines<P>() * padded_len<P>(); }
template <int P, int L>
constexpr int xfwd_lds_elems() { return L * padded_len<P>(); }
template <int P, int L>
constexpr int xinv_lds_elems()
{
    return (L * padded_len<P>() > 2 * L * (P / 2 + 1)) ? L * padded_len<P>() : 2 * L * (P / 2 + 1);
}
template <typename T, int PZ>
constexpr int kspace_z_lds_elems() { return 3 * PZ * kspace_z_cols<T>(); }
template <int P, int L = ky_lines<P>()>
constexpr int kspace_y_lds_elems() { return 3 * L * padded_len<P>(); }
template <int P>
constexpr int kspace_y2_lds_elems() { return 6 * ky2_lines<P>() * padded_len<P>(); }

}  // namespace mm
