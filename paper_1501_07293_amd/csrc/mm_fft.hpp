// mm_fft.hpp -- batched complex FFTs held in LDS (device side).
//
// A work-group owns a batch of lines of length P in LDS.  Each stage of a
// mixed-radix Stockham (autosort) decimation-in-time schedule reads R inputs
// spaced P/R apart, applies the twiddles exp(-2 pi i r k / (p R)) with
// k = i mod p (p = product of the earlier radices), runs a radix-R DFT in
// registers and writes the R outputs to j + r p with j = (i - k) R + k.
// Reads of one stage all complete (barrier) before any write, so a single LDS
// buffer suffices.  Only forward transforms are built; an inverse is
// conj(FFT(conj(x))), done by the callers at load and store.
//
// Twiddles come from a length-P table tw[t] = exp(-2 pi i t / P), built in
// FP64 and rounded once to the working precision.
#pragma once
#include "mm_common.hpp"

namespace mm {

// ---------------------------------------------------------------- radix DFTs
template <typename T, int R>
struct Dft;

template <typename T>
struct Dft<T, 2> {
    __device__ static inline void run(cpx<T>* v)
    {
        cpx<T> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    }
};

template <typename T>
__device__ inline void dft4(cpx<T>& x0, cpx<T>& x1, cpx<T>& x2, cpx<T>& x3)
{
    cpx<T> t0 = x0 + x2, t1 = x0 - x2, t2 = x1 + x3, t3 = mul_mi(x1 - x3);
    x0 = t0 + t2;
    x2 = t0 - t2;
    x1 = t1 + t3;
    x3 = t1 - t3;
}

template <typename T>
struct Dft<T, 4> {
    __device__ static inline void run(cpx<T>* v) { dft4(v[0], v[1], v[2], v[3]); }
};

template <typename T>
struct Dft<T, 8> {
    __device__ static inline void run(cpx<T>* v)
    {
        const T c = (T)0.70710678118654752440;
        cpx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
        cpx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
        dft4(e0, e1, e2, e3);
        dft4(o0, o1, o2, o3);
        // o_k *= exp(-2 pi i k / 8)
        o1 = {c * (o1.re + o1.im), c * (o1.im - o1.re)};
        o2 = mul_mi(o2);
        o3 = {c * (o3.im - o3.re), -c * (o3.re + o3.im)};
        v[0] = e0 + o0;
        v[4] = e0 - o0;
        v[1] = e1 + o1;
        v[5] = e1 - o1;
        v[2] = e2 + o2;
        v[6] = e2 - o2;
        v[3] = e3 + o3;
        v[7] = e3 - o3;
    }
};

// exp(-2 pi i j / 16) for j = 0..9 (the products n2 k1 of a 4x4 split)
template <typename T>
__device__ inline cpx<T> w16(int j)
{
    const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;
    const T c2 = (T)0.70710678118654752440;
    switch (j) {
    case 0: return {(T)1, (T)0};
    case 1: return {c1, -s1};
    case 2: return {c2, -c2};
    case 3: return {s1, -c1};
    case 4: return {(T)0, (T)-1};
    case 6: return {-c2, -c2};
    default: return {-c1, s1};  // j = 9 (only remaining product of {1,2,3}x{1,2,3})
    }
}

template <typename T>
struct Dft<T, 16> {
    __device__ static inline void run(cpx<T>* v)
    {
        // n = 4 n1 + n2, k = k1 + 4 k2
        cpx<T> a[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            a[n2][0] = v[n2];
            a[n2][1] = v[4 + n2];
            a[n2][2] = v[8 + n2];
            a[n2][3] = v[12 + n2];
            dft4(a[n2][0], a[n2][1], a[n2][2], a[n2][3]);
        }
#pragma unroll
        for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
            for (int k1 = 1; k1 < 4; ++k1) a[n2][k1] = cmul(a[n2][k1], w16<T>(n2 * k1));
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            cpx<T> b0 = a[0][k1], b1 = a[1][k1], b2 = a[2][k1], b3 = a[3][k1];
            dft4(b0, b1, b2, b3);
            v[k1] = b0;
            v[k1 + 4] = b1;
            v[k1 + 8] = b2;
            v[k1 + 12] = b3;
        }
    }
};

// Odd radices by symmetric pairs: y_k = x_0 + sum_n [(x_n + x_{R-n}) cos(2 pi n k/R)
//                                               - i (x_n - x_{R-n}) sin(2 pi n k/R)].
template <int R>
struct OddTab;
template <>
struct OddTab<3> {
    __device__ static inline double c(int j) { return j == 0 ? 1.0 : -0.5; }
    __device__ static inline double s(int j)
    {
        return j == 0 ? 0.0 : (j == 1 ? 0.86602540378443864676 : -0.86602540378443864676);
    }
};
template <>
struct OddTab<5> {
    __device__ static inline double c(int j)
    {
        switch (j) {
        case 0: return 1.0;
        case 1: case 4: return 0.30901699437494742410;
        default: return -0.80901699437494742410;
        }
    }
    __device__ static inline double s(int j)
    {
        switch (j) {
        case 0: return 0.0;
        case 1: return 0.95105651629515357212;
        case 2: return 0.58778525229247312917;
        case 3: return -0.58778525229247312917;
        default: return -0.95105651629515357212;
        }
    }
};
template <>
struct OddTab<7> {
    __device__ static inline double c(int j)
    {
        switch (j) {
        case 0: return 1.0;
        case 1: case 6: return 0.62348980185873353053;
        case 2: case 5: return -0.22252093395631440429;
        default: return -0.90096886790241912624;
        }
    }
    __device__ static inline double s(int j)
    {
        switch (j) {
        case 0: return 0.0;
        case 1: return 0.78183148246802980871;
        case 2: return 0.97492791218182360702;
        case 3: return 0.43388373911755812048;
        case 4: return -0.43388373911755812048;
        case 5: return -0.97492791218182360702;
        default: return -0.78183148246802980871;
        }
    }
};

template <typename T, int R>
__device__ inline void dft_odd(cpx<T>* v)
{
    constexpr int H = (R - 1) / 2;
    cpx<T> a[H], b[H];
#pragma unroll
    for (int n = 1; n <= H; ++n) {
        a[n - 1] = v[n] + v[R - n];
        b[n - 1] = mul_mi(v[n] - v[R - n]);
    }
    cpx<T> x0 = v[0];
    cpx<T> y0 = x0;
#pragma unroll
    for (int n = 0; n < H; ++n) y0 = y0 + a[n];
    cpx<T> y[R];
    y[0] = y0;
#pragma unroll
    for (int k = 1; k < R; ++k) {
        cpx<T> acc = x0;
#pragma unroll
        for (int n = 1; n <= H; ++n) {
            const int j = (n * k) % R;
            acc = acc + scale(a[n - 1], (T)OddTab<R>::c(j)) + scale(b[n - 1], (T)OddTab<R>::s(j));
        }
        y[k] = acc;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = y[k];
}

template <typename T>
struct Dft<T, 3> {
    __device__ static inline void run(cpx<T>* v) { dft_odd<T, 3>(v); }
};
template <typename T>
struct Dft<T, 5> {
    __device__ static inline void run(cpx<T>* v) { dft_odd<T, 5>(v); }
};
template <typename T>
struct Dft<T, 7> {
    __device__ static inline void run(cpx<T>* v) { dft_odd<T, 7>(v); }
};

// Radix schedule of the power-of-two lengths compiled per size: stage radices
// R0, R1, R2 (NS stages), R0 >= the others so the first stage takes the most
// points per thread.
template <int P>
struct Sched;
template <> struct Sched<2> { static constexpr int NS = 1, R0 = 2, R1 = 0, R2 = 0; };
template <> struct Sched<4> { static constexpr int NS = 1, R0 = 4, R1 = 0, R2 = 0; };
template <> struct Sched<8> { static constexpr int NS = 1, R0 = 8, R1 = 0, R2 = 0; };
template <> struct Sched<16> { static constexpr int NS = 1, R0 = 16, R1 = 0, R2 = 0; };
template <> struct Sched<32> { static constexpr int NS = 2, R0 = 8, R1 = 4, R2 = 0; };
template <> struct Sched<64> { static constexpr int NS = 2, R0 = 8, R1 = 8, R2 = 0; };
template <> struct Sched<128> { static constexpr int NS = 2, R0 = 16, R1 = 8, R2 = 0; };
template <> struct Sched<256> { static constexpr int NS = 2, R0 = 16, R1 = 16, R2 = 0; };
template <> struct Sched<512> { static constexpr int NS = 3, R0 = 8, R1 = 8, R2 = 8; };
template <> struct Sched<1024> { static constexpr int NS = 3, R0 = 16, R1 = 16, R2 = 4; };
template <> struct Sched<2048> { static constexpr int NS = 3, R0 = 16, R1 = 16, R2 = 8; };
template <> struct Sched<4096> { static constexpr int NS = 3, R0 = 16, R1 = 16, R2 = 16; };
// mixed-radix lengths 32 q (q = 3, 5, 6, 7) for the line passes: a first radix of
// 16, the odd factor in the middle, an even radix last (the pruned inverse keeps
// the outputs below P / 2 by dropping the upper half of the last butterflies)
template <> struct Sched<96> { static constexpr int NS = 3, R0 = 16, R1 = 3, R2 = 2; };
template <> struct Sched<160> { static constexpr int NS = 3, R0 = 16, R1 = 5, R2 = 2; };
template <> struct Sched<192> { static constexpr int NS = 3, R0 = 16, R1 = 3, R2 = 4; };
template <> struct Sched<224> { static constexpr int NS = 3, R0 = 16, R1 = 7, R2 = 2; };

// ---------------------------------------------------------------- LDS geometry
// Line l, element e sits at (l % LI) * LSi + (l / LI) * LSo + e * ES.
struct LdsGeom {
    int nlines, LI, LSi, LSo, ES;
};

// One Stockham stage.  LINE_FAST: consecutive threads take consecutive lines
// (the lines are interleaved columns, LSi == 1); otherwise consecutive threads
// take consecutive butterflies of one line.
template <typename T, int NT, int R, bool LINE_FAST>
__device__ inline void fft_stage(cpx<T>* lds, const LdsGeom g, int P, int p, int tstride,
                                 const cpx<T>* __restrict__ tw, int tid)
{
    constexpr int MAXB = (kElemsPerThread + R - 1) / R;
    const int m = P / R;
    const int nbf = g.nlines * m;
    cpx<T> v[MAXB][R];
    int base[MAXB], iw[MAXB];
    if constexpr (LINE_FAST) {
        // column-wise stages: neighbouring threads read the same twiddle; the
        // register budget of these kernels is tight, so each butterfly loads its own
#pragma unroll
        for (int q = 0; q < MAXB; ++q) {
            const int b = tid + q * NT;
            base[q] = -1;
            if (b < nbf) {
                const int l = b % g.nlines, i = b / g.nlines;
                const int lb = (l % g.LI) * g.LSi + (l / g.LI) * g.LSo;
                base[q] = lb;
                iw[q] = i;
#pragma unroll
                for (int r = 0; r < R; ++r) v[q][r] = lds[lb + (i + r * m) * g.ES];
                const int k = i % p;
                if (k != 0) {
#pragma unroll
                    for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], tw[r * k * tstride]);
                }
                Dft<T, R>::run(v[q]);
            }
        }
    } else {
        // row-wise stages: every twiddle of the stage is loaded before the first is
        // used (one memory latency per stage); k = 0 reads tw[0] = 1, product skipped
        cpx<T> w[MAXB][R];
#pragma unroll
        for (int q = 0; q < MAXB; ++q) {
            const int b = tid + q * NT;
            const bool ok = b < nbf;
            const int i = ok ? b % m : 0, l = b / m;
            base[q] = ok ? (l % g.LI) * g.LSi + (l / g.LI) * g.LSo : -1;
            iw[q] = i;
            const int k = i % p;
#pragma unroll
            for (int r = 1; r < R; ++r) w[q][r] = tw[r * k * tstride];
        }
#pragma unroll
        for (int q = 0; q < MAXB; ++q) {
            if (base[q] >= 0) {
                const int lb = base[q], i = iw[q];
#pragma unroll
                for (int r = 0; r < R; ++r) v[q][r] = lds[lb + (i + r * m) * g.ES];
                if (i % p != 0) {
#pragma unroll
                    for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], w[q][r]);
                }
                Dft<T, R>::run(v[q]);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        if (base[q] >= 0) {
            const int i = iw[q];
            const int k = i % p;
            const int j = (i - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[base[q] + (j + r * p) * g.ES] = v[q][r];
        }
    }
    __syncthreads();
}

// As lds_fft for one power-of-two length P fixed at compile time: every radix,
// span and twiddle stride is a constant.
template <typename T, int NT, int P, bool LINE_FAST>
__device__ inline void lds_fft_fixed(cpx<T>* lds, const LdsGeom g, const cpx<T>* __restrict__ tw, int tid);

// Full forward FFT of every line in LDS.  Caller synchronises before the call;
// the call ends with a barrier.
template <typename T, int NT, bool LINE_FAST>
__device__ inline void lds_fft(cpx<T>* lds, const LdsGeom g, const FftPlan& pl,
                               const cpx<T>* __restrict__ tw, int tid)
{
    for (int s = 0; s < pl.nst; ++s) {
        const int p = pl.span[s], ts = pl.tstride[s];
        switch (pl.radix[s]) {
        case 2: fft_stage<T, NT, 2, LINE_FAST>(lds, g, pl.P, p, ts, tw, tid); break;
        case 3: fft_stage<T, NT, 3, LINE_FAST>(lds, g, pl.P, p, ts, tw, tid); break;
        case 4: fft_stage<T, NT, 4, LINE_FAST>(lds, g, pl.P, p, ts, tw, tid); break;
        case 5: fft_stage<T, NT, 5, LINE_FAST>(lds, g, pl.P, p, ts, tw, tid); break;
        case 7: fft_stage<T, NT, 7, LINE_FAST>(lds, g, pl.P, p, ts, tw, tid); break;
        case 8: fft_stage<T, NT, 8, LINE_FAST>(lds, g, pl.P, p, ts, tw, tid); break;
        default: fft_stage<T, NT, 16, LINE_FAST>(lds, g, pl.P, p, ts, tw, tid); break;
        }
    }
}

template <typename T, int NT, int P, bool LINE_FAST>
__device__ inline void lds_fft_fixed(cpx<T>* lds, const LdsGeom g, const cpx<T>* __restrict__ tw, int tid)
{
    using S = Sched<P>;
    // Stockham stage s of radix R over spans p: twiddle stride P / (p R)
    fft_stage<T, NT, S::R0, LINE_FAST>(lds, g, P, 1, P / S::R0, tw, tid);
    if constexpr (S::NS > 1)
        fft_stage<T, NT, S::R1, LINE_FAST>(lds, g, P, S::R0, P / (S::R0 * S::R1), tw, tid);
    if constexpr (S::NS > 2)
        fft_stage<T, NT, S::R2, LINE_FAST>(lds, g, P, S::R0 * S::R1, P / (S::R0 * S::R1 * S::R2), tw, tid);
}

}  // namespace mm
