// mm_fused.hpp -- the fused stage pass of small grids: x inverse of the demag
// spectrum, the LLG + RK4 stage update, and x forward of the stage output, for a
// block of rows of one plane and all three components in one work-group.
//
// A small grid evaluates its field in three to five passes (x forward, the y / z
// passes, x inverse) and then runs the stage update: four to six dependent
// launches per RK4 stage, each a few microseconds of latency.  Here the x
// inverse leaves the demag field of the block in LDS, the stage update reads it
// there (and m, its neighbours, m_n and the accumulator from global memory, as
// the plain stage kernel does), and the x forward of the block's new state
// writes the half spectrum the next stage's y / z passes take: two launches per
// stage fewer.  The input and output spectra are different buffers (other
// work-groups still read the input).  Every per-cell operation is the one the
// separate passes perform, in the same order.
#pragma once
#include "mm_adjoint_body.hpp"
#include "mm_fast.hpp"
#include "mm_llg_body.hpp"

namespace mm {

// LDS of one work-group: per component the x-inverse staging (2L half-spectrum
// rows) or the FFT lines (L lines), whichever is larger, then the cells of the
// block [3][2L][P/2] as real values.
template <int P, int L>
constexpr int fused_region() { return (L * padded_len<P>() > 2 * L * (P / 2 + 1)) ? L * padded_len<P>() : 2 * L * (P / 2 + 1); }
template <typename T, int P, int L>
constexpr int fused_lds_bytes() { return (int)(3 * fused_region<P, L>() * sizeof(cpx<T>) + 3 * 2 * L * (P / 2) * sizeof(T)); }
// Threads per work-group: the 3 L lines take 3 L (P / R0) of them; small lines leave
// that below 256, and the gather, the stage update and the transposed store then
// run with 256 (one cell update per thread at 128x128x1 instead of six in one wave),
// the extra threads joining only the barriers of the line transforms.
template <int P, int L>
constexpr int fused_threads() { return 3 * L * (P / Sched<P>::R0) > 256 ? 3 * L * (P / Sched<P>::R0) : 256; }

// Work-group `tile` takes rows 2L t .. 2L t + 2L - 1 of plane z (tile = z tpp + t,
// tpp = ceil(ny / 2L)); fused_threads<P, L>() threads, the first 3 L (P / R0) of
// them (component, line l, lane u) for the line transforms.  Spectrum element
// (c, z, kx, y) at ((c nz + z) hx + kx) sy + y.  Needs 2 nx <= P (the pruned x
// lines) and open boundaries.
//
// fused_block: the x inverse of the block's rows of S_in into `cell` ([3][2L][P/2]
// real values; `pre` runs right after the gather's loads are issued), then
// `update` (which reads the cells' field there and leaves in their place what is
// to be transformed), then, if fwd, the x forward of `cell` into S_out.
template <typename T, int P, int L, class Pre, class Update>
__device__ inline void fused_block(const void* S_in, void* S_out, int64_t sy, const void* tw, int nx, int ny,
                                   int nz, int tile, bool fwd, cpx<T>* lds, T* cell, Pre pre, Update update)
{
    constexpr int R0 = Sched<P>::R0, TL = P / R0, NL = 3 * L * TL, LP = padded_len<P>();
    constexpr int NT = fused_threads<P, L>();
    constexpr int HX = P / 2 + 1, ROWS = 2 * L, REG = fused_region<P, L>(), XH = P / 2;
    const int tpp = (ny + ROWS - 1) / ROWS;
    const int z = tile / tpp, yb = (tile - z * tpp) * ROWS;
    const int tid = (int)threadIdx.x;
    const bool act = tid < NL;          // takes part in the line transforms
    const int lt = act ? tid : 0;
    const int comp = lt / (L * TL), l = (lt / TL) % L, u = lt % TL;
    cpx<T>* reg = lds + comp * REG;
    LineTw<T, P> W;
    W.load(u, (const cpx<T>*)tw);

    // ---- x inverse: gather the block's half-spectrum rows of the three components
    // (for one bin, the rows of the block are adjacent); every load is issued
    // before the first LDS store
    {
        const cpx<T>* src = (const cpx<T>*)S_in;
        constexpr int NEL = HX * ROWS, ITER = (3 * NEL + NT - 1) / NT;
        cpx<T> gv[ITER];
#pragma unroll
        for (int it = 0; it < ITER; ++it) {
            const int idx = tid + it * NT;
            const int c = idx / NEL, rem = idx - c * NEL, kx = rem / ROWS, rr = rem - kx * ROWS;
            const int y = yb + rr;
            gv[it] = cpx<T>{(T)0, (T)0};
            if (idx < 3 * NEL && y < ny) gv[it] = src[(((int64_t)c * nz + z) * HX + kx) * sy + y];
        }
        pre();
#pragma unroll
        for (int it = 0; it < ITER; ++it) {
            const int idx = tid + it * NT;
            if (idx < 3 * NEL) {
                const int c = idx / NEL, rem = idx - c * NEL, kx = rem / ROWS, rr = rem - kx * ROWS;
                lds[c * REG + rr * HX + kx] = gv[it];
            }
        }
    }
    __syncthreads();
    {
        const cpx<T>* ra = reg + (2 * l) * HX;
        const cpx<T>* rb = reg + (2 * l + 1) * HX;
        cpx<T> v[R0];
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = u + TL * r;
            cpx<T> A = {(T)0, (T)0}, B = {(T)0, (T)0};
            if (!act) {
            } else if (k < HX) {
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
        __syncthreads();  // every staged row is read before the lines reuse the LDS
        T* cl = cell + comp * (ROWS * XH);
        auto put = [&](int e, cpx<T> val) {  // rows 2l, 2l+1 of the block: re, -im
            if (e < nx) {
                cl[(2 * l) * XH + e] = val.re;
                cl[(2 * l + 1) * XH + e] = -val.im;
            }
        };
        if constexpr (Sched<P>::NS == 1) {
            if (act) {
#pragma unroll
                for (int r = 0; r < R0; ++r) put(r, v[r]);
            }
        } else {
            finish_line<T, P, true>(reg + l * LP, u, v, W, put, act);
        }
    }
    __syncthreads();

    update(z, yb);
    __syncthreads();

    // ---- x forward of the block's new rows, half spectrum stored transposed
    if (fwd) {
        const T* cl = cell + comp * (ROWS * XH);
        const int y0 = yb + 2 * l;
        const bool ok0 = y0 < ny, ok1 = y0 + 1 < ny;
        cpx<T> v[R0];
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int e = u + TL * r;
            cpx<T> x = {(T)0, (T)0};
            if (act && 2 * r < R0 && e < nx) {  // e >= P/2 is zero padding
                if (ok0) x.re = cl[(2 * l) * XH + e];
                if (ok1) x.im = cl[(2 * l + 1) * XH + e];
            }
            v[r] = x;
        }
        Dft<T, R0>::run(v);
        cpx<T>* ln = reg + l * LP;
        if constexpr (Sched<P>::NS == 1) {
            if (act) {
#pragma unroll
                for (int r = 0; r < R0; ++r) ln[pad16(r)] = v[r];
            }
        } else {
            finish_line<T, P>(ln, u, v, W, [&](int e, cpx<T> val) { ln[pad16(e)] = val; }, act);
        }
        __syncthreads();
        cpx<T>* out = (cpx<T>*)S_out;
        for (int idx = tid; idx < 3 * HX * L; idx += NT) {
            const int c = idx / (HX * L), rem = idx - c * (HX * L), q = rem % L, kx = rem / L;
            const cpx<T>* lq = lds + c * REG + q * LP;
            const cpx<T> zk = lq[pad16(kx)];
            const cpx<T> zm = lq[pad16(kx == 0 ? 0 : P - kx)];
            // Z = FFT(a + i b): A = (Z_k + conj Z_-k)/2, B = (Z_k - conj Z_-k)/(2i)
            const cpx<T> A = scale(zk + conj(zm), (T)0.5);
            const cpx<T> B = scale(mul_mi(zk - conj(zm)), (T)0.5);
            const int y = yb + 2 * q;
            cpx<T>* o = out + (((int64_t)c * nz + z) * HX + kx) * sy + y;
            if (y < ny) o[0] = A;
            if (y + 1 < ny) o[1] = B;
        }
    }
}


// The RK4 / Euler stage of the block (mm_llg_body.hpp's llg_cell on the demag field
// the x inverse left in LDS), then the x forward of the stage output.
template <typename T, int P, int L, bool PREFETCH>
__device__ inline void body_fused_stage(const FusedStageArgs<T>& f, int tile, cpx<T>* lds, T* cell)
{
    constexpr int NT = fused_threads<P, L>();
    constexpr int ROWS = 2 * L, XH = P / 2;
    const LlgArgs<T>& a = f.g;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int tpp = (ny + ROWS - 1) / ROWS;
    const int z = tile / tpp, yb = (tile - z * tpp) * ROWS;
    const int tid = (int)threadIdx.x;
    // The stage update's inputs of a chunk of CH of the thread's NC cells: m and its
    // six neighbours (a missing neighbour is the cell itself, Eq. 7, which adds
    // m - m = 0), m_n, the accumulator, Ku.  With PREFETCH, where all of a thread's
    // cells form one chunk, these loads are issued right after the gather's, before
    // the x inverse: the barriers of the transforms wait for LDS only, so their
    // latency passes while the lines are transformed (the gather's loads, issued
    // first, are the ones its LDS stores wait for).  The registers they hold lower
    // the waves per SIMD, which only launches of few work-groups can spare.
    constexpr int NC = (ROWS * XH + NT - 1) / NT, CH = NC < 3 ? NC : 3;
    constexpr bool PRE = PREFETCH && NC <= CH;
    const int64_t N = a.N, plane = (int64_t)nx * ny;
    T mv[CH][3][7], mnv[CH][3], acv[CH][3], kan[CH];
    auto load_chunk = [&](int q0) {
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int idx = tid + (q0 + q) * NT;
            const int r = idx / nx, i = idx - r * nx, j = yb + r;
            const bool in = q0 + q < NC && idx < ROWS * nx && j < ny;
            const int64_t c = in ? z * plane + (int64_t)j * nx + i : 0;
            const int64_t dxm = in && i > 0 ? -1 : 0, dxp = in && i < nx - 1 ? 1 : 0;
            const int64_t dym = in && j > 0 ? -(int64_t)nx : 0, dyp = in && j < ny - 1 ? (int64_t)nx : 0;
            const int64_t dzm = in && z > 0 ? -plane : 0, dzp = in && z < nz - 1 ? plane : 0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const T* uu = a.ms + d * N + c;
                mv[q][d][0] = uu[0];
                mv[q][d][1] = uu[dxm];
                mv[q][d][2] = uu[dxp];
                mv[q][d][3] = uu[dym];
                mv[q][d][4] = uu[dyp];
                mv[q][d][5] = uu[dzm];
                mv[q][d][6] = uu[dzp];
                mnv[q][d] = (T)0;
                acv[q][d] = (T)0;
                if (a.stage > 1) {
                    mnv[q][d] = a.mn[d * N + c];
                    acv[q][d] = a.acc[d * N + c];
                }
            }
            kan[q] = a.ku ? a.ku[c] : a.can;
        }
    };

    // stage update of the block's cells: the demag field from LDS, the rest as the
    // plain stage kernel reads it (the x, y, z neighbours in its order); the result
    // overwrites the cell's field in LDS.  A thread takes up to NC cells and issues
    // the loads of CH of them before their updates (the updates store to global
    // memory, so the compiler would not hoist later loads above them): one memory
    // latency per CH cells instead of one per cell.
    auto update = [&](int, int) {
        for (int q0 = 0; q0 < NC; q0 += CH) {
            if (!PRE) load_chunk(q0);
#pragma unroll
            for (int q = 0; q < CH; ++q) {
                const int idx = tid + (q0 + q) * NT;
                const int r = idx / nx, i = idx - r * nx, j = yb + r;
                if (q0 + q >= NC || idx >= ROWS * nx || j >= ny) break;
                const int64_t c = z * plane + (int64_t)j * nx + i;
                T m[3], lap[3], hd[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const T mc = mv[q][d][0];
                    T s = (T)0;
                    s += mv[q][d][1] - mc;
                    s += mv[q][d][2] - mc;
                    s += mv[q][d][3] - mc;
                    s += mv[q][d][4] - mc;
                    s += mv[q][d][5] - mc;
                    s += mv[q][d][6] - mc;
                    m[d] = mc;
                    lap[d] = s;
                    hd[d] = cell[d * ROWS * XH + r * XH + i];
                }
                T res[3];
                llg_cell<T>(a, c, m, lap, hd, mnv[q], acv[q], kan[q], res, f.hout);
#pragma unroll
                for (int d = 0; d < 3; ++d) cell[d * ROWS * XH + r * XH + i] = res[d];
            }
        }
    };
    auto pre = [&] {
        if constexpr (PRE) load_chunk(0);
    };
    fused_block<T, P, L>(f.S_in, f.S_out, f.sy, f.tw, nx, ny, nz, tile, true, lds, cell, pre, update);
}

// One stage of the reverse sweep on the block (FusedAdjArgs): the apply on the
// demag field of nu the x inverse left in LDS, then the stage before's nu (after
// the renormalisation of the step before in mode 2), whose x forward goes to
// S_out.  The exchange term of the apply reads nu at the six neighbours (a
// missing one is the cell itself, as in k_adj_apply), hence nu_in and nu_out are
// different buffers.  One cell's loads at a time per thread.
template <typename T, int P, int L>
__device__ inline void body_fused_adjoint(const FusedAdjArgs<T>& f, int tile, cpx<T>* lds, T* cell)
{
    constexpr int NT = fused_threads<P, L>();
    constexpr int ROWS = 2 * L, XH = P / 2, NC = (ROWS * XH + NT - 1) / NT;
    const AdjArgs<T>& a = f.a;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int tid = (int)threadIdx.x;
    const int64_t N = a.N, plane = (int64_t)nx * ny;
    auto update = [&](int z, int yb) {
        for (int q = 0; q < NC; ++q) {
            const int idx = tid + q * NT;
            const int r = idx / nx, i = idx - r * nx, j = yb + r;
            if (idx >= ROWS * nx || j >= ny) break;
            const int64_t c = z * plane + (int64_t)j * nx + i;
            const int64_t dxm = i > 0 ? -1 : 0, dxp = i < nx - 1 ? 1 : 0;
            const int64_t dym = j > 0 ? -(int64_t)nx : 0, dyp = j < ny - 1 ? (int64_t)nx : 0;
            const int64_t dzm = z > 0 ? -plane : 0, dzp = z < nz - 1 ? plane : 0;
            // apply: out = loc + cex Lap nu + hd(nu), out_x += Ku nu_x
            T out[3], nux = (T)0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const T* u = f.nu_in + d * N + c;
                const T uc = u[0];
                T acc = (T)0;
                acc += u[dxm] - uc;
                acc += u[dxp] - uc;
                acc += u[dym] - uc;
                acc += u[dyp] - uc;
                acc += u[dzm] - uc;
                acc += u[dzp] - uc;
                T v = a.loc[d * N + c] + a.cex * acc;
                v += cell[d * ROWS * XH + r * XH + i];
                out[d] = v;
                if (d == 0) nux = uc;
            }
            out[0] += (a.ku ? a.ku[c] : a.can) * nux;
            T accl[3], l[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                accl[d] = a.accl[d * N + c] + out[d];
                l[d] = f.cmu * a.mu[d * N + c] + f.ca * out[d];
            }
            // the accumulator carries on within the step; at a step boundary it is
            // the covector of the step before, used right here
            if (f.mode != 2) {
#pragma unroll
                for (int d = 0; d < 3; ++d) a.accl[d * N + c] = accl[d];
            }
            if (f.mode == 0) continue;
            const T* ms = f.ms;
            const T* hs = f.hs;
            if (f.mode == 2) {
                // the step before: lam is the accumulator just formed
                T msr[4][3], hsr[4][3], mu[3];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    ld3(f.st[s], N, c, msr[s]);
                    ld3(f.st[4 + s], N, c, hsr[s]);
                }
                adj_renorm_cell(msr, hsr, accl, a.G, a.alpha, mu);
                st3(a.mu, N, c, mu);
                st3(f.accl_prev, N, c, mu);
#pragma unroll
                for (int d = 0; d < 3; ++d) l[d] = mu[d] / (T)6;
                ms = f.st[3];
                hs = f.st[7];
            }
            T m[3], h[3], nu[3], loc[3];
            ld3(ms, N, c, m);
            ld3(hs, N, c, h);
            adj_nu_cell(m, h, l, a.G, a.alpha, nu, loc);
            st3(f.nu_out, N, c, nu);
            st3(a.loc, N, c, loc);
            if (a.dku) a.dku[c] += (double)nu[0] * (double)m[0] * a.kfac;
#pragma unroll
            for (int d = 0; d < 3; ++d) cell[d * ROWS * XH + r * XH + i] = nu[d];
        }
    };
    fused_block<T, P, L>(f.S_in, f.S_out, f.sy, f.tw, nx, ny, nz, tile, f.mode != 0, lds, cell, [] {}, update);
}

}  // namespace mm
