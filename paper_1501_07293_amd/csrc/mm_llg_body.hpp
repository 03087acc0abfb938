// mm_llg_body.hpp -- device body of the fused local-field + LLG + RK4-stage
// update, shared by the single-grid kernel (mm_llg.hip) and the batched one
// (mm_batch.hip).  See mm_llg.hip for the equations.
#pragma once
#include "mm_common.hpp"
#include "mm_kernels.hpp"


namespace mm {

// The stage update of cell c (Eq. 2 for the field of Eqs. 3-8, then the RK4 stage
// combine, or the explicit Euler step) from its m, Laplacian, demag field, m_n,
// RK4 accumulator and reduced anisotropy constant; writes the stage output (and
// the accumulator) and returns the stage output in res.  heff: where to write the
// reduced effective field of the cell as well (nullptr: nowhere).
template <typename T>
__device__ inline void llg_cell(const LlgArgs<T>& a, int64_t c, const T (&m)[3], const T (&lap)[3],
                                const T (&hd)[3], const T (&mn)[3], const T (&ac)[3], T kan, T (&res)[3],
                                T* heff = nullptr)
{
    const int64_t N = a.N;
    const T h[3] = {a.cex * lap[0] + kan * m[0] + a.hx + hd[0], a.cex * lap[1] + a.hy + hd[1],
                    a.cex * lap[2] + a.hz + hd[2]};
    if (heff) {
#pragma unroll
        for (int d = 0; d < 3; ++d) heff[d * N + c] = h[d];
    }
    const T tx = m[1] * h[2] - m[2] * h[1];
    const T ty = m[2] * h[0] - m[0] * h[2];
    const T tz = m[0] * h[1] - m[1] * h[0];
    const T dx = m[1] * tz - m[2] * ty;
    const T dy = m[2] * tx - m[0] * tz;
    const T dz = m[0] * ty - m[1] * tx;
    const T F[3] = {-a.gdt * (tx + a.alpha * dx), -a.gdt * (ty + a.alpha * dy),
                    -a.gdt * (tz + a.alpha * dz)};
    if (a.stage == 0) {  // explicit Euler with renormalisation
        T v[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) v[d] = m[d] + F[d];
        const T inv = (T)1 / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
#pragma unroll
        for (int d = 0; d < 3; ++d) res[d] = v[d] * inv;
    } else if (a.stage == 1) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            st_later(F[d], a.acc + d * N + c);
            res[d] = m[d] + (T)0.5 * F[d];
        }
    } else if (a.stage == 2 || a.stage == 3) {
        const T w = a.stage == 2 ? (T)0.5 : (T)1;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            st_later(ac[d] + (T)2 * F[d], a.acc + d * N + c);
            res[d] = mn[d] + w * F[d];
        }
    } else {
        T v[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) v[d] = mn[d] + (ac[d] + F[d]) / (T)6;
        const T inv = (T)1 / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
#pragma unroll
        for (int d = 0; d < 3; ++d) res[d] = v[d] * inv;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) a.out[d * N + c] = res[d];
}

// The stage update of the planes k0 .. k0+KZ-1 of column pc from the gathered
// m (col, planes k0-1 .. k0+KZ), Laplacian, demag field, m_n, RK4 accumulator
// and reduced anisotropy constant.
template <typename T, int KZ>
__device__ inline void llg_update(const LlgArgs<T>& a, int64_t pc, int k0, const T (&col)[KZ + 2][3],
                                  const T (&lap)[KZ][3], const T (&hd)[KZ][3],
                                  const T (&mn)[KZ][3], const T (&ac)[KZ][3], const T (&kan)[KZ])
{
    const int64_t plane = (int64_t)a.nx * a.ny;
#pragma unroll
    for (int q = 0; q < KZ; ++q) {
        const int k = k0 + q;
        if (k >= a.nz) break;
        T res[3];
        llg_cell<T>(a, pc + (int64_t)k * plane, col[q + 1], lap[q], hd[q], mn[q], ac[q], kan[q], res);
    }
}

// One thread per (x, y) column and chunk of KZ planes.  Every load of the
// chunk (m of planes k0-1 .. k0+KZ, in-plane neighbours, H_d, Ku, m_n, acc)
// is issued before the first store, so a thread keeps many loads in flight;
// the z neighbours inside the chunk come from registers, the x and y neighbours
// from rows that neighbouring threads load anyway.  Work-group b takes chunk
// b % nzc of the column block b / nzc: the chunks of one column block are
// consecutive work-groups, so the two planes a chunk shares with its z
// neighbours are read from HBM once and found in L2 the second time.

// Thread `lane` of work-group `blk` (0 <= blk < llg_blocks, 0 <= lane < kLlgNT);
// KZ = llg_z_for(a.nz), the chunk size llg_blocks counts with.
// A neighbour missing at the boundary is the cell itself (Eq. 7): its address
// is clamped to the cell's own, which adds mc - mc = 0, so every load is issued
// unconditionally and none waits on a per-lane branch.  Along a periodic axis
// (a.per) the neighbour across the boundary is the cell at the other end.
//
// TY > 1: the work-group's columns form a tile of kLlgNT / TY columns by TY rows
// (needs nx a multiple of kLlgNT / TY and ny of TY, so the tiles cover the plane
// exactly and llg_blocks counts them), so most y neighbours a thread reads are
// cells its own work-group loads.
template <typename T, int KZ, int TY = 1>
__device__ inline void body_llg_stage(const LlgArgs<T>& a, int64_t blk, int lane)
{
    const int64_t plane = (int64_t)a.nx * a.ny;
    const int nzc = (a.nz + KZ - 1) / KZ;
    const int kc = (int)(blk % nzc);
    int64_t pc;
    if constexpr (TY == 1) {
        pc = (blk / nzc) * kLlgNT + lane;
    } else {
        constexpr int TX = kLlgNT / TY;
        const int64_t cb = blk / nzc, tiles_x = a.nx / TX;
        const int64_t ty = cb / tiles_x, tx = cb - ty * tiles_x;
        pc = (ty * TY + lane / TX) * a.nx + tx * TX + lane % TX;
    }
    if (pc >= plane) return;
    const int i = (int)(pc % a.nx), j = (int)(pc / a.nx);
    const int k0 = kc * KZ;
    const int64_t N = a.N, sy = a.nx;
    const T* __restrict__ ms = a.ms;
    const bool px = a.per & 1, py = a.per & 2, pz = a.per & 4;
    T col[KZ + 2][3];
#pragma unroll
    for (int q = 0; q < KZ + 2; ++q) {
        const int k = k0 - 1 + q;  // planes beyond the far neighbour are loaded but unused
        const int kk = k < 0 ? (pz ? a.nz - 1 : 0) : (k >= a.nz ? (pz ? 0 : a.nz - 1) : k);
#pragma unroll
        for (int d = 0; d < 3; ++d) col[q][d] = ms[d * N + pc + kk * plane];
    }
    const int64_t dxm = i > 0 ? -1 : (px ? a.nx - 1 : 0), dxp = i < a.nx - 1 ? 1 : (px ? 1 - a.nx : 0);
    const int64_t dym = j > 0 ? -sy : (py ? (a.ny - 1) * sy : 0);
    const int64_t dyp = j < a.ny - 1 ? sy : (py ? (1 - a.ny) * sy : 0);
    T lap[KZ][3], hd[KZ][3], mn[KZ][3], ac[KZ][3], kan[KZ];
#pragma unroll
    for (int q = 0; q < KZ; ++q) {
        const int k = k0 + q;
        const bool in = k < a.nz;
        const int64_t c = pc + (int64_t)(in ? k : a.nz - 1) * plane;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T* u = ms + d * N + c;
            const T mc = col[q + 1][d];
            T acc = (T)0;
            acc += u[dxm] - mc;
            acc += u[dxp] - mc;
            acc += u[dym] - mc;
            acc += u[dyp] - mc;
            if (k > 0 || pz) acc += col[q][d] - mc;
            if (k < a.nz - 1 || pz) acc += col[q + 2][d] - mc;
            lap[q][d] = acc;
            hd[q][d] = (T)0;
            mn[q][d] = (T)0;
            ac[q][d] = (T)0;
            if (a.hd) hd[q][d] = ld_last(a.hd + d * N + c);
            if (a.stage > 1) {
                mn[q][d] = ld_last(a.mn + d * N + c);
                ac[q][d] = ld_last(a.acc + d * N + c);
            }
        }
        kan[q] = a.ku ? a.ku[c] : a.can;
    }
    llg_update<T, KZ>(a, pc, k0, col, lap, hd, mn, ac, kan);
}


}  // namespace mm
