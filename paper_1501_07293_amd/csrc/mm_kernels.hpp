// mm_kernels.hpp -- argument blocks and host launchers of every kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mm_common.hpp"

namespace mm {

// Forward transform along x of pairs of real rows (the two rows of a pair are
// the real and imaginary parts of one complex FFT), zero padded from nvalid
// to P; writes the half spectrum (hx = P/2+1 entries) of every row.
struct RowR2CArgs {
    const void* in;          // real rows
    int64_t in_row_stride;   // elements
    int nrows;               // real rows
    int nvalid;              // leading nonzero entries per row (<= P)
    void* out;               // complex rows
    int rows_per_plane;      // bin k of row r goes to (r / rpp) * plane_stride + (r % rpp) * rstride
    int64_t out_plane_stride;//   + k * kstride
    int64_t rstride;
    int64_t kstride;
    int hx;
    int lines_per_wg;        // complex lines (row pairs) per work-group
    FftPlan pl;
    const void* tw;
};

// Inverse transform along x (Hermitian half spectrum -> real rows), keeping
// the first nvalid outputs of every row.
struct RowC2RArgs {
    const void* in;          // complex rows (layout as RowR2CArgs::out)
    int rows_per_plane;
    int64_t in_plane_stride;
    int64_t rstride;
    int64_t kstride;
    int hx;
    int nrows;
    void* out;               // real rows
    int64_t out_row_stride;
    int nvalid;
    int lines_per_wg;
    FftPlan pl;
    const void* tw;
};

// Complex FFT along a strided axis of a column set.  Column c of plane q sits
// at q * plane_stride + (c / cols_per_row) * row2_stride + c % cols_per_row,
// consecutive elements es apart.  Inputs beyond nin are zero; the first nout
// outputs are stored; inverse = conjugate in and out (unnormalised).
struct ColArgs {
    void* buf;
    int nplanes;
    int64_t plane_stride;
    int ncols;
    int cols_per_row;
    int64_t row2_stride;
    int64_t es;
    int nin, nout;
    int inverse;
    int tw_cols;             // columns per work-group
    FftPlan pl;
    const void* tw;
};

// Complex FFT of contiguous lines (line l at buf + l * line_stride), in place.
struct LineArgs {
    void* buf;
    int nlines;
    int64_t line_stride;
    int nin, nout;
    int inverse;
    int lines_per_wg;
    FftPlan pl;
    const void* tw;
};

// k-space pass on the last non-trivial axis: forward FFT of the three
// components of a column set, the symmetric tensor product of Eq. 14 with the
// real kernel spectrum, inverse FFT, keep the first nvalid outputs.
struct KspArgs {
    void* buf;
    int64_t comp_stride;
    int ncols;
    int cols_per_row;
    int64_t row2_stride;
    int64_t es;
    int nvalid;
    int tw_cols;
    FftPlan pl;
    const void* tw;
    const void* kern;        // real octant [ncomp][Pz/2+1][hx][Py/2+1]
    int ncomp;               // 6 (3-D) or 4 (xx, xy, yy, zz when the grid is one cell thick)
    int axis_is_z;           // 1: column c is (kx, ky) = (c / Py, c % Py), transform over kz;
                             // 0: column c is kx, transform over ky
    int hx, Py, Pz;
    int64_t k_cs, k_zs, k_xs;  // octant strides for component, kz, kx (ky is contiguous)
};

// Fused y-z pass (3-pass schedule): one work-group per x bin holds the whole
// [3][Pz][Py] plane of that bin in LDS: y forward, z forward, Eq. 14 product,
// z inverse, y inverse, in place in S = [3][nz][hx][Sy].  For 3-D grids whose
// plane fits a work-group (3 Py Pz <= kElemsPerThread x threads).
struct KyzArgs {
    void* buf;
    int64_t comp_stride;     // nz * hx * Sy
    int64_t zs;              // hx * Sy: one z plane of S
    int Sy, hx, ny, nz, Py, Pz;
    FftPlan ply, plz;
    const void* twy;
    const void* twz;
    const void* kern;        // octant [6][Pz/2+1][hx][Py/2+1]
    int64_t k_cs, k_zs, k_xs;
};
template <typename T>
hipError_t launch_kspace_yz(const KyzArgs& a, int nt, hipStream_t s);

// Compile-time specialised passes for power-of-two sizes (mm_fast.hip).  Each
// launcher returns false (and launches nothing) when no specialisation fits.
struct YLineArgs {           // contiguous lines, transformed in place
    void* buf;
    int nlines;
    int64_t line_stride;
    int nin, nout;           // inputs beyond nin are zero; first nout outputs stored
    const void* tw;
    int kx_major;            // 0: lines in memory order; > 0: this many planes, and the
                             // lines taken bin by bin (every plane of bin 0 first)
};
struct XLineArgs {           // x pass over [nplanes][ny][nx] real rows <-> [nplanes][hx][srows] bins
    const void* in;
    void* out;
    int nplanes;
    int ny, nx;
    int64_t srows;
    const void* tw;
    int lines;               // complex lines (row pairs) per work-group: 4, 8 or 16
};
struct KzArgs {              // z k-space pass, columns (kx, ky) = (c / Py, c % Py)
    void* buf;
    int64_t comp_stride;
    int ncols;               // hx * Py; also the z stride
    int nz;
    int Py;
    const void* tw;
    const void* kern;        // octant [6][Pz/2+1][hx][Py/2+1]
    int64_t k_cs, k_zs, k_xs;
};
struct KyArgs {              // y k-space pass of a one-cell-thick grid, lines (component, kx)
    void* buf;
    int64_t comp_stride;     // hx * ny
    int64_t line_stride;     // ny
    int hx, ny;
    const void* tw;
    const void* kern;        // octant [4][1][hx][Py/2+1]: xx, xy, yy, zz
    int64_t k_cs, k_xs;
};
// y k-space pass of a two-cell-thick grid (nz = 2), lines (component, plane, kx).
// The coupling along z of two planes is taken directly, not by a z transform:
// with K^(d) the 2-D spectrum of the tensor plane at z offset d (observer minus
// source), the field of plane 0 is K^(0) M0 + K^(-1) M1 and of plane 1
// K^(1) M0 + K^(0) M1.  kern holds 10 real planes [10][hx][Py/2+1], scaled by
// 1 / (Px Py): xx0, xx1, xy0, xy1, Sxz, yy0, yy1, Syz, zz0, zz1, where d = 0
// planes end in 0, d = 1 planes in 1, and the d = 1 xz and yz spectra are
// i Sxz and i Syz (odd in x resp. y: imaginary).  Parities fill in the rest:
// K^(-1) equals K^(1) except xz and yz, which change sign; xy and Syz are odd in
// ky, the others even.
struct Ky2Args {
    void* buf;
    int64_t comp_stride;     // 2 hx ny
    int64_t plane_stride;    // hx ny
    int64_t line_stride;     // ny
    int hx, ny;
    const void* tw;
    const void* kern;
    int64_t k_cs, k_xs;      // plane stride hx (Py/2+1); kx stride Py/2+1
};
constexpr int kTwoPlaneTablePlanes = 10;
template <typename T>
bool launch_yline(const YLineArgs& a, int P, int inverse, hipStream_t s);
template <typename T>
bool launch_kspace_y(const KyArgs& a, int P, hipStream_t s);
// false when P has no specialised two-plane pass
template <typename T>
bool launch_kspace_y2(const Ky2Args& a, int P, hipStream_t s);
// Last-axis k-space pass with the length P fixed at compile time (P = 128 .. 1024);
// false when P has no such pass.
template <typename T>
bool launch_kspace_fixed(const KspArgs& a, int P, hipStream_t s);
template <typename T>
bool launch_xline(const XLineArgs& a, int P, int inverse, hipStream_t s);
template <typename T>
bool launch_kspace_z(const KzArgs& a, int PZ, hipStream_t s);

template <typename T>
hipError_t launch_row_r2c(const RowR2CArgs& a, int nt, hipStream_t s);
template <typename T>
hipError_t launch_row_c2r(const RowC2RArgs& a, int nt, hipStream_t s);
template <typename T>
hipError_t launch_col_fft(const ColArgs& a, int nt, hipStream_t s);
template <typename T>
hipError_t launch_kspace(const KspArgs& a, int nt, hipStream_t s);

// ---------------------------------------------------------------- setup
// Demag tensor component `comp` (0..5 = xx,xy,xz,yy,yz,zz) in the wrapped layout
// of a [Pz][Py][Px] FP64 array; kind 0 = Eqs. 10-11, 1 = Newell's averaged tensor.
// per: periodic axes (bit 0 x, 1 y, 2 z; there P = n), summed over the image
// nearest zero and `images` further images on each side.
hipError_t launch_tensor_wrapped(double* out, int kind, int comp, int nx, int ny, int nz, int Px,
                                 int Py, int Pz, int per, int images, hipStream_t s);
// All six components on the offset table [6][2nz-1][2ny-1][2nx-1] (FP64).
hipError_t launch_tensor_table(double* out, int kind, int nx, int ny, int nz, hipStream_t s);
// tw[t] = exp(-2 pi i t / P), computed in FP64, stored in T.
template <typename T>
hipError_t launch_twiddles(void* tw, int P, hipStream_t s);
// Real part of the octant of a [Pz][Py][sx] FP64 spectrum, times scale, to T,
// stored as [Pz/2+1][hx][Py/2+1].  Records max |imag| and max |real| (as FP64
// bits) in stats[0], stats[1].
template <typename T>
hipError_t launch_octant(void* out, const void* spec, int hx, int Py, int Pz, int64_t sx,
                         double scale, unsigned long long* imag_max_bits, hipStream_t s);
// The coefficient planes of one component for the two-plane schedule (see
// Ky2Args) from its [4][Py][sx] FP64 spectrum (Pz = 4): two planes for xx, xy,
// yy, zz, one for xz, yz, times scale = 1 / (Px Py).  Records, like
// launch_octant, the largest value that must vanish and the largest kept one.
template <typename T>
hipError_t launch_table_z2(void* out, const void* spec, int comp, int hx, int Py, int64_t sx,
                           double scale, unsigned long long* stats, hipStream_t s);

// ---------------------------------------------------------------- LLG
template <typename T>
struct LlgArgs {
    const T* ms;     // stage input
    const T* mn;     // state at the start of the step
    T* acc;          // RK4 accumulator
    T* out;          // stage output (m_n itself at stage 4)
    const T* hd;     // reduced demag field or nullptr
    const T* ku;     // reduced anisotropy map 2 Ku/(mu0 Ms^2) or nullptr
    int nx, ny, nz;
    int64_t N;
    T cex;           // 2 A / (mu0 Ms^2 delta^2)
    T can;           // 2 Ku / (mu0 Ms^2) when ku == nullptr
    T hx, hy, hz;    // reduced applied field H_ext / Ms
    T alpha;
    T gdt;           // gamma Ms dt / (1 + alpha^2)
    int stage;       // 1..4 (RK4 stages), 0 (explicit Euler with renormalisation)
    int per;         // periodic axes (bit 0 x, 1 y, 2 z): the exchange stencil wraps
};
// the LLG stage gives each thread one (x, y) column and llg_z_for(nz) consecutive
// planes (one for grids one cell thick, whose threads would otherwise load a
// clamped copy of the same plane, else kLlgZ); a work-group of kLlgNT threads
// covers kLlgNT consecutive columns of one chunk, and the chunks of the same
// columns are consecutive work-groups.  Two planes per thread rather than four
// halve the registers a thread holds (twice the waves per SIMD); on the
// 512x512x16 film that measured 1.332 -> 1.323 ms per FP32 step, FP64 equal.
constexpr int kLlgZ = 2;
constexpr int kLlgNT = 256;
__host__ __device__ constexpr int llg_z_for(int nz) { return nz == 1 ? 1 : kLlgZ; }
__host__ __device__ inline int64_t llg_blocks(int nx, int ny, int nz)
{
    const int kz = llg_z_for(nz);
    return ((int64_t)nx * ny + kLlgNT - 1) / kLlgNT * ((nz + kz - 1) / kz);
}
template <typename T>
hipError_t launch_llg_stage(const LlgArgs<T>& a, hipStream_t s);

// The fused stage pass of a small grid with open boundaries (x inverse, stage
// update, x forward of the stage output; mm_fused.hpp).
template <typename T>
struct FusedStageArgs {
    LlgArgs<T> g;        // the stage (open boundaries)
    const void* S_in;    // [3][nz][hx][sy] spectrum after the y / z passes (rows < ny read)
    void* S_out;         // [3][nz][hx][sy] half spectrum of the stage output (rows < ny written)
    int64_t sy;          // row stride of both spectra
    const void* tw;      // x twiddles (Px)
    T* hout;             // the stage's reduced effective field [3][nz][ny][nx], or nullptr
};
// Rows per work-group / 2 (L in 1, 2, 4) the pass takes for a grid of `rows` x rows
// (ny nz), 0 when no fused pass of length Px exists (or 2 nx > Px).
int fused_stage_lines(int Px, int nx, int rows, size_t esz);
template <typename T>
bool launch_fused_stage(const FusedStageArgs<T>& a, int Px, int L, hipStream_t s);

// Per-term field in A/m: term 0 exch, 1 anis, 2 demag, 3 ext, 4 effective.
template <typename T>
hipError_t launch_field_term(const LlgArgs<T>& a, int term, T Ms, T* out, hipStream_t s);

// FP64 reductions over m (and hd): out[0] = sum |dm|^2 over neighbour pairs,
// out[1] = sum ku_red (my^2 + mz^2), out[2] = sum m.hd, out[3] = sum m.hext,
// out[4..6] = sum m, out[7] = count of non-finite entries, out[8] = max over the
// cells of |m x h_eff| (reduced units).  partial holds nblocks * kRedSlots doubles.
constexpr int kRedSlots = 9;
// row = {t, sums[4..6] * inv_n}: one sample of the mean-magnetisation trace
hipError_t launch_trace_row(const double* sums, double inv_n, double t, double* row, hipStream_t s);
template <typename T>
hipError_t launch_reduce(const LlgArgs<T>& a, double* partial, int nblocks, double* out,
                         hipStream_t s);
int reduce_blocks(int64_t N);

// ---------------------------------------------------------------- adjoint
template <typename T>
struct AdjArgs {
    int nx, ny, nz;
    int64_t N;
    const T *mn, *m2, *m3, *m4;  // stage inputs of the step
    const T *h1, *h2, *h3, *h4;  // their reduced effective fields
    const T* lam;                // dLoss/dm at the end of the step
    T *mu, *dF, *accl, *nu, *loc;
    const T* hd;                 // reduced demag field of nu
    const T* ku;                 // reduced anisotropy map or nullptr
    T can, cex, G, alpha;        // G = gamma Ms dt / (1 + alpha^2)
    double* dku;                 // dLoss/dKu accumulator (FP64) or nullptr
    double kfac;                 // 2 / (mu0 Ms^2)
    int per;                     // periodic axes (bit 0 x, 1 y, 2 z): the stencil wraps
};
// One fused stage of the reverse sweep on fused-stage plans (mm_fused.hpp): the
// x inverse of the spectrum of nu's demag field, the apply of that stage (a =
// loc + Lop nu, accl += a, dF = cmu mu + ca a; accl stored in modes 0 and 1),
// then by `mode`
//   0: nothing more (the sweep's last stage);
//   1: nu and loc of the stage before at (ms, hs) from that dF;
//   2: the renormalisation of the step before (lam = the new accl, its stage
//      states and fields st[0..7]; mu and accl_prev = mu stored, dF = mu / 6),
//      then nu and loc of its last stage (st[3], st[7]);
// and for modes 1 and 2 the x forward of the new nu into S_out.
template <typename T>
struct FusedAdjArgs {
    AdjArgs<T> a;         // constants and buffers (mu, accl, loc, dku, ku); a.nu, a.hd unused
    const T* nu_in;       // nu of the stage applied (read with its neighbours)
    T* nu_out;            // nu of the stage before (another buffer)
    T cmu, ca;
    int mode;
    const T *ms, *hs;     // mode 1
    const T* st[8];       // mode 2: m_n, m2, m3, m4, h1 .. h4 of the step before
    T* accl_prev;         // mode 2: its accumulator (the other buffer)
    const void* S_in;
    void* S_out;
    int64_t sy;
    const void* tw;
};
template <typename T>
bool launch_fused_adjoint(const FusedAdjArgs<T>& a, int Px, int L, hipStream_t s);
template <typename T>
hipError_t launch_adj_renorm(const AdjArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_adj_nu(const AdjArgs<T>& a, const T* ms, const T* hs, hipStream_t s);
template <typename T>
hipError_t launch_adj_apply(const AdjArgs<T>& a, T cmu, T ca, hipStream_t s);
// g_v = (g_u - u (u . g_u)) / |v| per cell, u = v / |v|: the VJP of the normalisation.
// p[0 .. n) = 0, as a kernel on stream s.
hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_normalize_vjp(const T* v, const T* gu, T* gv, int64_t N, hipStream_t s);

// ---------------------------------------------------------------- batched
// One grid of a batch (device-resident descriptor).  Offsets count elements
// of the batch arrays: moff in the [3][N] vector arrays, soff in the complex
// spectrum, koff in the real kernel octants, twx/twy/twz in the complex
// twiddle tables.
struct BatchDesc {
    int nx, ny, nz, Px, Py, Pz, hx, Sy, three_d;
    int x_lines, y_lines, k_tw;
    int64_t moff, soff, koff, oct;
    int64_t twx, twy, twz;
    double hred[3];   // H_ext / Ms
    double cex;       // 2 A / (mu0 Ms^2 delta^2) of this grid
    double can;       // 2 Ku / (mu0 Ms^2) of this grid's material
    double alpha;     // damping of this grid's material
    double gdt;       // gamma Ms dt / (1 + alpha^2) for the batch's current dt
    FftPlan fx, fy, fz;
};
template <typename T>
struct BatchPass {
    const BatchDesc* d;
    int n;
    const int* prefix;   // n + 1 tile prefix sums of this pass
    const T* in;         // x forward: the stage input m
    T* out;              // x inverse: the demag field
    cpx<T>* S;
    const T* kern;
    const cpx<T>* tw;
};
template <typename T>
struct BatchLlg {
    const T* ms;
    const T* mn;
    T* acc;
    T* out;
    const T* hd;
    int stage;
};
// A size class of a batch: the grids whose padded length for one pass is P.
template <typename T>
struct BatchClass {
    const BatchDesc* d;
    const int* members;  // class-local index -> grid index
    const int* prefix;   // nmem + 1 tile prefix sums
    int nmem;
    const T* in;         // x forward: the stage input m
    T* out;              // x inverse: the demag field
    cpx<T>* S;
    const T* kern;
    const cpx<T>* tw;
};
// kind: 0 x forward, 1 y (inverse flag), 2 z k-space, 3 y k-space (one cell
// thick), 4 x inverse, 5 two-plane y k-space (two cells thick).  (LLG classes,
// grouped by planes per thread, launch through launch_batch_llg.)  Returns false when no specialised kernel has length P.
template <typename T>
bool launch_batch_class(int kind, int P, const BatchClass<T>& c, int tiles, int inverse, hipStream_t s);
// First radix of the specialised schedule of length P (0 if none), and the
// lines per work-group of the specialised y k-space pass.
int fast_first_radix(int P);
// Columns per work-group of the register z k-space pass (3 components each):
// 64 in FP32; 16 in FP64, where a 32-point double line per thread leaves one
// wave per SIMD, so smaller work-groups (less LDS each) put more waves on a CU
// (measured on the 512x512x16 film: 281 -> 253 us per launch).
constexpr int kspace_z_cols_for(size_t esz) { return esz == 8 ? 16 : 64; }
template <typename T>
constexpr int kspace_z_cols() { return kspace_z_cols_for(sizeof(T)); }
// Columns per work-group of the split-line z pass (FP64, two lanes per line):
// 32 (512-byte segments per plane; measured on the 512x512x16 film: 16 columns
// 255 us, 32 columns 240 us, 64 columns 325 us per launch)
constexpr int kspace_z_split_cols() { return 32; }
int fast_ky_lines(int P);
// kx bins per work-group of the two-plane y k-space pass (0 if P has none)
int fast_ky2_lines(int P);

// which: 0 x forward, 1 y (inverse flag), 2 k-space, 3 x inverse.
template <typename T>
hipError_t launch_batch_pass(int which, const BatchPass<T>& p, int total_tiles, int inverse, hipStream_t s);
// The LLG stage over the grids of class c, whose members all take kz =
// llg_z_for(nz) planes per thread; tiles = the class's llg_blocks total.
template <typename T>
hipError_t launch_batch_llg(int kz, const BatchClass<T>& c, int tiles, const BatchLlg<T>& g, hipStream_t s);

// m <- m / |m| per cell; counts zero-norm or non-finite cells into *bad.
template <typename T>
hipError_t launch_normalize(T* m, int64_t N, unsigned int* bad, hipStream_t s);

}  // namespace mm
