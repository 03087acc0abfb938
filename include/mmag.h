/*
 * mmag.h -- C ABI of the MI355X (gfx950) finite-difference micromagnetic step.
 *
 * The library evaluates the effective field of Zhu, arXiv:1501.07293, Sec. 2
 * (Eq. 3: exchange + uniaxial anisotropy + demagnetisation + applied field)
 * on an nx x ny x nz grid of cubic cells and advances the magnetisation with
 * the Landau-Lifshitz form of the LLG equation (Eq. 2) and classical RK4,
 * renormalising every cell once per step.
 *   - exchange: six-neighbour Laplacian, Neumann boundary (Sec. 2.1, Eqs. 5-7)
 *   - anisotropy: easy axis x, field on the x component (Sec. 2.2, Eq. 8)
 *   - demag: convolution of M with the tensor of Eqs. 10-11 (Sec. 2.3,
 *     Eqs. 12-13), evaluated by a zero-padded 3-D FFT (Eq. 14, Fig. 1)
 *
 * Conventions (every entry point):
 *   - Returns mm_status; 0 is success.  Nothing throws across the ABI.  On
 *     error, mm_last_error() returns a thread-local message.
 *   - Units are SI: lengths m, fields A/m, Ms A/m, A J/m, Ku J/m^3, gamma
 *     m/(A s) multiplying H in A/m, time s, energy J.
 *   - Arrays of vectors are planar [3][nz][ny][nx], x fastest, in the working
 *     precision of the handle (float for MM_F32, double for MM_F64).  Scalar
 *     maps are [nz][ny][nx].
 *   - `on_device` = 1: the pointer is device memory on the handle's device;
 *     0: host memory.  The caller owns every buffer it passes; the library
 *     keeps no pointer to caller arrays after a call returns.
 *   - Work is enqueued on the handle's stream (a hipStream_t passed as void*;
 *     NULL = the null stream).  mm_step returns without waiting; calls that
 *     return host values (get_energy, get_mean_m, get_* to host) synchronise.
 *   - A handle is not thread-safe; separate handles are independent.
 */
#ifndef MMAG_H
#define MMAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MM_OK = 0,
    MM_EINVAL = -1,      /* invalid argument (dims, material, dt, NaN / zero m, small workspace) */
    MM_ENOMEM = -2,      /* device allocation failed */
    MM_EHIP = -3,        /* HIP runtime error; mm_last_error() has the HIP text */
    MM_ESTATE = -4,      /* call order (e.g. step before set_m) */
    MM_ENOTSUP = -5,     /* valid but unsupported size / option */
    MM_ENONFINITE = -6   /* a reduction met NaN or Inf in m */
} mm_status;

typedef enum { MM_F32 = 0, MM_F64 = 1 } mm_precision;

typedef enum {
    MM_H_EXCH = 0,   /* Eqs. 5-7 */
    MM_H_ANIS = 1,   /* Eq. 8 */
    MM_H_DEMAG = 2,  /* Eqs. 12-14 */
    MM_H_EXT = 3,    /* applied field */
    MM_H_EFF = 4     /* Eq. 3, the sum */
} mm_term;

/* Option flags. */
#define MM_NO_DEMAG 0x1u   /* drop the demag term (exchange, anisotropy, applied only) */
#define MM_USE_GRAPH 0x2u  /* mm_step replays a captured hipGraph of whole RK4 steps */
#define MM_GENERIC_FFT 0x4u /* use the runtime-radix FFT passes even where a size-specialised
                               pass exists (both give the same result up to rounding) */
#define MM_POW2_PAD 0x10u  /* automatic padded sizes are the next power of two >= 2n-1 (instead of
                               the smallest 7-smooth size), so the size-specialised passes apply;
                               a batch created with it runs those passes, one launch per padded
                               size per pass */
/* Automatic padded sizes are the smallest length >= 2n-1 that has a
 * size-specialised pass: along x and y the powers of two and 96, 160, 192, 224
 * (mixed-radix 32 q, q = 3, 5, 6, 7), along z the powers of two.  Any such
 * length gives the same linear convolution (it is >= 2n-1); for grids of 33 to
 * 112 cells it pads less than MM_POW2_PAD (e.g. 33 -> 96 instead of 128), and a
 * batch created with it runs the size-class passes.  Excludes MM_POW2_PAD. */
#define MM_FAST_PAD 0x1000u
#define MM_NEWELL 0x20u    /* demag with Newell's cell-averaged tensor (Newell, Williams and Dunlop,
                               J. Geophys. Res. 98, 9551, 1993; cited in Sec. 2.3) instead of the
                               point-field tensor of Eqs. 10-11; see mm_demag_tensor_newell */
#define MM_PER_GRID_MATERIAL 0x40u /* mm_batch_create: `mat` points to n materials, one per grid
                                      (otherwise one material for every grid) */
/* Periodic boundary along an axis (the alternative to zero padding named in
 * Sec. 2.3): that axis is not padded (its FFT length is n, which must be
 * 7-smooth, and a power of two for the size-specialised passes), the exchange
 * stencil wraps around (the first and last cells are neighbours), and the
 * demag sum takes every source at the image nearest the observer plus
 * mm_options.images further images on each side (with an even period the two
 * images at distance n/2 count one half each, so the tensor keeps its
 * parities and its spectrum stays real).  The paper defines no periodic
 * tensor; this image window is the reading taken.  A periodic x or y axis needs
 * at least 2 cells (MM_ENOTSUP otherwise).  Setup cost grows as
 * (2 images + 1)^(periodic axes).  Single-grid handles (including the
 * adjoint): mm_batch_create returns MM_ENOTSUP for periodic grids. */
/* 3-D grids whose [3][Pz][Py] spectrum plane of one x bin fits a work-group
 * (3 Py Pz <= 16 x threads, e.g. 256x64x4): run the y forward, z k-space and y
 * inverse passes as one fused pass (three passes per field evaluation instead of
 * five).  Off by default: with one work-group per x bin it measured slower than
 * the five passes on such films (256x64x4 FP32: 0.17 against 0.10 ms per RK4
 * step); MM_AUTOTUNE times both schedules where the fused one applies. */
#define MM_FUSED_YZ 0x400u
/* Grids whose padded volume of the three components fits one work-group's LDS
 * (3 px py pz <= 16 x threads, e.g. 32x8x1 at 64x16 points): one work-group runs
 * the whole demag evaluation (every x, y and z transform of the padded volume,
 * the Eq. 14 product and the inverse) in a single launch instead of three or
 * five.  Off by default: it measured slower than the multi-pass schedules (the
 * 32x8x1 strip, FP32: 116 against 61 us per RK4 step), since one work-group runs
 * every stage back to back.  Ignored where the volume does not fit or MM_NO_DEMAG
 * is set; takes precedence over MM_FUSED_YZ; MM_AUTOTUNE times it where it
 * applies. */
#define MM_ONE_WG 0x800u
/* Grids of up to 2^20 cells with open boundaries and a size-specialised x pass
 * run each RK4 stage as the y / z passes (the y k-space pass of one-cell-thick
 * grids, the two-plane pass of grids two cells thick, else y forward, z k-space,
 * y inverse) and one fused pass doing the x inverse, the stage update and the x
 * forward of the stage output on a block of rows of one plane (the demag field
 * never leaves LDS): two launches per stage fewer.  Small grids are bound by the
 * latency of dependent launches, not by bandwidth (the 128x128x1 film: four
 * launches of 4-7 us per stage).  Results equal the separate passes to rounding.
 * This flag keeps the separate passes. */
#define MM_SPLIT_STAGE 0x2000u
#define MM_PERIODIC_X 0x80u
#define MM_PERIODIC_Y 0x100u
#define MM_PERIODIC_Z 0x200u
#define MM_AUTOTUNE 0x8u    /* mm_create times the candidate schedules of this grid (padded sizes
                               7-smooth vs power of two, specialised vs runtime-radix passes,
                               256 vs 512 threads, x lines per work-group, fused y-z pass, one
                               work-group) and keeps the fastest.  The candidates run in the
                               caller's workspace when it holds every one of them (the size
                               mm_workspace_query returns with this flag), else in one temporary
                               workspace that mm_create allocates and frees; the kernel spectrum
                               is built once per candidate padded size.  Results are cached per
                               process and, if MMAG_TUNE_CACHE names a file, across processes,
                               keyed by the GPU (architecture, name, compute units), the grid
                               and the options.  mm_batch_create times the batch layouts
                               (7-smooth padding, power-of-two padding with runtime-radix passes,
                               power-of-two padding with size-class passes) on one field
                               evaluation each and keeps the fastest (mm_batch_get_info reports
                               it); MM_POW2_PAD and MM_GENERIC_FFT are then ignored.  Explicit
                               px/py/pz/threads are ignored under this flag. */

typedef struct {
    int32_t nx, ny, nz; /* cells along x, y, z; each >= 1 */
    double cell;        /* cubic cell edge delta, m, > 0 */
} mm_grid;

typedef struct {
    double Ms;    /* saturation magnetisation, A/m, > 0 */
    double A;     /* exchange constant, J/m, >= 0 */
    double Ku;    /* uniaxial anisotropy along x, J/m^3 (uniform; see mm_set_ku_map) */
    double alpha; /* damping, >= 0 */
    double gamma; /* gyromagnetic ratio, m/(A s), > 0 (e.g. 2.211e5) */
} mm_material;

typedef struct {
    int32_t prec;        /* mm_precision */
    int32_t px, py, pz;  /* padded FFT sizes; 0 = automatic (2n if 7-smooth, else the
                            smallest 7-smooth size >= 2n-1; pz = 1 when nz = 1).  An explicit
                            size must be 7-smooth and >= 2n-1 (pz = 1 only when nz = 1).
                            A periodic axis takes n (0 or n accepted). */
    uint32_t flags;      /* MM_NO_DEMAG | MM_USE_GRAPH | MM_GENERIC_FFT | MM_AUTOTUNE | MM_POW2_PAD | MM_FAST_PAD |
                            MM_NEWELL | MM_PER_GRID_MATERIAL (batches) | MM_PERIODIC_X/Y/Z |
                            MM_FUSED_YZ | MM_ONE_WG | MM_SPLIT_STAGE (single-grid handles) */
    int32_t threads;     /* threads per FFT work-group: 0 = automatic, 256 or 512 */
    int32_t x_lines;     /* row pairs per work-group of the size-specialised x passes:
                            0 = automatic (FP32 8 forward, 4 inverse; FP64 4 and 4 at
                            1024 points), 4, 8 or 16 (both passes;
                            16 only where its LDS tile and
                            work-group fit; otherwise that pass runs the runtime-radix body) */
    int32_t images;      /* periodic axes: images on each side beyond the nearest, 0..64 */
} mm_options;

typedef struct {
    int32_t px, py, pz;  /* padded sizes */
    int32_t hx;          /* px/2 + 1 stored half-spectrum bins along x */
    int32_t ncomp;       /* 6 kernel spectra, or 4 (xx, xy, yy, zz) when nz == 1 */
    int32_t threads;     /* FFT work-group size in use */
    int64_t spectrum_elems; /* elements of the kernel spectrum: the octant, ncomp*(pz/2+1)*hx*(py/2+1),
                               or with two_plane the 10*hx*(py/2+1) coefficient planes */
    int32_t passes;      /* FFT passes per field evaluation (1 with MM_ONE_WG in use, 3 for
                            nz == 1, the two-plane schedule or the fused y-z pass, else 5) */
    double kernel_imag_ratio; /* max |Im| / max |Re| of the FP64 kernel spectrum (should be ~1e-16) */
    int32_t generic_fft; /* 1 when the runtime-radix passes are forced */
    int32_t tuned;       /* 1 when the schedule came from the autotuner */
    int32_t candidates;  /* schedules the autotuner timed (0 if cached or not tuned) */
    double tuned_demag_ms; /* the chosen schedule's time per demag evaluation, ms (0 if not tuned) */
    int32_t x_lines;     /* row pairs per work-group of the specialised x forward pass */
    int32_t x_lines_inv; /* ... and of the specialised x inverse pass */
    int32_t two_plane;   /* 1: the two-plane schedule of a grid two cells thick (nz == 2, open z,
                            specialised y passes): the x passes and one y k-space pass that
                            couples the two planes directly through the tensor planes at z
                            offsets -1, 0, 1 (Eqs. 12-13 split along z, Eq. 14 in x and y); no
                            z transform and no py-long spectrum in HBM.  The kernel spectrum is
                            then 10 real planes [10][hx][py/2+1] scaled by 1/(px py): xx0, xx1,
                            xy0, xy1, sxz, yy0, yy1, syz, zz0, zz1 (suffix 0: z offset 0; 1: z
                            offset +1, the observer above the source; at offset +1 the xz and
                            yz spectra are i sxz and i syz) */
    int32_t fused_stage; /* 1: RK4 stages run the fused stage pass (see MM_SPLIT_STAGE) */
} mm_plan_info;

typedef struct mm_sim mm_sim;

/* Bytes of device workspace mm_create needs for this grid and options. */
mm_status mm_workspace_query(const mm_grid* grid, const mm_options* opt, size_t* bytes);

/* Creates a handle.  d_workspace: caller-owned device memory of ws_bytes
 * (>= mm_workspace_query), 256-byte aligned; NULL lets the library allocate
 * (freed by mm_destroy).  Builds the demag tensor (Eqs. 10-11, FP64, origin
 * included) and its FP64 3-D FFT (the kernel spectrum, stored as a real
 * octant in the working precision) on `stream`.  *out is NULL on failure. */
mm_status mm_create(const mm_grid* grid, const mm_material* mat, const mm_options* opt,
                    void* d_workspace, size_t ws_bytes, void* stream, mm_sim** out);

/* Destroys a handle (NULL is accepted).  Waits for its stream. */
mm_status mm_destroy(mm_sim* sim);

mm_status mm_set_stream(mm_sim* sim, void* stream);

/* Sets m from [3][nz][ny][nx] values; each cell is normalised to unit length.
 * A zero-length or non-finite cell gives MM_EINVAL (and leaves no valid m). */
mm_status mm_set_m(mm_sim* sim, const void* m, int on_device);
mm_status mm_get_m(mm_sim* sim, void* out, int on_device);

/* Applied field, A/m, constant until changed. */
mm_status mm_set_hext(mm_sim* sim, const double h[3]);
mm_status mm_set_alpha(mm_sim* sim, double alpha);

/* Per-cell Ku map [nz][ny][nx] in J/m^3 (working precision); NULL restores the
 * uniform material Ku. */
mm_status mm_set_ku_map(mm_sim* sim, const void* ku, int on_device);

/* Advances nsteps classical RK4 steps of dt seconds (dt > 0, finite).  Each step
 * evaluates the effective field four times and renormalises m once.
 * Asynchronous on the handle's stream.  MM_ESTATE before mm_set_m. */
mm_status mm_step(mm_sim* sim, int64_t nsteps, double dt);

/* The paper's own integrator (its appendix script): nsteps explicit Euler steps,
 * m <- (m + dt f(m)) / |m + dt f(m)| per cell, one field evaluation per step.
 * Asynchronous on the handle's stream. */
mm_status mm_step_euler(mm_sim* sim, int64_t nsteps, double dt);

/* Integrators for mm_run_schedule. */
typedef enum { MM_RK4 = 0, MM_EULER = 1 } mm_method;

/* One piece of a time-dependent protocol: the switching experiment of Sec. 3
 * (standard problem #4, field 1) and its appendix script saturate along
 * (1,1,1), ramp that field down, relax at high damping, then reverse at low
 * damping while sampling the mean magnetisation.  During step n of the piece
 * (0 <= n < steps) the applied field is h0 + (h1 - h0) n / steps, A/m
 * (h1 = h0 holds it constant); alpha is the damping of the whole piece. */
typedef struct {
    int64_t steps;  /* >= 0 */
    double h0[3];   /* finite */
    double h1[3];   /* finite */
    double alpha;   /* finite, >= 0 */
} mm_segment;

/* Runs the pieces in order, `method` steps of dt (RK4 as mm_step, or explicit
 * Euler as mm_step_euler).  After every `every`-th step (every >= 1, counted
 * from the start of the call over all pieces) one trace row of 4 doubles
 * {t, <m_x>, <m_y>, <m_z>} is written: t is the time since the call's start in
 * seconds, <m> the FP64 mean of the unit vectors.  `trace` is DEVICE memory
 * of trace_cap rows (row-major), written by the library on the handle's
 * stream; it may be NULL when no row is due.  The number of rows due,
 * floor(sum(steps) / every), must fit trace_cap: otherwise MM_EINVAL before
 * any step.  The pieces are enqueued without host synchronisation between
 * them; the call returns after the stream has drained, with *rows (may be
 * NULL) = rows written.  Afterwards the handle's applied field is that of the
 * last step run and its damping that of the last piece.  Constant-field RK4
 * pieces use the graph replay of MM_USE_GRAPH when the handle has it. */
mm_status mm_run_schedule(mm_sim* sim, const mm_segment* segs, int32_t nseg, int32_t method,
                          double dt, int64_t every, double* trace, int64_t trace_cap,
                          int64_t* rows);

/* One term of the effective field at the current m, A/m, [3][nz][ny][nx]. */
mm_status mm_get_field(mm_sim* sim, int32_t term, void* out, int on_device);

/* Energies of Eq. 1 at the current m, J: {exchange, anisotropy, demag, Zeeman,
 * total}; FP64 reductions.  MM_ENONFINITE if m holds NaN or Inf. */
mm_status mm_get_energy(mm_sim* sim, double out[5]);

/* Mean of m over the cells (FP64). */
mm_status mm_get_mean_m(mm_sim* sim, double out[3]);

/* The largest torque over the cells, max |m x H_eff| in A/m (m the unit vector,
 * H_eff the full effective field of Eq. 3 at the current m), reduced in FP64
 * from the working-precision state in the same pass as the energies.  It
 * vanishes exactly at an equilibrium of Eq. 2 and serves as a relaxation
 * criterion (e.g. max |m x H_eff| / Ms < 1e-5).  Synchronises.  MM_ENONFINITE
 * if m holds NaN or Inf. */
mm_status mm_get_max_torque(mm_sim* sim, double* out);

mm_status mm_get_plan(mm_sim* sim, mm_plan_info* out);

/* Kernel-spectrum octant [ncomp][pz/2+1][hx][py/2+1] (ky fastest), working
 * precision, already scaled by 1/(px py pz) (the normalisation of the inverse
 * FFT).  Component order xx, xy, xz, yy, yz, zz, or xx, xy, yy, zz when ncomp == 4.
 * With the two-plane schedule (mm_plan_info.two_plane) the 10 coefficient
 * planes described there instead. */
mm_status mm_get_kernel_spectrum(mm_sim* sim, void* out, int on_device);

/* Demag tensor of Eqs. 10-11 over every offset |I|<nx, |J|<ny, |K|<nz, FP64,
 * dimensionless: d_out[6][2nz-1][2ny-1][2nx-1] (device memory, caller-owned),
 * component order xx, xy, xz, yy, yz, zz, offset index (K+nz-1, J+ny-1, I+nx-1). */
mm_status mm_demag_tensor(int32_t nx, int32_t ny, int32_t nz, double* d_out, void* stream);

/* Newell's cell-averaged tensor (the alternative Sec. 2.3 cites) in the same sign
 * convention (K = -N, K(0) = -I/3) and the same layout as mm_demag_tensor.  FP64:
 * the exact 27-point second differences of Newell's f and g within a distance
 * of 8 cells, beyond it the point field of Eqs. 10-11 averaged over the
 * observer's cell by 4-point Gauss-Legendre quadrature per axis; relative error
 * ~2e-10 of the largest entry at any offset. */
mm_status mm_demag_tensor_newell(int32_t nx, int32_t ny, int32_t nz, double* d_out, void* stream);

/* ---- batched form --------------------------------------------------------
 * n independent grids of uneven sizes (each its own padding and applied
 * field, one material for all or, with MM_PER_GRID_MATERIAL, one per grid; one
 * precision) advanced together: every pass of a field
 * evaluation and every LLG stage is one kernel launch over all grids, and with
 * MM_USE_GRAPH mm_batch_step replays captured RK4 steps.  m arrays are the
 * concatenation, grid by grid, of [3][nz][ny][nx] blocks.  Sizes must fit the
 * 256-thread FFT work-group (padded lengths up to 4096, last axis up to 1365).
 * hext: [n][3] applied fields in A/m (NULL = zero).  Ownership, streams and
 * errors as for the single-grid handle. */
typedef struct mm_batch mm_batch;
mm_status mm_batch_workspace_query(int32_t n, const mm_grid* grids, const mm_options* opt,
                                   size_t* bytes);
mm_status mm_batch_create(int32_t n, const mm_grid* grids, const mm_material* mat,
                          const double* hext, const mm_options* opt, void* d_workspace,
                          size_t ws_bytes, void* stream, mm_batch** out);
mm_status mm_batch_destroy(mm_batch* b);
mm_status mm_batch_set_stream(mm_batch* b, void* stream);
mm_status mm_batch_set_m(mm_batch* b, const void* m, int on_device);
mm_status mm_batch_get_m(mm_batch* b, void* out, int on_device);
mm_status mm_batch_step(mm_batch* b, int64_t nsteps, double dt);
/* One term of every grid's effective field (Eq. 3; terms as mm_get_field) at
 * the current m, A/m, laid out grid by grid like m.  The demag term runs the
 * batch's own passes (the layout mm_batch_step uses). */
mm_status mm_batch_get_field(mm_batch* b, int32_t term, void* out, int on_device);
mm_status mm_batch_cells(mm_batch* b, int64_t* total_cells);

/* The layout a batch runs on (for MM_AUTOTUNE, the one that won). */
typedef struct {
    int64_t cells;           /* cells over all grids */
    int32_t n;               /* grids */
    int32_t pow2_pad;        /* 1: padded sizes are powers of two; 0: 7-smooth */
    int32_t size_classes;    /* 1: the size-class passes (one launch per padded length per
                                pass); 0: the runtime-radix passes (one launch per pass) */
    int32_t tuned;           /* 1: chosen by MM_AUTOTUNE */
    int32_t tune_candidates; /* layouts timed */
    int32_t fast_pad;        /* 1: padded sizes from the specialised set (MM_FAST_PAD) */
    double tuned_ms;         /* the winner's time of one field evaluation of every grid, ms */
    size_t workspace_bytes;  /* device bytes the layout uses */
} mm_batch_info;
mm_status mm_batch_get_info(mm_batch* b, mm_batch_info* out);
/* The plan of grid i (0 <= i < n) as the batch runs it: padded sizes (which the
 * size-class layouts may raise above the grid's own automatic ones), stored x
 * bins, kernel-spectrum size, passes and the two-plane schedule.  The tuner
 * fields are 0.  MM_EINVAL for a NULL argument or i out of range. */
mm_status mm_batch_get_grid_plan(mm_batch* b, int32_t i, mm_plan_info* out);

/* ---- differentiation (adjoint) ------------------------------------------
 * Gradients of a loss of the final state of an RK4 rollout with respect to the
 * per-cell anisotropy map (set by mm_set_ku_map) and the initial state, by the
 * discrete adjoint of the RK4 step with renormalisation (hand-written
 * vector-Jacobian products; the transposed demag convolution is the demag
 * convolution itself, the tensor being symmetric and even).
 *
 * mm_rollout: nsteps RK4 steps of dt from the current m, like mm_step, and
 *   stores the state at the start of every segment of ckpt_every steps into
 *   d_ckpt (device, caller-owned, ceil(nsteps/ckpt_every) x [3][nz][ny][nx]).
 *   The steps replay captured hipGraphs (whatever MM_USE_GRAPH says).
 * mm_adjoint_workspace_query: device bytes mm_backward needs for ckpt_every:
 *   8 state-sized vectors per step of a segment (its stage states and stage
 *   fields, stored while the segment is recomputed from its checkpoint), 7
 *   working vectors and N doubles, so memory grows with ckpt_every (about
 *   8 ckpt_every x 12 N bytes in FP32) and compute does not.
 * mm_backward: given d_lam_final = dLoss/dm at the final state ([3][nz][ny][nx],
 *   working precision, device), recomputes each segment from its checkpoint once
 *   and runs the reverse sweep over it (each segment one replay of a captured
 *   hipGraph, kept on the handle for the next call with the same segment length,
 *   dt, workspace, damping, applied field and Ku-map presence); writes d_dku =
 *   dLoss/dKu per cell (FP64, device, N values; loss units per J/m^3) and, if
 *   d_dm0 is not NULL, dLoss/dm0 with respect to the normalised initial state
 *   ([3][nz][ny][nx], working precision, device; mm_normalize_backward carries it
 *   to the raw state given to mm_set_m).  nsteps, dt and ckpt_every must be those
 *   of the rollout, with Ku map, alpha and H_ext unchanged.  The handle's m is
 *   not touched.  Uses the caller's adjoint workspace. */
mm_status mm_rollout(mm_sim* sim, int64_t nsteps, double dt, int64_t ckpt_every, void* d_ckpt);
mm_status mm_adjoint_workspace_query(mm_sim* sim, int64_t ckpt_every, size_t* bytes);
mm_status mm_backward(mm_sim* sim, int64_t nsteps, double dt, int64_t ckpt_every,
                      const void* d_ckpt, const void* d_lam_final, double* d_dku, void* d_dm0,
                      void* d_adj_ws, size_t adj_ws_bytes);

/* ---- allocation-free adjoint ---------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture,
 * tight training or serving loops, harnesses that forbid hipMalloc.
 *
 * mm_backward_noalloc: mm_backward without the workspace arguments; same inputs,
 *   outputs, preconditions and results.  Its adjoint workspace is a static
 *   device array of MM_NOALLOC_SCRATCH_BYTES inside the library: each GPU that
 *   runs the library holds its own copy from module load until the process
 *   ends, and its address on a device is taken once, when the first handle is
 *   created there.  Returns MM_EINVAL when mm_adjoint_workspace_query(ckpt_every)
 *   exceeds MM_NOALLOC_SCRATCH_BYTES (about 76 MiB for a 128x128x1 FP32 grid at
 *   ckpt_every 50), MM_EHIP if the array's address could not be found.  Calls no
 *   hipMalloc, hipFree, or allocating library routine, captures and instantiates
 *   no graph: only kernel launches and device-to-device copies on the handle's
 *   stream (every launch made directly, so it is slower than mm_backward's graph
 *   replay on small grids).  Every call on one GPU, from any handle, uses that
 *   GPU's one array, which keeps the last call's contents (the library clears
 *   what must start at zero): calls that overlap on one GPU (two streams, two
 *   threads) race and must be serialised by the caller. */
#define MM_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
mm_status mm_backward_noalloc(mm_sim* sim, int64_t nsteps, double dt, int64_t ckpt_every,
                              const void* d_ckpt, const void* d_lam_final, double* d_dku,
                              void* d_dm0);

/* The gradient through the normalisation that mm_set_m applies: given a raw
 * initial state v ([3][nz][ny][nx], device, working precision, every cell
 * nonzero) and g_u = dLoss/du for u = v/|v| (e.g. mm_backward's d_dm0), writes
 * g_v = dLoss/dv = (g_u - u (u . g_u)) / |v| per cell into d_gv (device; may
 * alias d_gu).  Asynchronous on the handle's stream. */
mm_status mm_normalize_backward(mm_sim* sim, const void* d_v, const void* d_gu, void* d_gv);

/* Per-kernel timing with HIP events on the handle's stream.  kernel: 0 x-forward,
 * 1 y-forward, 2 k-space, 3 y-inverse, 4 x-inverse, 5 LLG stage.  While a
 * profile is open mm_step launches kernels directly (no graph replay) and
 * brackets launches of that kernel with an event pair: the first of every
 * `every` launches (mm_profile_sample, default 1 = each launch; an event pair
 * costs the stream a few microseconds, so a long timed run samples).
 * mm_profile_end synchronises and returns the summed duration (ms) and the
 * number of launches timed. */
mm_status mm_profile_begin(mm_sim* sim, int32_t kernel);
mm_status mm_profile_sample(mm_sim* sim, int32_t every);
mm_status mm_profile_end(mm_sim* sim, double* total_ms, int64_t* launches);
const char* mm_kernel_name(int32_t kernel);

const char* mm_status_string(mm_status s);
const char* mm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MMAG_H */
