// mm_api.hip -- host side of the library: argument checks, plan (padded sizes,
// radix schedules, tile shapes), workspace carve-up, the one-time kernel
// spectrum build, the RK4 driver with optional hipGraph replay, field and
// energy read-out, and per-kernel event timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <array>
#include <iterator>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mmag.h"
#include "mm_demag1.hpp"
#include "mm_kernels.hpp"

using namespace mm;

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kMu0 = 4.0e-7 * kPi;

thread_local std::string g_err;

mm_status fail(mm_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(MM_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,   \
                        __LINE__);                                                            \
    } while (0)

bool smooth7(int n)
{
    if (n < 1) return false;
    for (int p : {2, 3, 5, 7})
        while (n % p == 0) n /= p;
    return n == 1;
}

int auto_pad(int n)
{
    if (smooth7(2 * n)) return 2 * n;
    int p = 2 * n - 1;
    while (!smooth7(p)) ++p;
    return p;
}

bool make_fft_plan(int P, FftPlan* pl)
{
    memset(pl, 0, sizeof *pl);
    pl->P = P;
    int rest = P, span = 1, s = 0;
    const int order[] = {16, 8, 4, 2, 3, 5, 7};
    while (rest > 1) {
        int r = 0;
        for (int c : order)
            if (rest % c == 0) {
                r = c;
                break;
            }
        if (r == 0 || s >= kMaxStages) return false;
        pl->radix[s] = r;
        pl->span[s] = span;
        pl->tstride[s] = P / (span * r);
        span *= r;
        rest /= r;
        ++s;
    }
    pl->nst = s;
    return true;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// The smallest padded length >= v that has size-specialised passes: powers of
// two, and along x and y also 96, 160, 192 and 224 (32 q, q = 3, 5, 6, 7).
int fast_pad_length(int v, bool line_axis)
{
    int q = 2;
    while (q < v) q <<= 1;
    if (line_axis)
        for (int m : {96, 160, 192, 224})
            if (m >= v && m < q) return m;
    return q;
}

struct Plan {
    int nx, ny, nz;
    int64_t N;
    int Px, Py, Pz, hx;
    int64_t sx;        // row stride (complex elements) of the working spectrum
    int64_t sxd;       // row stride of the FP64 setup spectrum
    bool three_d;
    int ncomp;
    int nt;
    int prec;
    size_t esz;        // sizeof(T)
    FftPlan fx, fy, fz;
    int x_lines, y_tw, k_tw;
    int xl, xl_inv;    // complex lines per work-group of the specialised x passes (forward, inverse)
    int64_t S_planes, S_rows;  // spectrum [3][S_planes][hx][S_rows]
    int per;                   // periodic axes: bit 0 x, bit 1 y, bit 2 z
    bool yz;                   // 3-D: the fused y-z pass replaces y forward, z k-space, y inverse
    bool wg1;                  // one work-group runs the whole demag evaluation (small grids)
    int images;                // images on each side beyond the nearest (periodic axes)
    bool zd;                   // two cells along z: the two-plane y k-space pass replaces y forward,
                               // z k-space and y inverse (the z coupling taken directly)
    bool fs;                   // small and open: the fused stage pass (x inverse, stage update,
                               // x forward) with a second spectrum buffer, two launches per RK4
                               // stage fewer
    int fs_lines;              // its row pairs per work-group
    int64_t oct_elems;         // per component (two-plane schedule: per coefficient plane)
    int kplanes;               // blocks of oct_elems in the kernel region (ncomp, or 10)
    // workspace offsets
    size_t o_mn, o_ma, o_mb, o_acc, o_hd, o_ku, o_S, o_S2, o_kern, o_twx, o_twy, o_twz;
    size_t o_twxd, o_twyd, o_twzd, o_red, o_redout, o_flags, o_setR, o_setS, total;
};

// The fused stage pass applies up to this many cells: beyond, the separate
// passes (whose x transposes move 128-byte segments) are bandwidth-bound, not
// latency-bound.
constexpr int64_t kFusedStageMaxCells = (int64_t)1 << 20;

mm_status build_plan(const mm_grid* g, const mm_options* o, Plan* p)
{
    if (!g) return fail(MM_EINVAL, "grid is NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1)
        return fail(MM_EINVAL, "grid dims must be >= 1 (got %d x %d x %d)", g->nx, g->ny, g->nz);
    if (!(g->cell > 0.0) || !std::isfinite(g->cell))
        return fail(MM_EINVAL, "cell size must be finite and > 0");
    mm_options def{};
    if (!o) o = &def;
    if (o->prec != MM_F32 && o->prec != MM_F64) return fail(MM_EINVAL, "prec must be MM_F32 or MM_F64");
    *p = Plan{};
    p->nx = g->nx;
    p->ny = g->ny;
    p->nz = g->nz;
    p->N = (int64_t)g->nx * g->ny * g->nz;
    if (p->N > (int64_t)1 << 30) return fail(MM_ENOTSUP, "grid too large (%lld cells)", (long long)p->N);
    p->prec = o->prec;
    p->esz = o->prec == MM_F32 ? 4 : 8;
    p->three_d = g->nz > 1;
    const bool pow2pad = (o->flags & MM_POW2_PAD) != 0;
    const bool fastpad = (o->flags & MM_FAST_PAD) != 0;
    if (pow2pad && fastpad) return fail(MM_EINVAL, "MM_POW2_PAD and MM_FAST_PAD exclude each other");
    p->per = ((o->flags & MM_PERIODIC_X) ? 1 : 0) | ((o->flags & MM_PERIODIC_Y) ? 2 : 0) |
             ((o->flags & MM_PERIODIC_Z) ? 4 : 0);
    if (o->images < 0 || o->images > 64) return fail(MM_EINVAL, "images must be in 0..64");
    p->images = o->images;
    auto pick = [pow2pad, fastpad](int n, int req, bool allow1, bool periodic, int* out) -> mm_status {
        if (periodic) {  // no zero padding: the FFT runs over the period itself
            // a one-cell period along x or y would need one-point transforms on those
            // axes, which no pass takes; along z the one-cell-thick schedule serves it
            if (n == 1 && !allow1) return fail(MM_ENOTSUP, "a periodic x or y axis needs at least 2 cells");
            if (req != 0 && req != n)
                return fail(MM_EINVAL, "a periodic axis of %d cells takes padded size %d (got %d)", n, n, req);
            if (!smooth7(n)) return fail(MM_ENOTSUP, "a periodic axis needs a 7-smooth length (got %d)", n);
            *out = n;
            return MM_OK;
        }
        if (req == 0) {
            if (allow1 && n == 1)
                *out = 1;
            else if (pow2pad) {
                int q = 2;
                while (q < 2 * n - 1) q <<= 1;
                *out = q;
            } else if (fastpad) {
                *out = fast_pad_length(2 * n - 1, !allow1);
            } else
                *out = auto_pad(n);
            return MM_OK;
        }
        if (req == 1 && allow1 && n == 1) {
            *out = 1;
            return MM_OK;
        }
        if (req < 2 * n - 1 || !smooth7(req))
            return fail(MM_EINVAL, "padded size %d must be 7-smooth and >= 2n-1 = %d", req, 2 * n - 1);
        *out = req;
        return MM_OK;
    };
    mm_status st;
    if ((st = pick(g->nx, o->px, false, p->per & 1, &p->Px)) != MM_OK) return st;
    if ((st = pick(g->ny, o->py, false, p->per & 2, &p->Py)) != MM_OK) return st;
    if ((st = pick(g->nz, o->pz, true, p->per & 4, &p->Pz)) != MM_OK) return st;
    if (p->Pz == 1 && g->nz != 1) return fail(MM_EINVAL, "pz = 1 needs nz = 1");
    // a padded z axis with nz == 1 still works through the 3-D schedule
    p->three_d = p->Pz > 1;
    p->hx = p->Px / 2 + 1;
    const int sx_align = p->esz == 4 ? 8 : 4;
    p->sx = (p->hx + sx_align - 1) / sx_align * sx_align;
    p->sxd = (p->hx + 3) / 4 * 4;
    p->ncomp = p->three_d ? 6 : 4;
    // FFT work-group size: each thread keeps kElemsPerThread elements; the
    // k-space pass holds 3 components of its last axis.
    const int last = p->three_d ? p->Pz : p->Py;
    int nt = o->threads;
    if (nt != 0 && nt != 256 && nt != 512) return fail(MM_EINVAL, "threads must be 0, 256 or 512");
    auto fits = [&](int t) {
        const int cap = kElemsPerThread * t;
        return p->Px <= cap && p->Py <= cap && p->Pz <= cap && 3 * last <= cap;
    };
    if (nt == 0) nt = fits(256) ? 256 : 512;
    if (!fits(nt)) return fail(MM_ENOTSUP, "padded sizes %d x %d x %d exceed the FFT work-group capacity",
                               p->Px, p->Py, p->Pz);
    p->nt = nt;
    p->yz = p->three_d && (o->flags & MM_FUSED_YZ) && 3LL * p->Py * p->Pz <= (int64_t)kElemsPerThread * nt;
    p->wg1 = (o->flags & MM_ONE_WG) && !(o->flags & MM_NO_DEMAG) &&
             3LL * p->Px * p->Py * p->Pz <= (int64_t)kElemsPerThread * nt;
    if (p->wg1) p->yz = false;
    if (o->x_lines != 0 && o->x_lines != 4 && o->x_lines != 8 && o->x_lines != 16)
        return fail(MM_EINVAL, "x_lines must be 0, 4, 8 or 16");
    // automatic: work-groups of at least 512 threads forward and 256 inverse (a line of
    // P points takes P / R0 threads), 4 to 16 lines; at P = 1024 that is 8 lines forward
    // (128-byte transposed segments) and 4 inverse (more work-groups per CU for its
    // gather).  In FP64 the forward takes the inverse's count too: 8 double lines of
    // 1024 points fill 139 KB of LDS, one work-group per CU (measured on the
    // 512x512x16 film: 96.5 -> 78.2 us per launch with 4).  An explicit value sets both.
    {
        const int r0 = fast_first_radix(p->Px);
        const int tl = r0 > 0 ? p->Px / r0 : 64;
        auto lines_for = [&](int threads) {
            const int l = threads / std::max(1, tl);
            return l >= 16 ? 16 : (l >= 8 ? 8 : 4);
        };
        p->xl = o->x_lines ? o->x_lines : lines_for(p->esz == 8 ? 256 : 512);
        p->xl_inv = o->x_lines ? o->x_lines : lines_for(256);
    }
    if (!make_fft_plan(p->Px, &p->fx) || !make_fft_plan(p->Py, &p->fy) || !make_fft_plan(p->Pz, &p->fz))
        return fail(MM_EINVAL, "padded sizes must be 7-smooth");
    const int cap = kElemsPerThread * nt, ldscap = cap + 64;
    p->x_lines = std::min(cap / p->Px, ldscap / (p->Px + 1));
    p->y_tw = std::max(1, std::min(64, cap / p->Py));
    p->k_tw = std::max(1, std::min(64, cap / (3 * last)));
    // two cells along z with an open z axis (Pz = 4) and a specialised two-plane
    // pass of length Py: no z transform and no Py-long spectrum in HBM
    p->zd = p->nz == 2 && p->Pz == 4 && !(p->per & 4) && !p->yz && !p->wg1 &&
            !(o->flags & MM_GENERIC_FFT) && fast_ky2_lines(p->Py) > 0 && p->ny <= p->Py &&
            !(p->esz == 8 && p->Py > 1024);
    // open, small (latency-bound), with the specialised passes: the fused stage pass
    // (the y / z passes of one-cell-thick and thicker grids run between its launches)
    p->fs_lines = 0;
    if (p->per == 0 && !p->yz && !p->wg1 && p->N <= kFusedStageMaxCells &&
        !(o->flags & (MM_GENERIC_FFT | MM_SPLIT_STAGE | MM_NO_DEMAG)) && 2 * p->ny <= p->Py &&
        (p->three_d || fast_ky_lines(p->Py) > 0))
        p->fs_lines = fused_stage_lines(p->Px, p->nx, p->ny * p->nz, p->esz);
    p->fs = p->fs_lines > 0;
    // spectrum [3][nz][hx][S_rows]: the y pass expands ny rows to Py in place on 3-D grids
    p->S_planes = p->nz;
    p->S_rows = (p->three_d && !p->zd) ? p->Py : p->ny;
    if (p->zd) {
        p->oct_elems = (int64_t)(p->Py / 2 + 1) * p->hx;
        p->kplanes = kTwoPlaneTablePlanes;
    } else {
        p->oct_elems = (int64_t)(p->Pz / 2 + 1) * (p->Py / 2 + 1) * p->hx;
        p->kplanes = p->ncomp;
    }
    // workspace
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    const size_t vec = 3 * (size_t)p->N * p->esz;
    p->o_mn = take(vec);
    p->o_ma = take(vec);
    p->o_mb = take(vec);
    p->o_acc = take(vec);
    p->o_hd = take(vec);
    p->o_ku = take((size_t)p->N * p->esz);
    p->o_S = take(3 * (size_t)p->S_planes * p->hx * p->S_rows * 2 * p->esz);
    p->o_S2 = p->fs ? take(3 * (size_t)p->S_planes * p->hx * p->S_rows * 2 * p->esz) : 0;
    p->o_kern = take((size_t)p->kplanes * p->oct_elems * p->esz);
    p->o_twx = take((size_t)p->Px * 2 * p->esz);
    p->o_twy = take((size_t)p->Py * 2 * p->esz);
    p->o_twz = take((size_t)p->Pz * 2 * p->esz);
    p->o_twxd = take((size_t)p->Px * 16);
    p->o_twyd = take((size_t)p->Py * 16);
    p->o_twzd = take((size_t)p->Pz * 16);
    p->o_red = take(1024 * kRedSlots * sizeof(double));
    p->o_redout = take(kRedSlots * sizeof(double));
    p->o_flags = take(64);
    p->o_setR = take((size_t)p->Px * p->Py * p->Pz * sizeof(double));
    p->o_setS = take((size_t)p->Pz * p->Py * p->sxd * 16);
    p->total = off;
    return MM_OK;
}

bool check_material(const mm_material* m)
{
    return m && m->Ms > 0 && std::isfinite(m->Ms) && m->A >= 0 && std::isfinite(m->A) &&
           std::isfinite(m->Ku) && m->alpha >= 0 && std::isfinite(m->alpha) && m->gamma > 0 &&
           std::isfinite(m->gamma);
}

}  // namespace

// ---------------------------------------------------------------- static scratch
// The adjoint workspace of mm_backward_noalloc, for callers that cannot allocate:
// a file-scope device array, so each GPU that runs the library holds its own copy
// (from module load until the process ends).  Host code never passes the array's
// name to a kernel or a copy: its address on a device comes from
// hipGetSymbolAddress, taken once per device at mm_create (scratch_address).
constexpr size_t kNoAllocScratchBytes = MM_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_addr;  // device -> its copy of `scratch`

// The address of `scratch` on device dev, which must be the current device.
mm_status scratch_address(int dev, char** out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return MM_OK;
    }
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(MM_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_addr[dev] = static_cast<char*>(ptr);
    *out = static_cast<char*>(ptr);
    return MM_OK;
}

struct mm_sim {
    Plan p;
    mm_material mat;
    double cell;
    uint32_t flags;
    char* ws;
    bool own_ws;
    hipStream_t stream;
    hipStream_t cap_stream;
    double hext[3];
    double alpha;
    bool has_m;
    bool has_ku_map;
    double imag_ratio;
    int tuned, tune_candidates;
    double tuned_ms;
    // graph
    hipGraph_t graph;
    hipGraphExec_t gexec;
    bool graph_valid;
    double graph_dt;
    int graph_chunk;
    int graph_method;
    hipGraphExec_t rem_exec = nullptr;  // fused-stage steps: the remainder of a step count
    int64_t rem_len = 0;                // past whole chunks (e.g. 2 of a 50-step segment)
    // reverse-sweep graphs: one per segment length (a full segment and the
    // shorter last one), valid while the baked-in arguments are unchanged
    struct BwdGraph {
        hipGraphExec_t exec = nullptr;
        int64_t len = 0;
        double dt = 0, alpha = 0, hext[3] = {0, 0, 0};
        bool ku_map = false;
        const char* ws = nullptr;
    };
    BwdGraph bwd[2];
    // this handle's device and that device's copy of the static adjoint scratch
    // (nullptr, with the reason in scratch_err, when its address was not found)
    int device;
    char* scratch;
    std::string scratch_err;
    // profiling: launches of kernel prof_kernel, one in prof_every bracketed by events
    int prof_kernel;
    int prof_every;
    int64_t prof_seen;
    bool prof_armed;
    std::vector<hipEvent_t> ev;
    size_t ev_used;

    template <typename T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

namespace {

enum { KX_FWD = 0, KY_FWD = 1, KSPACE = 2, KY_INV = 3, KX_INV = 4, KLLG = 5, KCOUNT = 6 };

mm_status prof_pre(mm_sim* s, int kid, hipStream_t st)
{
    if (s->prof_kernel != kid) return MM_OK;
    s->prof_armed = s->prof_seen++ % s->prof_every == 0;
    if (!s->prof_armed) return MM_OK;
    if (s->ev_used + 2 > s->ev.size()) {
        for (int q = 0; q < 256; ++q) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            s->ev.push_back(e);
        }
    }
    HIP_TRY(hipEventRecord(s->ev[s->ev_used], st));
    return MM_OK;
}

mm_status prof_post(mm_sim* s, int kid, hipStream_t st)
{
    if (s->prof_kernel != kid || !s->prof_armed) return MM_OK;
    HIP_TRY(hipEventRecord(s->ev[s->ev_used + 1], st));
    s->ev_used += 2;
    s->prof_armed = false;
    return MM_OK;
}

#define LAUNCH(kid, call)                                                     \
    do {                                                                      \
        mm_status ps_ = prof_pre(s, kid, st);                                 \
        if (ps_ != MM_OK) return ps_;                                         \
        HIP_TRY(call);                                                        \
        ps_ = prof_post(s, kid, st);                                          \
        if (ps_ != MM_OK) return ps_;                                         \
    } while (0)

// ---- the five passes of one demag evaluation.  Spectrum S = [3][nz][hx][Sy]
// (Sy = Py on 3-D grids, ny otherwise).  Each pass uses the size-specialised
// kernel when one exists (and MM_GENERIC_FFT is not set), else the generic one.
struct PassCtx {
    const Plan& p;
    void* S;
    int64_t Sy, plane;
    int nplanes;
    bool fast;
    const void *twx, *twy, *twz, *kern;
};

PassCtx pass_ctx(const mm_sim* s)
{
    const Plan& p = s->p;
    return PassCtx{p,
                   s->at<char>(p.o_S),
                   p.S_rows,
                   (int64_t)p.hx * p.S_rows,
                   3 * p.nz,
                   !(s->flags & MM_GENERIC_FFT),
                   s->at<char>(p.o_twx),
                   s->at<char>(p.o_twy),
                   s->at<char>(p.o_twz),
                   s->at<char>(p.o_kern)};
}

template <typename T>
hipError_t pass_x_forward(const PassCtx& c, const T* m, hipStream_t st)
{
    const Plan& p = c.p;
    XLineArgs xa{m, c.S, c.nplanes, p.ny, p.nx, c.Sy, c.twx, p.xl};
    if (c.fast && launch_xline<T>(xa, p.Px, 0, st)) return hipGetLastError();
    RowR2CArgs r{};
    r.in = m;
    r.in_row_stride = p.nx;
    r.nrows = c.nplanes * p.ny;
    r.nvalid = p.nx;
    r.out = c.S;
    r.rows_per_plane = p.ny;
    r.out_plane_stride = c.plane;
    r.rstride = 1;
    r.kstride = c.Sy;
    r.hx = p.hx;
    r.lines_per_wg = p.x_lines;
    r.pl = p.fx;
    r.tw = c.twx;
    return launch_row_r2c<T>(r, p.nt, st);
}

template <typename T>
hipError_t pass_y(const PassCtx& c, int inverse, hipStream_t st)
{
    const Plan& p = c.p;
    const int nin = inverse ? p.Py : p.ny, nout = inverse ? p.ny : p.Py;
    // in FP32 the inverse takes its lines bin by bin (every plane of a bin, then the next
    // bin), the order in which the k-space pass wrote them (its column blocks run
    // bin-major): 63.6 -> 58.7 us per y inverse on the 512x512x16 film, 1.357 -> 1.337 ms
    // per RK4 step; the same order for the forward pass, or a reversed k-space pass, gained
    // nothing, and in FP64 it is slower (116 -> 136 us)
    YLineArgs ya{c.S, c.nplanes * p.hx, c.Sy, nin, nout, c.twy, (inverse && p.esz == 4) ? c.nplanes : 0};
    if (c.fast && launch_yline<T>(ya, p.Py, inverse, st)) return hipGetLastError();
    ColArgs cy{};
    cy.buf = c.S;
    cy.nplanes = c.nplanes;
    cy.plane_stride = c.plane;
    cy.ncols = p.hx;
    cy.cols_per_row = 1;
    cy.row2_stride = c.Sy;
    cy.es = 1;
    cy.nin = nin;
    cy.nout = nout;
    cy.inverse = inverse;
    cy.tw_cols = p.y_tw;
    cy.pl = p.fy;
    cy.tw = c.twy;
    return launch_col_fft<T>(cy, p.nt, st);
}

template <typename T>
hipError_t pass_kspace(const PassCtx& c, hipStream_t st)
{
    const Plan& p = c.p;
    const int64_t k_xs = p.Py / 2 + 1, k_zs = (int64_t)p.hx * (p.Py / 2 + 1);
    KspArgs k{};
    k.buf = c.S;
    k.kern = c.kern;
    k.ncomp = p.ncomp;
    k.hx = p.hx;
    k.Py = p.Py;
    k.Pz = p.Pz;
    k.k_cs = p.oct_elems;
    k.k_zs = k_zs;
    k.k_xs = k_xs;
    k.tw_cols = p.k_tw;
    if (p.three_d) {
        KzArgs kz{c.S, (int64_t)p.nz * c.plane, (int)c.plane, p.nz, p.Py, c.twz, c.kern, p.oct_elems,
                  k_zs, k_xs};
        if (c.fast && launch_kspace_z<T>(kz, p.Pz, st)) return hipGetLastError();
        k.comp_stride = (int64_t)p.nz * c.plane;
        k.ncols = (int)c.plane;
        k.cols_per_row = (int)c.plane;
        k.row2_stride = 0;
        k.es = c.plane;
        k.nvalid = p.nz;
        k.pl = p.fz;
        k.tw = c.twz;
        k.axis_is_z = 1;
        if (c.fast && launch_kspace_fixed<T>(k, p.Pz, st)) return hipGetLastError();
    } else {
        KyArgs ky{c.S, c.plane, c.Sy, p.hx, p.ny, c.twy, c.kern, p.oct_elems, k_xs};
        if (c.fast && launch_kspace_y<T>(ky, p.Py, st)) return hipGetLastError();
        k.comp_stride = c.plane;
        k.ncols = p.hx;
        k.cols_per_row = 1;
        k.row2_stride = c.Sy;
        k.es = 1;
        k.nvalid = p.ny;
        k.pl = p.fy;
        k.tw = c.twy;
        k.axis_is_z = 0;
    }
    return launch_kspace<T>(k, p.nt, st);
}

template <typename T>
hipError_t pass_x_inverse(const PassCtx& c, T* h, hipStream_t st)
{
    const Plan& p = c.p;
    XLineArgs xa{c.S, h, c.nplanes, p.ny, p.nx, c.Sy, c.twx, p.xl_inv};
    if (c.fast && launch_xline<T>(xa, p.Px, 1, st)) return hipGetLastError();
    RowC2RArgs r{};
    r.in = c.S;
    r.rows_per_plane = p.ny;
    r.in_plane_stride = c.plane;
    r.rstride = 1;
    r.kstride = c.Sy;
    r.hx = p.hx;
    r.nrows = c.nplanes * p.ny;
    r.out = h;
    r.out_row_stride = p.nx;
    r.nvalid = p.nx;
    r.lines_per_wg = p.x_lines;
    r.pl = p.fx;
    r.tw = c.twx;
    return launch_row_c2r<T>(r, p.nt, st);
}

template <typename T>
hipError_t pass_kspace_yz(const PassCtx& c, hipStream_t st)
{
    const Plan& p = c.p;
    KyzArgs a{};
    a.buf = c.S;
    a.comp_stride = (int64_t)p.nz * c.plane;
    a.zs = c.plane;
    a.Sy = (int)c.Sy;
    a.hx = p.hx;
    a.ny = p.ny;
    a.nz = p.nz;
    a.Py = p.Py;
    a.Pz = p.Pz;
    a.ply = p.fy;
    a.plz = p.fz;
    a.twy = c.twy;
    a.twz = c.twz;
    a.kern = c.kern;
    a.k_cs = p.oct_elems;
    a.k_zs = (int64_t)p.hx * (p.Py / 2 + 1);
    a.k_xs = p.Py / 2 + 1;
    return launch_kspace_yz<T>(a, p.nt, st);
}

template <typename T>
hipError_t pass_kspace_y2(const PassCtx& c, hipStream_t st)
{
    const Plan& p = c.p;
    const Ky2Args a{c.S, 2 * c.plane, c.plane, c.Sy, p.hx, p.ny, c.twy, c.kern, p.oct_elems, p.Py / 2 + 1};
    if (!launch_kspace_y2<T>(a, p.Py, st)) return hipErrorInvalidValue;  // the plan checked P
    return hipGetLastError();
}

template <typename T>
hipError_t pass_demag_1wg(const PassCtx& c, const T* m, T* hd, hipStream_t st)
{
    const Plan& p = c.p;
    Demag1Args a{};
    a.m = m;
    a.hd = hd;
    a.nx = p.nx;
    a.ny = p.ny;
    a.nz = p.nz;
    a.Px = p.Px;
    a.Py = p.Py;
    a.Pz = p.Pz;
    a.hx = p.hx;
    a.plx = p.fx;
    a.ply = p.fy;
    a.plz = p.fz;
    a.twx = c.twx;
    a.twy = c.twy;
    a.twz = c.twz;
    a.kern = c.kern;
    a.ncomp = p.ncomp;
    a.k_cs = p.oct_elems;
    a.k_zs = (int64_t)p.hx * (p.Py / 2 + 1);
    a.k_xs = p.Py / 2 + 1;
    return launch_demag_1wg<T>(a, p.nt, st);
}

// Demag field (reduced, h = H/Ms) of msrc into hd: Eq. 14 with zero padding
// (none along periodic axes); five passes, three with the fused y-z pass, or one
// work-group for the whole evaluation of a small grid.
template <typename T>
mm_status demag(mm_sim* s, const T* msrc, T* hd, hipStream_t st)
{
    const PassCtx c = pass_ctx(s);
    if (c.p.wg1) {
        LAUNCH(KSPACE, pass_demag_1wg<T>(c, msrc, hd, st));
        return MM_OK;
    }
    if (c.p.yz) {
        LAUNCH(KX_FWD, pass_x_forward<T>(c, msrc, st));
        LAUNCH(KSPACE, pass_kspace_yz<T>(c, st));
        LAUNCH(KX_INV, pass_x_inverse<T>(c, hd, st));
        return MM_OK;
    }
    if (c.p.zd) {
        LAUNCH(KX_FWD, pass_x_forward<T>(c, msrc, st));
        LAUNCH(KSPACE, pass_kspace_y2<T>(c, st));
        LAUNCH(KX_INV, pass_x_inverse<T>(c, hd, st));
        return MM_OK;
    }
    LAUNCH(KX_FWD, pass_x_forward<T>(c, msrc, st));
    if (c.p.three_d) LAUNCH(KY_FWD, pass_y<T>(c, 0, st));
    LAUNCH(KSPACE, pass_kspace<T>(c, st));
    if (c.p.three_d) LAUNCH(KY_INV, pass_y<T>(c, 1, st));
    LAUNCH(KX_INV, pass_x_inverse<T>(c, hd, st));
    return MM_OK;
}

template <typename T>
LlgArgs<T> llg_args(const mm_sim* s, double dt)
{
    const Plan& p = s->p;
    const double Ms = s->mat.Ms;
    LlgArgs<T> a{};
    a.nx = p.nx;
    a.ny = p.ny;
    a.nz = p.nz;
    a.N = p.N;
    a.per = p.per;
    a.cex = (T)(2.0 * s->mat.A / (kMu0 * Ms * Ms * s->cell * s->cell));
    a.can = (T)(2.0 * s->mat.Ku / (kMu0 * Ms * Ms));
    a.hx = (T)(s->hext[0] / Ms);
    a.hy = (T)(s->hext[1] / Ms);
    a.hz = (T)(s->hext[2] / Ms);
    a.alpha = (T)s->alpha;
    a.gdt = (T)(s->mat.gamma * Ms * dt / (1.0 + s->alpha * s->alpha));
    a.ku = s->has_ku_map ? s->at<T>(p.o_ku) : nullptr;
    a.hd = (s->flags & MM_NO_DEMAG) ? nullptr : s->at<T>(p.o_hd);
    return a;
}

}  // namespace


namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// One RK4 step of dt on stream st.  Stage inputs cycle m_n -> m_a -> m_b -> m_a;
// stage 4 writes the renormalised result back into m_n.
template <typename T>
mm_status rk4_fused_steps(mm_sim* s, int64_t nsteps, double dt, bool prologue, hipStream_t st);

template <typename T>
mm_status rk4_step(mm_sim* s, double dt, hipStream_t st)
{
    const Plan& p = s->p;
    if (p.fs) return rk4_fused_steps<T>(s, 1, dt, true, st);
    T* mn = s->at<T>(p.o_mn);
    T* ma = s->at<T>(p.o_ma);
    T* mb = s->at<T>(p.o_mb);
    T* acc = s->at<T>(p.o_acc);
    T* hd = s->at<T>(p.o_hd);
    T* src[4] = {mn, ma, mb, ma};
    T* dst[4] = {ma, mb, ma, mn};
    LlgArgs<T> a = llg_args<T>(s, dt);
    a.mn = mn;
    a.acc = acc;
    for (int stg = 0; stg < 4; ++stg) {
        if (!(s->flags & MM_NO_DEMAG)) {
            mm_status r = demag<T>(s, src[stg], hd, st);
            if (r != MM_OK) return r;
        }
        a.ms = src[stg];
        a.out = dst[stg];
        a.stage = stg + 1;
        LAUNCH(KLLG, launch_llg_stage<T>(a, st));
    }
    return MM_OK;
}

// The passes between the x forward and the x inverse of one demag evaluation, in
// place on c.S: the two-plane y pass, or y forward, the k-space pass (along z, or
// along y on one-cell-thick grids) and y inverse.
template <typename T>
mm_status demag_mid(mm_sim* s, const PassCtx& c, hipStream_t st)
{
    if (c.p.zd) {
        LAUNCH(KSPACE, pass_kspace_y2<T>(c, st));
        return MM_OK;
    }
    if (c.p.three_d) LAUNCH(KY_FWD, pass_y<T>(c, 0, st));
    LAUNCH(KSPACE, pass_kspace<T>(c, st));
    if (c.p.three_d) LAUNCH(KY_INV, pass_y<T>(c, 1, st));
    return MM_OK;
}

// RK4 steps of a fused-stage plan (small, open).  The spectrum of the stage input
// sits in S: the prologue forms it for m_n (x forward); each stage then runs the
// y / z passes on it in place and the fused pass, which writes the stage output
// and its x half spectrum into the other buffer.  Four stages per step return the
// spectrum to S, holding that of the new m_n.
template <typename T>
mm_status rk4_fused_steps(mm_sim* s, int64_t nsteps, double dt, bool prologue, hipStream_t st)
{
    const Plan& p = s->p;
    T* mn = s->at<T>(p.o_mn);
    T* ma = s->at<T>(p.o_ma);
    T* mb = s->at<T>(p.o_mb);
    T* src[4] = {mn, ma, mb, ma};
    T* dst[4] = {ma, mb, ma, mn};
    PassCtx c = pass_ctx(s);
    void* bufs[2] = {s->at<char>(p.o_S), s->at<char>(p.o_S2)};
    if (prologue) LAUNCH(KX_FWD, pass_x_forward<T>(c, mn, st));
    FusedStageArgs<T> f{};
    f.g = llg_args<T>(s, dt);
    f.g.mn = mn;
    f.g.acc = s->at<T>(p.o_acc);
    f.g.hd = nullptr;
    f.sy = c.Sy;
    f.tw = c.twx;
    for (int64_t n = 0; n < nsteps; ++n) {
        for (int stg = 0; stg < 4; ++stg) {
            c.S = bufs[stg & 1];
            mm_status r = demag_mid<T>(s, c, st);
            if (r != MM_OK) return r;
            f.g.ms = src[stg];
            f.g.out = dst[stg];
            f.g.stage = stg + 1;
            f.S_in = bufs[stg & 1];
            f.S_out = bufs[(stg + 1) & 1];
            LAUNCH(KLLG, launch_fused_stage<T>(f, p.Px, p.fs_lines, st) ? hipGetLastError()
                                                                            : hipErrorInvalidValue);
        }
    }
    return MM_OK;
}

template <typename T>
mm_status build_kernel_spectrum(mm_sim* s, hipStream_t st)
{
    const Plan& p = s->p;
    HIP_TRY(launch_twiddles<T>(s->at<char>(p.o_twx), p.Px, st));
    HIP_TRY(launch_twiddles<T>(s->at<char>(p.o_twy), p.Py, st));
    HIP_TRY(launch_twiddles<T>(s->at<char>(p.o_twz), p.Pz, st));
    HIP_TRY(launch_twiddles<double>(s->at<char>(p.o_twxd), p.Px, st));
    HIP_TRY(launch_twiddles<double>(s->at<char>(p.o_twyd), p.Py, st));
    HIP_TRY(launch_twiddles<double>(s->at<char>(p.o_twzd), p.Pz, st));
    unsigned long long* stats = s->at<unsigned long long>(p.o_flags);
    HIP_TRY(hipMemsetAsync(stats, 0, 64, st));
    if (s->flags & MM_NO_DEMAG) return MM_OK;
    double* R = s->at<double>(p.o_setR);
    void* Sd = s->at<char>(p.o_setS);
    const int comps6[6] = {0, 1, 2, 3, 4, 5};
    const int comps4[4] = {0, 1, 3, 5};  // xx, xy, yy, zz: xz and yz vanish on one plane
    const int* comps = p.ncomp == 6 ? comps6 : comps4;
    const double scale = 1.0 / ((double)p.Px * p.Py * p.Pz);
    const int nt = p.nt;
    const int cap = kElemsPerThread * nt, ldscap = cap + 64;
    for (int q = 0; q < p.ncomp; ++q) {
        HIP_TRY(launch_tensor_wrapped(R, (s->flags & MM_NEWELL) ? 1 : 0, comps[q], p.nx, p.ny, p.nz,
                                      p.Px, p.Py, p.Pz, p.per, p.images, st));
        RowR2CArgs xr{};
        xr.in = R;
        xr.in_row_stride = p.Px;
        xr.nrows = p.Py * p.Pz;
        xr.nvalid = p.Px;
        xr.out = Sd;
        xr.rows_per_plane = p.Py * p.Pz;
        xr.out_plane_stride = 0;
        xr.rstride = p.sxd;
        xr.kstride = 1;
        xr.hx = p.hx;
        xr.lines_per_wg = std::min(cap / p.Px, ldscap / (p.Px + 1));
        xr.pl = p.fx;
        xr.tw = s->at<char>(p.o_twxd);
        if (xr.lines_per_wg < 1) return fail(MM_ENOTSUP, "px too large for the FP64 setup FFT");
        HIP_TRY(launch_row_r2c<double>(xr, nt, st));
        ColArgs c{};
        c.buf = Sd;
        c.nplanes = p.Pz;
        c.plane_stride = (int64_t)p.Py * p.sxd;
        c.ncols = p.hx;
        c.cols_per_row = p.hx;
        c.row2_stride = 0;
        c.es = p.sxd;
        c.nin = p.Py;
        c.nout = p.Py;
        c.inverse = 0;
        c.tw_cols = std::max(1, std::min(64, cap / p.Py));
        c.pl = p.fy;
        c.tw = s->at<char>(p.o_twyd);
        if (p.Py > cap) return fail(MM_ENOTSUP, "py too large for the FP64 setup FFT");
        HIP_TRY(launch_col_fft<double>(c, nt, st));
        if (p.Pz > 1) {
            ColArgs z{};
            z.buf = Sd;
            z.nplanes = 1;
            z.plane_stride = 0;
            z.ncols = p.Py * p.hx;
            z.cols_per_row = p.hx;
            z.row2_stride = p.sxd;
            z.es = (int64_t)p.Py * p.sxd;
            z.nin = p.Pz;
            z.nout = p.Pz;
            z.inverse = 0;
            z.tw_cols = std::max(1, std::min(64, cap / p.Pz));
            z.pl = p.fz;
            z.tw = s->at<char>(p.o_twzd);
            HIP_TRY(launch_col_fft<double>(z, nt, st));
        }
        if (p.zd) {
            // planes: xx 0-1, xy 2-3, xz 4, yy 5-6, yz 7, zz 8-9
            static const int first_plane[6] = {0, 2, 4, 5, 7, 8};
            HIP_TRY(launch_table_z2<T>(s->at<char>(p.o_kern) + (size_t)first_plane[q] * p.oct_elems * p.esz,
                                       Sd, comps[q], p.hx, p.Py, p.sxd, 1.0 / ((double)p.Px * p.Py), stats,
                                       st));
        } else {
            HIP_TRY(launch_octant<T>(s->at<char>(p.o_kern) + (size_t)q * p.oct_elems * p.esz, Sd, p.hx,
                                     p.Py, p.Pz, p.sxd, scale, stats, st));
        }
    }
    unsigned long long h[2];
    HIP_TRY(hipMemcpyAsync(h, stats, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double im, re;
    memcpy(&im, &h[0], 8);
    memcpy(&re, &h[1], 8);
    s->imag_ratio = re > 0 ? im / re : 0.0;
    return MM_OK;
}

// Explicit Euler + renormalisation (the paper's integrator): ping-pong between
// m_n and m_a, one field evaluation per step; the result ends in m_n.
// Applied field during step n of a schedule piece: h0 + (h1 - h0) n / steps.
void piece_field(const mm_segment& g, int64_t n, double h[3])
{
    const double f = g.steps > 0 ? (double)n / (double)g.steps : 0.0;
    for (int c = 0; c < 3; ++c) h[c] = g.h0[c] + (g.h1[c] - g.h0[c]) * f;
}

bool piece_ramps(const mm_segment& g)
{
    return g.h0[0] != g.h1[0] || g.h0[1] != g.h1[1] || g.h0[2] != g.h1[2];
}

// nsteps explicit Euler steps; with a schedule piece g, step n takes the field of
// the piece's step n0 + n.
template <typename T>
mm_status euler_impl(mm_sim* s, int64_t nsteps, double dt, const mm_segment* g = nullptr,
                     int64_t n0 = 0, hipStream_t st = nullptr, bool prologue = true)
{
    const Plan& p = s->p;
    if (!st) st = s->stream;
    T* bufs[2] = {s->at<T>(p.o_mn), s->at<T>(p.o_ma)};
    T* hd = s->at<T>(p.o_hd);
    LlgArgs<T> a = llg_args<T>(s, dt);
    a.stage = 0;
    if (p.fs && !(s->flags & MM_NO_DEMAG)) {
        // fused stage plans: the spectrum of m_n from the prologue (or left by the
        // previous even group of steps), then per step the y / z passes and one fused
        // pass (x inverse, Euler update, x forward of the new m); m and the spectrum
        // both alternate between two buffers
        PassCtx c = pass_ctx(s);
        void* sb[2] = {s->at<char>(p.o_S), s->at<char>(p.o_S2)};
        if (prologue) LAUNCH(KX_FWD, pass_x_forward<T>(c, bufs[0], st));
        FusedStageArgs<T> f{};
        f.g = a;
        f.g.acc = s->at<T>(p.o_acc);
        f.g.hd = nullptr;
        f.sy = c.Sy;
        f.tw = c.twx;
        for (int64_t n = 0; n < nsteps; ++n) {
            if (g) {
                piece_field(*g, n0 + n, s->hext);
                f.g.hx = (T)(s->hext[0] / s->mat.Ms);
                f.g.hy = (T)(s->hext[1] / s->mat.Ms);
                f.g.hz = (T)(s->hext[2] / s->mat.Ms);
            }
            c.S = sb[n & 1];
            mm_status r = demag_mid<T>(s, c, st);
            if (r != MM_OK) return r;
            f.g.ms = f.g.mn = bufs[n & 1];
            f.g.out = bufs[(n + 1) & 1];
            f.S_in = sb[n & 1];
            f.S_out = sb[(n + 1) & 1];
            LAUNCH(KLLG, launch_fused_stage<T>(f, p.Px, p.fs_lines, st) ? hipGetLastError()
                                                                        : hipErrorInvalidValue);
        }
        if (nsteps & 1)
            HIP_TRY(hipMemcpyAsync(bufs[0], bufs[1], 3 * (size_t)p.N * sizeof(T), hipMemcpyDeviceToDevice, st));
        return MM_OK;
    }
    for (int64_t n = 0; n < nsteps; ++n) {
        T* src = bufs[n & 1];
        T* dst = bufs[(n + 1) & 1];
        if (g) {
            piece_field(*g, n0 + n, s->hext);
            a.hx = (T)(s->hext[0] / s->mat.Ms);
            a.hy = (T)(s->hext[1] / s->mat.Ms);
            a.hz = (T)(s->hext[2] / s->mat.Ms);
        }
        if (!(s->flags & MM_NO_DEMAG)) {
            mm_status r = demag<T>(s, src, hd, st);
            if (r != MM_OK) return r;
        }
        a.ms = src;
        a.mn = src;
        a.acc = s->at<T>(p.o_acc);
        a.out = dst;
        LAUNCH(KLLG, launch_llg_stage<T>(a, st));
    }
    if (nsteps & 1)
        HIP_TRY(hipMemcpyAsync(bufs[0], bufs[1], 3 * (size_t)p.N * sizeof(T), hipMemcpyDeviceToDevice, st));
    return MM_OK;
}

void drop_graph(mm_sim* s)
{
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->rem_exec) (void)hipGraphExecDestroy(s->rem_exec);
    s->gexec = nullptr;
    s->graph = nullptr;
    s->rem_exec = nullptr;
    s->rem_len = 0;
    s->graph_valid = false;
}

void drop_bwd_graphs(mm_sim* s)
{
    for (auto& g : s->bwd) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = mm_sim::BwdGraph{};
    }
}

// Steps of a fused-stage plan: one prologue per call (the spectrum of m_n), then
// the steps, replaying captured 8-step graphs that leave S as they found it.
template <typename T>
mm_status fused_step_impl(mm_sim* s, int64_t nsteps, double dt, bool use_graph)
{
    hipStream_t st = s->stream;
    if (nsteps <= 0) return MM_OK;
    if (!use_graph) return rk4_fused_steps<T>(s, nsteps, dt, true, st);
    // 32 steps a graph: on the 128x128x1 film 49.9 -> 49.4 us per step against 8
    // (fewer graph launches; a rollout segment of 50 steps is one chunk and 18 steps)
    const int chunk = 32;
    if (!s->graph_valid || s->graph_dt != dt || s->graph_method != MM_RK4) {
        drop_graph(s);
        HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
        mm_status r = rk4_fused_steps<T>(s, chunk, dt, false, s->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
        if (r != MM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return r;
        }
        if (e != hipSuccess) return fail(MM_EHIP, "graph capture: %s", hipGetErrorString(e));
        s->graph = g;
        HIP_TRY(hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0));
        s->graph_valid = true;
        s->graph_dt = dt;
        s->graph_chunk = chunk;
        s->graph_method = MM_RK4;
    }
    // the steps past whole chunks replay a graph of their own (kept while the chunk
    // graph is valid, for one remainder length)
    const int64_t rem = nsteps % s->graph_chunk;
    if (rem > 0 && (!s->rem_exec || s->rem_len != rem)) {
        if (s->rem_exec) (void)hipGraphExecDestroy(s->rem_exec);
        s->rem_exec = nullptr;
        s->rem_len = 0;
        HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
        mm_status r = rk4_fused_steps<T>(s, rem, dt, false, s->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
        if (r == MM_OK && e == hipSuccess) e = hipGraphInstantiate(&s->rem_exec, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (r != MM_OK) return r;
        if (e != hipSuccess) return fail(MM_EHIP, "graph capture: %s", hipGetErrorString(e));
        s->rem_len = rem;
    }
    if (mm_status r = rk4_fused_steps<T>(s, 0, dt, true, st); r != MM_OK) return r;  // prologue
    for (int64_t n = 0; n + s->graph_chunk <= nsteps; n += s->graph_chunk) HIP_TRY(hipGraphLaunch(s->gexec, st));
    if (rem > 0) HIP_TRY(hipGraphLaunch(s->rem_exec, st));
    return MM_OK;
}

template <typename T>
mm_status step_impl(mm_sim* s, int64_t nsteps, double dt, bool force_graph = false)
{
    hipStream_t st = s->stream;
    const bool use_graph = ((s->flags & MM_USE_GRAPH) || force_graph) && s->prof_kernel < 0;
    if (s->p.fs) return fused_step_impl<T>(s, nsteps, dt, use_graph);
    if (!use_graph) {
        for (int64_t n = 0; n < nsteps; ++n) {
            mm_status r = rk4_step<T>(s, dt, st);
            if (r != MM_OK) return r;
        }
        return MM_OK;
    }
    const int chunk = 8;
    if (!s->graph_valid || s->graph_dt != dt || s->graph_method != MM_RK4) {
        drop_graph(s);
        HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
        mm_status r = MM_OK;
        for (int q = 0; q < chunk && r == MM_OK; ++q) r = rk4_step<T>(s, dt, s->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
        if (r != MM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return r;
        }
        if (e != hipSuccess) return fail(MM_EHIP, "graph capture: %s", hipGetErrorString(e));
        s->graph = g;
        HIP_TRY(hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0));
        s->graph_valid = true;
        s->graph_dt = dt;
        s->graph_chunk = chunk;
        s->graph_method = MM_RK4;
    }
    int64_t n = 0;
    for (; n + s->graph_chunk <= nsteps; n += s->graph_chunk) HIP_TRY(hipGraphLaunch(s->gexec, st));
    for (; n < nsteps; ++n) {
        mm_status r = rk4_step<T>(s, dt, st);
        if (r != MM_OK) return r;
    }
    return MM_OK;
}

// nsteps Euler steps under the handle's constant field; with MM_USE_GRAPH whole
// groups of 8 steps replay a captured graph (shared slot with the RK4 graph).
template <typename T>
mm_status euler_steps(mm_sim* s, int64_t nsteps, double dt)
{
    const bool use_graph = (s->flags & MM_USE_GRAPH) && s->prof_kernel < 0;
    const int chunk = 8;  // even: the captured steps end in m_n (and a fused plan's
                          // spectrum in S) without a copy
    if (!use_graph || nsteps < chunk) return euler_impl<T>(s, nsteps, dt);
    if (!s->graph_valid || s->graph_dt != dt || s->graph_method != MM_EULER) {
        drop_graph(s);
        HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
        // a fused plan's graph takes the spectrum of m_n as it finds it in S
        mm_status r = euler_impl<T>(s, chunk, dt, nullptr, 0, s->cap_stream, false);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
        if (r != MM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return r;
        }
        if (e != hipSuccess) return fail(MM_EHIP, "graph capture: %s", hipGetErrorString(e));
        s->graph = g;
        HIP_TRY(hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0));
        s->graph_valid = true;
        s->graph_dt = dt;
        s->graph_chunk = chunk;
        s->graph_method = MM_EULER;
    }
    if (s->p.fs && !(s->flags & MM_NO_DEMAG)) {
        const PassCtx c = pass_ctx(s);
        hipStream_t st = s->stream;
        LAUNCH(KX_FWD, pass_x_forward<T>(c, s->at<T>(s->p.o_mn), st));
    }
    int64_t n = 0;
    for (; n + s->graph_chunk <= nsteps; n += s->graph_chunk) HIP_TRY(hipGraphLaunch(s->gexec, s->stream));
    // the remainder continues from the spectrum the groups left in S, as one plain
    // call would (the fused pass's x forward and the x forward pass round alike only
    // up to the compiler's contractions)
    return n < nsteps ? euler_impl<T>(s, nsteps - n, dt, nullptr, 0, nullptr, false) : MM_OK;
}

// One row of the mean-magnetisation trace, enqueued on the handle's stream.
template <typename T>
mm_status trace_sample(mm_sim* s, double t, double* row)
{
    const Plan& p = s->p;
    LlgArgs<T> a = llg_args<T>(s, 0.0);
    T* mn = s->at<T>(p.o_mn);
    a.ms = mn;
    a.mn = mn;
    a.hd = nullptr;
    double* dout = s->at<double>(p.o_redout);
    HIP_TRY(launch_reduce<T>(a, s->at<double>(p.o_red), reduce_blocks(p.N), dout, s->stream));
    HIP_TRY(launch_trace_row(dout, 1.0 / (double)p.N, t, row, s->stream));
    return MM_OK;
}

// The pieces of a time-dependent protocol, sampled every `every` steps.
template <typename T>
mm_status schedule_impl(mm_sim* s, const mm_segment* segs, int nseg, int method, double dt,
                        int64_t every, double* trace, int64_t* rows)
{
    int64_t done = 0, nrow = 0;
    for (int q = 0; q < nseg; ++q) {
        const mm_segment& g = segs[q];
        const bool ramp = piece_ramps(g);
        s->alpha = g.alpha;
        s->graph_valid = false;
        if (!ramp)
            for (int c = 0; c < 3; ++c) s->hext[c] = g.h0[c];
        for (int64_t n = 0; n < g.steps;) {
            const int64_t run = std::min(g.steps - n, every - done % every);
            mm_status r = MM_OK;
            if (method == MM_EULER) {
                r = ramp ? euler_impl<T>(s, run, dt, &g, n) : euler_steps<T>(s, run, dt);
            } else if (!ramp) {
                r = step_impl<T>(s, run, dt);
            } else {
                for (int64_t k = 0; k < run && r == MM_OK; ++k) {
                    piece_field(g, n + k, s->hext);
                    r = rk4_step<T>(s, dt, s->stream);
                }
            }
            if (r != MM_OK) return r;
            n += run;
            done += run;
            if (done % every == 0) {
                if ((r = trace_sample<T>(s, (double)done * dt, trace + 4 * nrow)) != MM_OK) return r;
                ++nrow;
            }
        }
        s->graph_valid = false;
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (rows) *rows = nrow;
    return MM_OK;
}

template <typename T>
mm_status field_impl(mm_sim* s, int term, void* out, int on_device)
{
    const Plan& p = s->p;
    hipStream_t st = s->stream;
    LlgArgs<T> a = llg_args<T>(s, 0.0);
    T* mn = s->at<T>(p.o_mn);
    a.ms = mn;
    a.mn = mn;
    if (!(s->flags & MM_NO_DEMAG) && (term == MM_H_DEMAG || term == MM_H_EFF)) {
        mm_status r = demag<T>(s, mn, s->at<T>(p.o_hd), st);
        if (r != MM_OK) return r;
    }
    T* dst = on_device ? (T*)out : s->at<T>(p.o_mb);
    HIP_TRY(launch_field_term<T>(a, term, (T)s->mat.Ms, dst, st));
    if (!on_device) {
        HIP_TRY(hipMemcpyAsync(out, dst, 3 * p.N * sizeof(T), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    return MM_OK;
}

template <typename T>
mm_status reduce_impl(mm_sim* s, double out[kRedSlots])
{
    const Plan& p = s->p;
    hipStream_t st = s->stream;
    LlgArgs<T> a = llg_args<T>(s, 0.0);
    T* mn = s->at<T>(p.o_mn);
    a.ms = mn;
    a.mn = mn;
    if (!(s->flags & MM_NO_DEMAG)) {
        mm_status r = demag<T>(s, mn, s->at<T>(p.o_hd), st);
        if (r != MM_OK) return r;
    }
    double* dout = s->at<double>(p.o_redout);
    HIP_TRY(launch_reduce<T>(a, s->at<double>(p.o_red), reduce_blocks(p.N), dout, st));
    HIP_TRY(hipMemcpyAsync(out, dout, kRedSlots * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return MM_OK;
}

template <typename T>
mm_status set_m_impl(mm_sim* s, const void* m, int on_device)
{
    const Plan& p = s->p;
    hipStream_t st = s->stream;
    T* mn = s->at<T>(p.o_mn);
    HIP_TRY(hipMemcpyAsync(mn, m, 3 * p.N * sizeof(T),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    unsigned int* bad = reinterpret_cast<unsigned int*>(s->at<char>(p.o_flags) + 32);
    HIP_TRY(hipMemsetAsync(bad, 0, sizeof(unsigned int), st));
    HIP_TRY(launch_normalize<T>(mn, p.N, bad, st));
    unsigned int nbad = 0;
    HIP_TRY(hipMemcpyAsync(&nbad, bad, sizeof nbad, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (nbad) {
        s->has_m = false;
        return fail(MM_EINVAL, "m has %u zero-length or non-finite cells", nbad);
    }
    s->has_m = true;
    return MM_OK;
}

// ---------------------------------------------------------------- adjoint
// Adjoint workspace: per step of a segment its start state, the three later
// stage states and the four stage fields (8 vectors, stored while the segment is
// recomputed from its checkpoint), 7 working vectors, and the FP64 dLoss/dKu
// accumulator.
constexpr int kAdjPerStep = 8, kAdjWork = 7;

size_t adj_bytes(const Plan& p, int64_t ck)
{
    const size_t vec = align256(3 * (size_t)p.N * p.esz);
    return ((size_t)ck * kAdjPerStep + kAdjWork) * vec + align256((size_t)p.N * sizeof(double));
}

// nsteps RK4 steps; the state at the start of every segment of ck steps goes to
// its checkpoint slot, and the steps of a segment replay captured graphs.
template <typename T>
mm_status rollout_impl(mm_sim* s, int64_t nsteps, double dt, int64_t ck, T* ckpt)
{
    const Plan& p = s->p;
    const size_t vec = 3 * (size_t)p.N;
    T* mn = s->at<T>(p.o_mn);
    for (int64_t n = 0; n < nsteps; n += ck) {
        HIP_TRY(hipMemcpyAsync(ckpt + (n / ck) * vec, mn, vec * sizeof(T), hipMemcpyDeviceToDevice,
                               s->stream));
        mm_status r = step_impl<T>(s, std::min(ck, nsteps - n), dt, true);
        if (r != MM_OK) return r;
    }
    return MM_OK;
}

// Buffers of the reverse sweep, carved from the caller's adjoint workspace.
template <typename T>
struct AdjBufs {
    T* slot;  // [ck][8][3N]: per step m_n, m_2, m_3, m_4, h_1 .. h_4
    T *lam, *accl, *mu, *dF, *nu, *loc, *scr;
    double* dku;
    size_t vbytes;
    T* at(int64_t n, int q) const
    {
        return reinterpret_cast<T*>(reinterpret_cast<char*>(slot) + ((size_t)n * kAdjPerStep + q) * vbytes);
    }
};

// One segment of `len` steps whose start state is already in slot 0: the forward
// recompute, storing every stage state and stage field, then the reverse sweep
// from the covector in b.lam (left in b.lam on return).  Enqueued on st; every
// pointer it uses is fixed for a given workspace, so it can be captured.
template <typename T>
mm_status backward_segment(mm_sim* s, const AdjBufs<T>& b, int64_t len, double dt, hipStream_t st)
{
    const Plan& p = s->p;
    const bool with_demag = !(s->flags & MM_NO_DEMAG);
    T* hd = s->at<T>(p.o_hd);
    LlgArgs<T> la = llg_args<T>(s, dt);
    la.acc = b.scr;
    if (p.fs && with_demag) {
        // fused stages (small grids): the y / z passes and one fused pass per stage,
        // which also stores the stage's effective field; the segment's
        // final stage output is not needed (the next segment starts from its
        // checkpoint) and goes to the reverse sweep's still unused mu buffer
        PassCtx c = pass_ctx(s);
        void* bufs[2] = {s->at<char>(p.o_S), s->at<char>(p.o_S2)};
        HIP_TRY(pass_x_forward<T>(c, b.at(0, 0), st));
        FusedStageArgs<T> f{};
        f.g = la;
        f.g.hd = nullptr;
        f.sy = c.Sy;
        f.tw = c.twx;
        for (int64_t n = 0; n < len; ++n) {
            f.g.mn = b.at(n, 0);
            for (int stg = 0; stg < 4; ++stg) {
                c.S = bufs[stg & 1];
                mm_status r = demag_mid<T>(s, c, st);
                if (r != MM_OK) return r;
                f.g.ms = b.at(n, stg);
                f.g.out = (stg == 3 && n == len - 1) ? b.mu : (stg < 3 ? b.at(n, stg + 1) : b.at(n + 1, 0));
                f.g.stage = stg + 1;
                f.hout = b.at(n, 4 + stg);
                f.S_in = bufs[stg & 1];
                f.S_out = bufs[(stg + 1) & 1];
                if (!launch_fused_stage<T>(f, p.Px, p.fs_lines, st))
                    return fail(MM_ENOTSUP, "no fused stage pass of length %d", p.Px);
                HIP_TRY(hipGetLastError());
            }
        }
    }
    for (int64_t n = 0; n < len && !(p.fs && with_demag); ++n) {
        la.mn = b.at(n, 0);
        for (int stg = 0; stg < 4; ++stg) {
            la.ms = b.at(n, stg);
            if (with_demag) {
                mm_status r = demag<T>(s, la.ms, hd, st);
                if (r != MM_OK) return r;
            }
            HIP_TRY(launch_field_term<T>(la, 4, (T)1, b.at(n, 4 + stg), st));
            if (stg == 3 && n == len - 1) break;  // the next segment starts from its checkpoint
            la.out = stg < 3 ? b.at(n, stg + 1) : b.at(n + 1, 0);
            la.stage = stg + 1;
            HIP_TRY(launch_llg_stage<T>(la, st));
        }
    }
    AdjArgs<T> aa{};
    aa.nx = p.nx;
    aa.ny = p.ny;
    aa.nz = p.nz;
    aa.N = p.N;
    aa.mu = b.mu;
    aa.dF = b.dF;
    aa.nu = b.nu;
    aa.loc = b.loc;
    aa.hd = with_demag ? hd : nullptr;
    aa.ku = la.ku;
    aa.can = la.can;
    aa.cex = la.cex;
    aa.G = la.gdt;
    aa.alpha = la.alpha;
    aa.dku = b.dku;
    aa.kfac = 2.0 / (kMu0 * s->mat.Ms * s->mat.Ms);
    aa.per = p.per;
    T* lam = b.lam;
    T* accl = b.accl;
    const T cmu[4] = {(T)0, (T)(1.0 / 6.0), (T)(2.0 / 6.0), (T)(2.0 / 6.0)};
    const T ca[4] = {(T)0, (T)0.5, (T)0.5, (T)1};
    if (p.fs && with_demag) {
        // fused reverse sweep: the renormalisation and last-stage nu of the last step
        // and the x forward of that nu; then per stage the y / z passes and one fused
        // pass (x inverse of nu's field, the apply, and the stage before's nu, or at
        // a step boundary the renormalisation of the step before and its last
        // stage's nu, with the x forward of the new nu).  The spectrum and nu
        // alternate between two buffers (scr is free once the recompute is done).
        PassCtx c = pass_ctx(s);
        void* sb[2] = {s->at<char>(p.o_S), s->at<char>(p.o_S2)};
        T* nub[2] = {b.nu, b.scr};
        const int64_t nl = len - 1;
        aa.mn = b.at(nl, 0);
        aa.m2 = b.at(nl, 1);
        aa.m3 = b.at(nl, 2);
        aa.m4 = b.at(nl, 3);
        aa.h1 = b.at(nl, 4);
        aa.h2 = b.at(nl, 5);
        aa.h3 = b.at(nl, 6);
        aa.h4 = b.at(nl, 7);
        aa.lam = lam;
        aa.accl = accl;
        aa.nu = nub[0];
        HIP_TRY(launch_adj_renorm<T>(aa, st));
        HIP_TRY(launch_adj_nu<T>(aa, b.at(nl, 3), b.at(nl, 7), st));
        c.S = sb[0];
        HIP_TRY(pass_x_forward<T>(c, nub[0], st));
        FusedAdjArgs<T> fa{};
        fa.a = aa;
        fa.sy = c.Sy;
        fa.tw = c.twx;
        int k = 0;  // fused passes so far: spectrum sb[k & 1], nu nub[k & 1]
        for (int64_t n = len - 1; n >= 0; --n) {
            for (int stg = 3; stg >= 0; --stg, ++k) {
                c.S = sb[k & 1];
                mm_status r = demag_mid<T>(s, c, st);
                if (r != MM_OK) return r;
                fa.a.accl = accl;
                fa.nu_in = nub[k & 1];
                fa.nu_out = nub[(k + 1) & 1];
                fa.cmu = cmu[stg];
                fa.ca = ca[stg];
                fa.S_in = sb[k & 1];
                fa.S_out = sb[(k + 1) & 1];
                if (stg > 0) {
                    fa.mode = 1;
                    fa.ms = b.at(n, stg - 1);
                    fa.hs = b.at(n, 4 + stg - 1);
                } else if (n > 0) {
                    fa.mode = 2;
                    for (int q = 0; q < 8; ++q) fa.st[q] = b.at(n - 1, q);
                    fa.accl_prev = lam;  // the step before's accumulator once swapped
                } else {
                    fa.mode = 0;
                }
                if (!launch_fused_adjoint<T>(fa, p.Px, p.fs_lines, st))
                    return fail(MM_ENOTSUP, "no fused adjoint pass of length %d", p.Px);
                HIP_TRY(hipGetLastError());
            }
            std::swap(lam, accl);
        }
    }
    for (int64_t n = len - 1; n >= 0 && !(p.fs && with_demag); --n) {
        aa.mn = b.at(n, 0);
        aa.m2 = b.at(n, 1);
        aa.m3 = b.at(n, 2);
        aa.m4 = b.at(n, 3);
        aa.h1 = b.at(n, 4);
        aa.h2 = b.at(n, 5);
        aa.h3 = b.at(n, 6);
        aa.h4 = b.at(n, 7);
        aa.lam = lam;
        aa.accl = accl;
        // reverse: renormalisation, then stages 4..1
        HIP_TRY(launch_adj_renorm<T>(aa, st));
        for (int stg = 3; stg >= 0; --stg) {
            HIP_TRY(launch_adj_nu<T>(aa, b.at(n, stg), b.at(n, 4 + stg), st));
            if (with_demag) {
                mm_status r = demag<T>(s, b.nu, hd, st);
                if (r != MM_OK) return r;
            }
            HIP_TRY(launch_adj_apply<T>(aa, cmu[stg], ca[stg], st));
        }
        std::swap(lam, accl);
    }
    if (lam != b.lam)  // an odd number of steps: the covector ends in the other buffer
        HIP_TRY(hipMemcpyAsync(b.lam, lam, 3 * (size_t)p.N * sizeof(T), hipMemcpyDeviceToDevice, st));
    return MM_OK;
}

// Runs backward_segment for `len` steps, replaying a captured graph when one for
// the same length, workspace and step parameters exists, else capturing one
// (eagerly while a profile is open).
template <typename T>
mm_status backward_segment_graph(mm_sim* s, const AdjBufs<T>& b, int64_t len, double dt, const char* ws)
{
    if (s->prof_kernel >= 0) return backward_segment<T>(s, b, len, dt, s->stream);
    auto same = [&](const mm_sim::BwdGraph& g) {
        return g.exec && g.len == len && g.dt == dt && g.alpha == s->alpha && g.ws == ws &&
               g.ku_map == s->has_ku_map && g.hext[0] == s->hext[0] && g.hext[1] == s->hext[1] &&
               g.hext[2] == s->hext[2];
    };
    mm_sim::BwdGraph* hit = nullptr;
    for (auto& g : s->bwd)
        if (same(g)) hit = &g;
    if (!hit) {
        // replace a slot of another length if there is one, else the first
        hit = &s->bwd[0];
        for (auto& g : s->bwd)
            if (!g.exec || g.len != len) {
                hit = &g;
                break;
            }
        if (hit->exec) (void)hipGraphExecDestroy(hit->exec);
        *hit = mm_sim::BwdGraph{};
        HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
        mm_status r = backward_segment<T>(s, b, len, dt, s->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
        if (r != MM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return r;
        }
        if (e != hipSuccess) return fail(MM_EHIP, "graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&hit->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            hit->exec = nullptr;
            return fail(MM_EHIP, "graph instantiate: %s", hipGetErrorString(e));
        }
        hit->len = len;
        hit->dt = dt;
        hit->alpha = s->alpha;
        hit->ws = ws;
        hit->ku_map = s->has_ku_map;
        for (int c = 0; c < 3; ++c) hit->hext[c] = s->hext[c];
    }
    HIP_TRY(hipGraphLaunch(hit->exec, s->stream));
    return MM_OK;
}

// The reverse sweep over every segment, last first, in the adjoint workspace ws
// (adj_bytes(p, ck) bytes, 256-byte aligned).  graphs: replay a captured graph
// per segment; otherwise every launch is made directly on the handle's stream
// (nothing is captured or instantiated, and the only operations are kernel
// launches and device-to-device copies, so a caller may capture the whole call).
template <typename T>
mm_status backward_impl(mm_sim* s, int64_t nsteps, double dt, int64_t ck, const T* ckpt,
                        const T* lam_final, double* dku, T* dm0, char* ws, bool graphs)
{
    const Plan& p = s->p;
    hipStream_t st = s->stream;
    const size_t vec = 3 * (size_t)p.N, vbytes = align256(vec * sizeof(T));
    AdjBufs<T> b{};
    b.vbytes = vbytes;
    b.slot = reinterpret_cast<T*>(ws);
    char* q = ws + (size_t)ck * kAdjPerStep * vbytes;
    auto take = [&]() {
        T* r = reinterpret_cast<T*>(q);
        q += vbytes;
        return r;
    };
    b.lam = take();
    b.accl = take();
    b.mu = take();
    b.dF = take();
    b.nu = take();
    b.loc = take();
    b.scr = take();
    b.dku = reinterpret_cast<double*>(q);
    HIP_TRY(hipMemcpyAsync(b.lam, lam_final, vec * sizeof(T), hipMemcpyDeviceToDevice, st));
    HIP_TRY(launch_zero_f64(b.dku, p.N, st));
    const int64_t nseg = (nsteps + ck - 1) / ck;
    for (int64_t g = nseg - 1; g >= 0; --g) {
        const int64_t len = std::min(ck, nsteps - g * ck);
        HIP_TRY(hipMemcpyAsync(b.at(0, 0), ckpt + g * vec, vec * sizeof(T), hipMemcpyDeviceToDevice, st));
        mm_status r = graphs ? backward_segment_graph<T>(s, b, len, dt, ws) : backward_segment<T>(s, b, len, dt, st);
        if (r != MM_OK) return r;
    }
    HIP_TRY(hipMemcpyAsync(dku, b.dku, (size_t)p.N * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (dm0) HIP_TRY(hipMemcpyAsync(dm0, b.lam, vec * sizeof(T), hipMemcpyDeviceToDevice, st));
    return MM_OK;
}

// ---------------------------------------------------------------- batched
constexpr int kBatchLlgKind = 6;
struct BatchClassHost {
    int kind;  // 0 x passes, 1 y passes, 2 z k-space, 3 y k-space, 5 two-plane y k-space,
               // kBatchLlgKind the LLG stage (P = planes per thread)
    int P;
    std::vector<int> members, prefix;
    size_t off;  // element offset of members, then prefix, in the device int array
};

bool fast_supported(int kind, int P, size_t esz)
{
    if (fast_first_radix(P) == 0) return false;
    switch (kind) {
    case 0: return P >= 16 && P <= (esz == 8 ? 1024 : 2048);
    case 1: return P >= 16 && P <= 2048;
    case 2: return P >= 2 && P <= (esz == 8 ? 32 : 64);
    case 5: return fast_ky2_lines(P) > 0;
    default: return P >= 16 && P <= 1024;
    }
}

struct BatchLayout {
    std::vector<Plan> plans;
    bool fast = false;
    std::vector<BatchClassHost> classes;
    size_t o_classes = 0;
    int64_t class_ints = 0;
    std::vector<BatchDesc> desc;
    std::vector<int> prefix[4];   // runtime-radix passes: x forward, y, k-space, x inverse
    int64_t vec_elems = 0, S_elems = 0, kern_elems = 0, tw_elems = 0, cells = 0;
    size_t scratch = 0;
    size_t o_desc, o_prefix, o_mn, o_ma, o_mb, o_acc, o_hd, o_S, o_kern, o_tw, o_flags, o_scratch, total;
    int prec;
    size_t esz;
    bool plan_generic = false;  // the plans were built with the runtime-radix passes forced
    std::vector<std::array<int, 2>> pad;  // per grid explicit (px, py), 0 = automatic
};

mm_status batch_layout_plans(int32_t n, const mm_grid* grids, const mm_options* opt, bool classes,
                             BatchLayout* L);
bool merge_small_classes(int32_t n, BatchLayout* L);
mm_status batch_layout_offsets(int32_t n, BatchLayout* L);

mm_status batch_layout(int32_t n, const mm_grid* grids, const mm_options* opt, BatchLayout* L)
{
    if (n < 1) return fail(MM_EINVAL, "batch needs at least one grid");
    if (!grids) return fail(MM_EINVAL, "grids is NULL");
    if (opt && (opt->flags & (MM_PERIODIC_X | MM_PERIODIC_Y | MM_PERIODIC_Z)))
        return fail(MM_ENOTSUP, "batches take open boundaries only (periodic axes set)");
    mm_options o = opt ? *opt : mm_options{};
    o.threads = 256;
    // size classes (the specialised passes) are wanted with power-of-two or fast
    // padding; otherwise every grid runs the runtime-radix passes, whose plans
    // must not take the two-plane schedule.  If some grid has no size class, the
    // layout is built again that way.
    const bool want_fast = (o.flags & (MM_POW2_PAD | MM_FAST_PAD)) && !(o.flags & MM_GENERIC_FFT);
    for (int attempt = want_fast ? 0 : 1; attempt < 2; ++attempt) {
        mm_options oa = o;
        if (attempt == 1) oa.flags |= MM_GENERIC_FFT;
        L->plan_generic = attempt == 1;
        L->pad.assign(n, {0, 0});
        // size classes holding a small share of the cells are padded up into the next
        // class of their axis (at most a few rounds: each round removes a class)
        for (int round = 0; round < 8; ++round) {
            mm_status st = batch_layout_plans(n, grids, &oa, want_fast && attempt == 0, L);
            if (st != MM_OK) return st;
            if (!L->fast || !merge_small_classes(n, L)) break;
        }
        if (L->fast || !want_fast) break;
    }
    return batch_layout_offsets(n, L);
}

// A size class costs one launch per pass whatever its size (a few microseconds
// of fill and drain).  The grids of an x or y class holding under 1/32 of the
// batch's cells move to the next larger padded length of that axis present in
// the batch: any length >= 2n - 1 gives the same linear convolution, and the
// few extra bytes of those grids cost less than the launches they save.
// Returns true when some grid moved (the plans must then be rebuilt).
bool merge_small_classes(int32_t n, BatchLayout* L)
{
    bool moved = false;
    for (int axis = 0; axis < 2; ++axis) {
        std::map<int, int64_t> cells;  // padded length -> cells of its grids
        for (int s = 0; s < n; ++s) cells[axis ? L->plans[s].Py : L->plans[s].Px] += L->plans[s].N;
        if (cells.size() < 2) continue;
        for (auto it = cells.begin(); std::next(it) != cells.end(); ++it) {
            if (it->second * 32 >= L->cells) continue;
            const int to = std::next(it)->first;
            for (int s = 0; s < n; ++s) {
                const Plan& p = L->plans[s];
                if ((axis ? p.Py : p.Px) == it->first) {
                    L->pad[s][axis] = to;
                    moved = true;
                }
            }
            break;  // one class per axis and round; the plans are rebuilt in between
        }
    }
    return moved;
}

mm_status batch_layout_plans(int32_t n, const mm_grid* grids, const mm_options* opt, bool classes,
                             BatchLayout* L)
{
    const mm_options& o = *opt;
    L->vec_elems = L->S_elems = L->kern_elems = L->tw_elems = L->cells = 0;
    L->scratch = 0;
    L->class_ints = 0;
    L->plans.assign(n, Plan{});
    L->desc.resize(n);
    for (int q = 0; q < 4; ++q) L->prefix[q].assign(n + 1, 0);
    for (int s = 0; s < n; ++s) {
        Plan& p = L->plans[s];
        mm_options og = o;
        if (s < (int)L->pad.size()) {
            og.px = L->pad[s][0];
            og.py = L->pad[s][1];
        }
        mm_status st = build_plan(&grids[s], &og, &p);
        if (st != MM_OK) {
            std::string keep = g_err;
            return fail(st, "grid %d: %s", s, keep.c_str());
        }
        const int cap = kElemsPerThread * 256, ldscap = cap + 64;
        BatchDesc& d = L->desc[s];
        memset(&d, 0, sizeof d);
        d.nx = p.nx;
        d.ny = p.ny;
        d.nz = p.nz;
        d.Px = p.Px;
        d.Py = p.Py;
        d.Pz = p.Pz;
        d.hx = p.hx;
        d.Sy = (int)p.S_rows;
        d.three_d = p.three_d ? 1 : 0;
        d.x_lines = p.x_lines;
        d.y_lines = std::min(cap / p.Py, ldscap / (p.Py + 1));
        d.k_tw = p.k_tw;
        d.moff = L->vec_elems;
        d.soff = L->S_elems;
        d.koff = L->kern_elems;
        d.oct = p.oct_elems;
        d.twx = L->tw_elems;
        d.twy = d.twx + p.Px;
        d.twz = d.twy + p.Py;
        d.fx = p.fx;
        d.fy = p.fy;
        d.fz = p.fz;
        L->vec_elems += 3 * p.N;
        L->S_elems += 3 * (int64_t)p.nz * p.hx * p.S_rows;
        L->kern_elems += (int64_t)p.kplanes * p.oct_elems;
        L->tw_elems += p.Px + p.Py + p.Pz;
        L->cells += p.N;
        L->scratch = std::max(L->scratch, p.total);
        const int npairs = (3 * p.nz * p.ny + 1) / 2;
        const int tiles[4] = {
            (npairs + p.x_lines - 1) / p.x_lines,
            p.three_d ? (3 * p.nz * p.hx + d.y_lines - 1) / d.y_lines : 0,
            p.three_d ? (int)((p.hx * (int64_t)p.Py + p.k_tw - 1) / p.k_tw) : (p.hx + p.k_tw - 1) / p.k_tw,
            (npairs + p.x_lines - 1) / p.x_lines};
        for (int q = 0; q < 4; ++q) L->prefix[q][s + 1] = L->prefix[q][s] + tiles[q];
    }
    L->prec = o.prec;
    L->esz = o.prec == MM_F32 ? 4 : 8;
    // size classes for the specialised passes (power-of-two or fast padding)
    L->fast = false;
    L->classes.clear();
    if (classes) {
        bool ok = true;
        auto cls = [&](int kind, int P) -> BatchClassHost& {
            for (auto& c : L->classes)
                if (c.kind == kind && c.P == P) return c;
            L->classes.push_back(BatchClassHost{kind, P, {}, {0}, 0});
            return L->classes.back();
        };
        for (int s = 0; s < n && ok; ++s) {
            const Plan& p = L->plans[s];
            // n: the valid samples along the axis; the size-class bodies prune the
            // second half of each line, so they need 2n <= P
            auto add = [&](int kind, int P, int n, int tiles) {
                if (!fast_supported(kind, P, L->esz) || 2 * n > P) {
                    ok = false;
                    return;
                }
                BatchClassHost& c = cls(kind, P);
                c.members.push_back(s);
                c.prefix.push_back(c.prefix.back() + tiles);
            };
            add(0, p.Px, p.nx, 3 * p.nz * ((p.ny + 15) / 16));
            if (!ok) break;
            if (p.zd) {
                const int L2 = fast_ky2_lines(p.Py);
                add(5, p.Py, p.ny, (p.hx + L2 - 1) / L2);
            } else if (p.three_d) {
                const int Ly = 256 / (p.Py / std::max(1, fast_first_radix(p.Py)));
                add(1, p.Py, p.ny, (3 * p.nz * p.hx + Ly - 1) / Ly);
                if (!ok) break;
                const int zc = kspace_z_cols_for(L->esz);
                add(2, p.Pz, p.nz, (int)((p.hx * (int64_t)p.Py + zc - 1) / zc));
            } else {
                const int Lk = std::max(1, fast_ky_lines(p.Py));
                add(3, p.Py, p.ny, (p.hx + Lk - 1) / Lk);
            }
        }
        if (ok)
            L->fast = true;
        else
            L->classes.clear();
    }
    // LLG classes (every layout): the grids grouped by planes per thread
    for (int s = 0; s < n; ++s) {
        const Plan& p = L->plans[s];
        const int kz = llg_z_for(p.nz);
        BatchClassHost* c = nullptr;
        for (auto& e : L->classes)
            if (e.kind == kBatchLlgKind && e.P == kz) c = &e;
        if (!c) {
            L->classes.push_back(BatchClassHost{kBatchLlgKind, kz, {}, {0}, 0});
            c = &L->classes.back();
        }
        c->members.push_back(s);
        c->prefix.push_back(c->prefix.back() + (int)llg_blocks(p.nx, p.ny, p.nz));
    }
    int64_t at = 0;
    for (auto& c : L->classes) {
        c.off = at;
        at += (int64_t)c.members.size() + (int64_t)c.prefix.size();
    }
    L->class_ints = at;
    return MM_OK;
}

mm_status batch_layout_offsets(int32_t n, BatchLayout* L)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    const size_t vec = (size_t)L->vec_elems * L->esz;
    L->o_desc = take(n * sizeof(BatchDesc));
    L->o_prefix = take(4 * (size_t)(n + 1) * sizeof(int));
    L->o_mn = take(vec);
    L->o_ma = take(vec);
    L->o_mb = take(vec);
    L->o_acc = take(vec);
    L->o_hd = take(vec);
    L->o_S = take((size_t)L->S_elems * 2 * L->esz);
    L->o_kern = take((size_t)L->kern_elems * L->esz);
    L->o_tw = take((size_t)L->tw_elems * 2 * L->esz);
    L->o_flags = take(64);
    L->o_classes = take((size_t)std::max<int64_t>(L->class_ints, 1) * sizeof(int));
    L->o_scratch = take(L->scratch);
    L->total = off;
    return MM_OK;
}

}  // namespace

struct mm_batch {
    BatchLayout L;
    int n;
    std::vector<mm_material> mats;  // one per grid
    double desc_dt;                 // the dt the descriptors' gdt was computed for
    uint32_t flags;
    char* ws;
    bool own_ws;
    hipStream_t stream, cap_stream;
    bool has_m;
    hipGraph_t graph;
    hipGraphExec_t gexec;
    bool graph_valid;
    double graph_dt;
    int graph_chunk;
    int tuned, tune_candidates;
    double tuned_ms;
    template <typename U>
    U* at(size_t off) const { return reinterpret_cast<U*>(ws + off); }
};

namespace {

// One demag field evaluation of every grid: the passes from m (in) to the
// field in the hd region, as size-class launches (power-of-two padding) or one
// runtime-radix launch per pass.
template <typename T>
mm_status batch_demag(mm_batch* b, const T* in, hipStream_t st)
{
    const BatchLayout& L = b->L;
    const int* pre = b->at<int>(L.o_prefix);
    const int n = b->n;
    if (L.fast) {
        BatchClass<T> bc{};
        bc.d = b->at<BatchDesc>(L.o_desc);
        bc.S = b->at<cpx<T>>(L.o_S);
        bc.kern = b->at<T>(L.o_kern);
        bc.tw = b->at<cpx<T>>(L.o_tw);
        bc.out = b->at<T>(L.o_hd);
        bc.in = in;
        const int* cints = b->at<int>(L.o_classes);
        auto run_classes = [&](int kind, int launch_kind, int inverse) -> mm_status {
            for (const BatchClassHost& c : L.classes) {
                if (c.kind != kind) continue;
                bc.members = cints + c.off;
                bc.prefix = cints + c.off + c.members.size();
                bc.nmem = (int)c.members.size();
                if (!launch_batch_class<T>(launch_kind, c.P, bc, c.prefix.back(), inverse, st))
                    return fail(MM_ENOTSUP, "no specialised pass of length %d", c.P);
                HIP_TRY(hipGetLastError());
            }
            return MM_OK;
        };
        mm_status r;
        if ((r = run_classes(0, 0, 0)) != MM_OK) return r;  // x forward
        if ((r = run_classes(1, 1, 0)) != MM_OK) return r;  // y forward
        if ((r = run_classes(2, 2, 0)) != MM_OK) return r;  // z k-space
        if ((r = run_classes(3, 3, 0)) != MM_OK) return r;  // y k-space
        if ((r = run_classes(5, 5, 0)) != MM_OK) return r;  // two-plane y k-space
        if ((r = run_classes(1, 1, 1)) != MM_OK) return r;  // y inverse
        return run_classes(0, 4, 0);                         // x inverse
    }
    BatchPass<T> p{};
    p.d = b->at<BatchDesc>(L.o_desc);
    p.n = n;
    p.S = b->at<cpx<T>>(L.o_S);
    p.kern = b->at<T>(L.o_kern);
    p.tw = b->at<cpx<T>>(L.o_tw);
    p.out = b->at<T>(L.o_hd);
    p.in = in;
    p.prefix = pre + 0 * (n + 1);
    HIP_TRY(launch_batch_pass<T>(0, p, L.prefix[0][n], 0, st));
    p.prefix = pre + 1 * (n + 1);
    HIP_TRY(launch_batch_pass<T>(1, p, L.prefix[1][n], 0, st));
    p.prefix = pre + 2 * (n + 1);
    HIP_TRY(launch_batch_pass<T>(2, p, L.prefix[2][n], 0, st));
    p.prefix = pre + 1 * (n + 1);
    HIP_TRY(launch_batch_pass<T>(1, p, L.prefix[1][n], 1, st));
    p.prefix = pre + 3 * (n + 1);
    HIP_TRY(launch_batch_pass<T>(3, p, L.prefix[3][n], 0, st));
    return MM_OK;
}

template <typename T>
mm_status batch_rk4_step(mm_batch* b, double dt, hipStream_t st)
{
    const BatchLayout& L = b->L;
    T* mn = b->at<T>(L.o_mn);
    T* ma = b->at<T>(L.o_ma);
    T* mb = b->at<T>(L.o_mb);
    T* acc = b->at<T>(L.o_acc);
    T* hd = b->at<T>(L.o_hd);
    T* src[4] = {mn, ma, mb, ma};
    T* dst[4] = {ma, mb, ma, mn};
    const bool with_demag = !(b->flags & MM_NO_DEMAG);
    BatchClass<T> bc{};
    bc.d = b->at<BatchDesc>(L.o_desc);
    const int* cints = b->at<int>(L.o_classes);
    BatchLlg<T> g{};
    g.mn = mn;
    g.acc = acc;
    g.hd = with_demag ? hd : nullptr;
    for (int stg = 0; stg < 4; ++stg) {
        if (with_demag)
            if (mm_status r = batch_demag<T>(b, src[stg], st); r != MM_OK) return r;
        g.ms = src[stg];
        g.out = dst[stg];
        g.stage = stg + 1;
        for (const BatchClassHost& c : L.classes) {
            if (c.kind != kBatchLlgKind) continue;
            bc.members = cints + c.off;
            bc.prefix = cints + c.off + c.members.size();
            bc.nmem = (int)c.members.size();
            HIP_TRY(launch_batch_llg<T>(c.P, bc, c.prefix.back(), g, st));
        }
    }
    return MM_OK;
}

void batch_drop_graph(mm_batch* b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->graph_valid = false;
}

// Each grid's gamma Ms dt / (1 + alpha^2), evaluated as the single-grid step does,
// goes into its descriptor when dt changes (before any graph capture).
mm_status batch_set_dt(mm_batch* b, double dt)
{
    if (b->desc_dt == dt) return MM_OK;
    for (int s = 0; s < b->n; ++s) {
        const mm_material& m = b->mats[s];
        b->L.desc[s].gdt = m.gamma * m.Ms * dt / (1.0 + m.alpha * m.alpha);
    }
    HIP_TRY(hipMemcpyAsync(b->at<char>(b->L.o_desc), b->L.desc.data(), b->n * sizeof(BatchDesc),
                           hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->desc_dt = dt;
    return MM_OK;
}

template <typename T>
mm_status batch_step_impl(mm_batch* b, int64_t nsteps, double dt)
{
    hipStream_t st = b->stream;
    if (mm_status r = batch_set_dt(b, dt); r != MM_OK) return r;
    if (!(b->flags & MM_USE_GRAPH)) {
        for (int64_t q = 0; q < nsteps; ++q) {
            mm_status r = batch_rk4_step<T>(b, dt, st);
            if (r != MM_OK) return r;
        }
        return MM_OK;
    }
    const int chunk = 8;
    if (!b->graph_valid || b->graph_dt != dt) {
        batch_drop_graph(b);
        HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        mm_status r = MM_OK;
        for (int q = 0; q < chunk && r == MM_OK; ++q) r = batch_rk4_step<T>(b, dt, b->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
        if (r != MM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return r;
        }
        if (e != hipSuccess) return fail(MM_EHIP, "graph capture: %s", hipGetErrorString(e));
        b->graph = g;
        HIP_TRY(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
        b->graph_valid = true;
        b->graph_dt = dt;
        b->graph_chunk = chunk;
    }
    int64_t q = 0;
    for (; q + b->graph_chunk <= nsteps; q += b->graph_chunk) HIP_TRY(hipGraphLaunch(b->gexec, st));
    for (; q < nsteps; ++q) {
        mm_status r = batch_rk4_step<T>(b, dt, st);
        if (r != MM_OK) return r;
    }
    return MM_OK;
}

template <typename T>
mm_status batch_set_m_impl(mm_batch* b, const void* m, int on_device)
{
    const BatchLayout& L = b->L;
    hipStream_t st = b->stream;
    T* mn = b->at<T>(L.o_mn);
    HIP_TRY(hipMemcpyAsync(mn, m, (size_t)L.vec_elems * sizeof(T),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    unsigned int* bad = reinterpret_cast<unsigned int*>(b->at<char>(L.o_flags));
    HIP_TRY(hipMemsetAsync(bad, 0, sizeof(unsigned int), st));
    for (int s = 0; s < b->n; ++s)
        HIP_TRY(launch_normalize<T>(mn + L.desc[s].moff, L.plans[s].N, bad, st));
    unsigned int nbad = 0;
    HIP_TRY(hipMemcpyAsync(&nbad, bad, sizeof nbad, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (nbad) {
        b->has_m = false;
        return fail(MM_EINVAL, "m has %u zero-length or non-finite cells", nbad);
    }
    b->has_m = true;
    return MM_OK;
}

// One term of every grid's effective field at the current m, A/m, written grid
// by grid like m: the demag passes of the whole batch, then the local terms of
// each grid.
template <typename T>
mm_status batch_field_impl(mm_batch* b, int term, void* out, int on_device)
{
    const BatchLayout& L = b->L;
    hipStream_t st = b->stream;
    T* mn = b->at<T>(L.o_mn);
    const bool with_demag = !(b->flags & MM_NO_DEMAG);
    if (with_demag && (term == MM_H_DEMAG || term == MM_H_EFF))
        if (mm_status r = batch_demag<T>(b, mn, st); r != MM_OK) return r;
    T* dst = on_device ? static_cast<T*>(out) : b->at<T>(L.o_mb);
    T* hd = b->at<T>(L.o_hd);
    for (int s = 0; s < b->n; ++s) {
        const Plan& p = L.plans[s];
        const BatchDesc& d = L.desc[s];
        LlgArgs<T> a{};
        a.nx = p.nx;
        a.ny = p.ny;
        a.nz = p.nz;
        a.N = p.N;
        a.cex = (T)d.cex;
        a.can = (T)d.can;
        a.hx = (T)d.hred[0];
        a.hy = (T)d.hred[1];
        a.hz = (T)d.hred[2];
        a.ms = mn + d.moff;
        a.mn = a.ms;
        a.hd = with_demag ? hd + d.moff : nullptr;
        HIP_TRY(launch_field_term<T>(a, term, (T)b->mats[s].Ms, dst + d.moff, st));
    }
    if (!on_device) {
        HIP_TRY(hipMemcpyAsync(out, dst, (size_t)L.vec_elems * sizeof(T), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    return MM_OK;
}

// ---------------------------------------------------------------- batch autotuner
// Candidate layouts of a batch: 7-smooth padding with the runtime-radix passes
// (the default), power-of-two padding with the runtime-radix passes, and
// power-of-two padding with the size-class passes when every padded length has
// one.  A candidate whose padded sizes equal an earlier one's is dropped.
std::vector<mm_options> batch_tune_candidates(int32_t n, const mm_grid* grids, const mm_options* opt)
{
    const uint32_t base = opt->flags & ~(uint32_t)(MM_AUTOTUNE | MM_POW2_PAD | MM_FAST_PAD | MM_GENERIC_FFT);
    const uint32_t variants[4] = {base, base | MM_POW2_PAD | MM_GENERIC_FFT, base | MM_POW2_PAD,
                                  base | MM_FAST_PAD};
    std::vector<mm_options> out;
    std::vector<BatchLayout> kept;
    for (uint32_t f : variants) {
        mm_options c = *opt;
        c.px = c.py = c.pz = 0;
        c.flags = f;
        BatchLayout L;
        if (batch_layout(n, grids, &c, &L) != MM_OK) continue;
        if ((f & (MM_POW2_PAD | MM_FAST_PAD)) && !(f & MM_GENERIC_FFT) && !L.fast) continue;
        bool dup = false;
        for (const BatchLayout& K : kept) {
            if (K.fast != L.fast) continue;
            bool same = true;
            for (int s = 0; s < n && same; ++s)
                same = K.plans[s].Px == L.plans[s].Px && K.plans[s].Py == L.plans[s].Py &&
                       K.plans[s].Pz == L.plans[s].Pz;
            dup = dup || same;
        }
        if (dup) continue;
        out.push_back(c);
        kept.push_back(std::move(L));
    }
    return out;
}

// Mean time of one field evaluation of every grid, on zero-filled state,
// spectra and twiddles (the passes' cost does not depend on the values).
template <typename T>
mm_status time_batch_demag(mm_batch* b, double* ms_out)
{
    const BatchLayout& L = b->L;
    hipStream_t st = b->stream;
    HIP_TRY(hipMemsetAsync(b->at<char>(L.o_mn), 0, L.o_flags - L.o_mn, st));
    const T* mn = b->at<T>(L.o_mn);
    for (int w = 0; w < 2; ++w)
        if (mm_status r = batch_demag<T>(b, mn, st); r != MM_OK) return r;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int reps = 5;
    mm_status r = MM_OK;
    hipError_t e = hipEventRecord(e0, st);
    for (int q = 0; q < reps && r == MM_OK && e == hipSuccess; ++q) r = batch_demag<T>(b, mn, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != MM_OK) return r;
    if (e != hipSuccess) return fail(MM_EHIP, "batch autotune timing: %s", hipGetErrorString(e));
    *ms_out = ms / reps;
    return MM_OK;
}

// ---------------------------------------------------------------- autotuner
struct TuneChoice {
    int px, py, pz, generic, threads, xl;
    double ms;
    int fused;  // 1: the fused y-z pass, 2: one work-group for the whole evaluation
};

std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune_cache;
bool g_tune_file_loaded = false;

// The GPU the current device is: architecture, name and compute units (a tuned
// schedule is only reused on the same kind of GPU).
std::string device_tag()
{
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string tag = std::string(prop.gcnArchName) + "/" + prop.name + "/" + std::to_string(prop.multiProcessorCount);
    for (char& ch : tag)
        if (ch == ' ' || ch == '\t') ch = '_';
    return tag;
}

std::string tune_key(const mm_grid* g, const mm_options* o)
{
    std::ostringstream k;
    k << device_tag() << ":" << g->nx << "x" << g->ny << "x" << g->nz << ":p" << o->prec << ":d" << ((o->flags & MM_NO_DEMAG) ? 0 : 1)
      << ":b" << ((o->flags >> 7) & 7) << "i" << o->images << ":t" << ((o->flags & MM_NEWELL) ? 1 : 0)
      << ":f" << ((o->flags & MM_FUSED_YZ) ? 1 : 0) << ((o->flags & MM_ONE_WG) ? 1 : 0);
    return k.str();
}

void tune_file_load()
{
    if (g_tune_file_loaded) return;
    g_tune_file_loaded = true;
    const char* path = getenv("MMAG_TUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    std::string key;
    TuneChoice c;
    while (f >> key >> c.px >> c.py >> c.pz >> c.generic >> c.threads >> c.xl >> c.ms >> c.fused)
        g_tune_cache[key] = c;
}

void tune_file_append(const std::string& key, const TuneChoice& c)
{
    const char* path = getenv("MMAG_TUNE_CACHE");
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    f << key << " " << c.px << " " << c.py << " " << c.pz << " " << c.generic << " " << c.threads << " "
      << c.xl << " " << c.ms << " " << c.fused << "\n";
}

int next_pow2_at_least(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

template <typename T>
mm_status time_demag(mm_sim* s, hipStream_t st, double* ms_out)
{
    const Plan& p = s->p;
    T* mn = s->at<T>(p.o_mn);
    T* hd = s->at<T>(p.o_hd);
    HIP_TRY(hipMemsetAsync(mn, 0, 3 * (size_t)p.N * sizeof(T), st));
    for (int w = 0; w < 2; ++w) {
        mm_status r = demag<T>(s, mn, hd, st);
        if (r != MM_OK) return r;
    }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int reps = 5;
    HIP_TRY(hipEventRecord(e0, st));
    for (int q = 0; q < reps; ++q) {
        mm_status r = demag<T>(s, mn, hd, st);
        if (r != MM_OK) return r;
    }
    HIP_TRY(hipEventRecord(e1, st));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_out = ms / reps;
    return MM_OK;
}

// Candidate schedules of a grid: padded sizes (7-smooth default vs the power of
// two that the specialised passes handle), specialised vs runtime-radix
// passes, and the runtime-radix work-group size.
std::vector<mm_options> tune_candidates(const mm_grid* g, const mm_options* o)
{
    // a periodic axis has one size, its period (requested as 0)
    const bool perx = o->flags & MM_PERIODIC_X, pery = o->flags & MM_PERIODIC_Y;
    const bool perz = o->flags & MM_PERIODIC_Z;
    std::vector<int> pxs{perx ? 0 : auto_pad(g->nx)}, pys{pery ? 0 : auto_pad(g->ny)};
    std::vector<int> pzs{perz ? 0 : (g->nz == 1 ? 1 : auto_pad(g->nz))};
    auto add_pow2 = [](std::vector<int>& v, int n) {
        const int q = next_pow2_at_least(2 * n - 1);
        if (q != v[0] && q <= 4096) v.push_back(q);
    };
    auto add_fast = [](std::vector<int>& v, int n) {  // a mixed-radix length with specialised passes
        const int q = fast_pad_length(2 * n - 1, true);
        if (std::find(v.begin(), v.end(), q) == v.end() && q <= 4096) v.push_back(q);
    };
    if (!perx) add_pow2(pxs, g->nx);
    if (!pery) add_pow2(pys, g->ny);
    if (g->nz > 1 && !perz) add_pow2(pzs, g->nz);
    if (!perx) add_fast(pxs, g->nx);
    if (!pery) add_fast(pys, g->ny);
    std::vector<mm_options> out;
    for (int px : pxs)
        for (int py : pys)
            for (int pz : pzs)
                for (int generic = 0; generic < 2; ++generic)
                    for (int threads : {256, 512})
                        for (int xl : {8, 4}) {
                        if (!generic && threads == 512) continue;  // the specialised passes fix their shape
                        if (generic && xl == 4) continue;          // only the specialised x passes use it
                        mm_options c = *o;
                        c.px = px;
                        c.py = py;
                        c.pz = pz;
                        c.threads = threads;
                        c.x_lines = xl;
                        c.flags = (o->flags & ~(MM_AUTOTUNE | MM_USE_GRAPH | MM_GENERIC_FFT | MM_POW2_PAD |
                                                MM_FAST_PAD)) |
                                  (generic ? MM_GENERIC_FFT : 0u);
                        Plan p;
                        if (build_plan(g, &c, &p) != MM_OK) continue;
                        out.push_back(c);
                        mm_options f = c;  // the same schedule with the fused y-z pass, where it applies
                        f.flags |= MM_FUSED_YZ;
                        if (!(c.flags & MM_FUSED_YZ) && build_plan(g, &f, &p) == MM_OK && p.yz) out.push_back(f);
                        mm_options w = c;  // one work-group for the whole evaluation, where it fits
                        w.flags = (w.flags & ~MM_FUSED_YZ) | MM_ONE_WG;
                        if (!(c.flags & MM_ONE_WG) && build_plan(g, &w, &p) == MM_OK && p.wg1) out.push_back(w);
                    }
    return out;
}

// Times every candidate on one workspace: the caller's when it holds every
// candidate (mm_workspace_query with MM_AUTOTUNE returns that size), else one
// allocated here for the largest.  Candidates that share padded sizes share the
// workspace layout, the twiddles and the kernel spectrum, which are built once
// per padded size; the schedule options (pass family, work-group size, x lines,
// fused y-z or one work-group) are then switched on the same handle.
mm_status autotune(const mm_grid* g, const mm_material* mat, const mm_options* o, hipStream_t st,
                   void* d_ws, size_t ws_bytes, TuneChoice* best, int* ncand)
{
    best->ms = 1e300;
    *ncand = 0;
    std::vector<mm_options> cands;
    std::vector<Plan> plans;
    size_t need = 0;
    for (const mm_options& c : tune_candidates(g, o)) {
        Plan p;
        if (build_plan(g, &c, &p) != MM_OK) continue;
        cands.push_back(c);
        plans.push_back(p);
        need = std::max(need, p.total);
    }
    void* w = d_ws;
    bool own = false;
    if (!w || ws_bytes < need) {
        if (hipMalloc(&w, need) != hipSuccess) return fail(MM_ENOMEM, "autotune workspace of %zu bytes", need);
        own = true;
    }
    std::vector<bool> done(cands.size(), false);
    for (size_t i = 0; i < cands.size(); ++i) {
        if (done[i]) continue;
        mm_sim* t = nullptr;
        mm_status r = mm_create(g, mat, &cands[i], w, need, st, &t);
        for (size_t j = i; j < cands.size(); ++j) {
            const Plan& pi = plans[i];
            const Plan& pj = plans[j];
            if (done[j] || pj.Px != pi.Px || pj.Py != pi.Py || pj.Pz != pi.Pz || pj.total != pi.total ||
                pj.o_kern != pi.o_kern || pj.o_S != pi.o_S || pj.o_twz != pi.o_twz || pj.zd != pi.zd ||
                pj.fs != pi.fs)
                continue;
            done[j] = true;
            if (r != MM_OK) continue;
            t->p = pj;  // same layout, spectrum and twiddles; another schedule
            t->flags = cands[j].flags;
            double ms = 0;
            mm_status rj = pj.prec == MM_F32 ? time_demag<float>(t, st, &ms) : time_demag<double>(t, st, &ms);
            if (rj != MM_OK) continue;
            ++*ncand;
            const mm_options& c = cands[j];
            if (ms < best->ms)
                *best = TuneChoice{c.px, c.py, c.pz, (c.flags & MM_GENERIC_FFT) ? 1 : 0, c.threads, c.x_lines, ms,
                                   (c.flags & MM_ONE_WG) ? 2 : ((c.flags & MM_FUSED_YZ) ? 1 : 0)};
        }
        if (t) mm_destroy(t);
    }
    if (own) (void)hipFree(w);
    if (*ncand == 0) return fail(MM_ENOTSUP, "no schedule of this grid could be built");
    return MM_OK;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

mm_status mm_workspace_query(const mm_grid* grid, const mm_options* opt, size_t* bytes)
{
    if (!bytes) return fail(MM_EINVAL, "bytes is NULL");
    Plan p;
    mm_status st = build_plan(grid, opt, &p);
    if (st != MM_OK) return st;
    *bytes = p.total;
    if (opt && (opt->flags & MM_AUTOTUNE))  // room for whichever schedule wins
        for (const mm_options& c : tune_candidates(grid, opt)) {
            Plan q;
            if (build_plan(grid, &c, &q) == MM_OK) *bytes = std::max(*bytes, q.total);
        }
    return MM_OK;
}

mm_status mm_create(const mm_grid* grid, const mm_material* mat, const mm_options* opt,
                    void* d_workspace, size_t ws_bytes, void* stream, mm_sim** out)
{
    if (!out) return fail(MM_EINVAL, "out is NULL");
    *out = nullptr;
    if (opt && (opt->flags & MM_AUTOTUNE)) {
        Plan probe;
        mm_status st0 = build_plan(grid, opt, &probe);  // argument checks first
        if (st0 != MM_OK) return st0;
        if (!check_material(mat))
            return fail(MM_EINVAL, "material needs Ms > 0, A >= 0, alpha >= 0, gamma > 0, all finite");
        const std::string key = tune_key(grid, opt);
        TuneChoice ch{};
        int ncand = 0;
        bool have = false;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            tune_file_load();
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                ch = it->second;
                have = true;
            }
        }
        if (!have) {
            mm_status r = autotune(grid, mat, opt, as_stream(stream), d_workspace, ws_bytes, &ch, &ncand);
            if (r != MM_OK) return r;
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_cache[key] = ch;
            tune_file_append(key, ch);
        }
        mm_options c = *opt;
        c.px = ch.px;
        c.py = ch.py;
        c.pz = ch.pz;
        c.threads = ch.threads;
        c.x_lines = ch.xl;
        c.flags = (opt->flags & ~(MM_AUTOTUNE | MM_GENERIC_FFT)) | (ch.generic ? MM_GENERIC_FFT : 0u) |
                  (ch.fused == 1 ? MM_FUSED_YZ : 0u) | (ch.fused == 2 ? MM_ONE_WG : 0u);
        mm_status r = mm_create(grid, mat, &c, d_workspace, ws_bytes, stream, out);
        if (r == MM_OK) {
            (*out)->tuned = 1;
            (*out)->tune_candidates = ncand;
            (*out)->tuned_ms = ch.ms;
        }
        return r;
    }
    Plan p;
    mm_status st = build_plan(grid, opt, &p);
    if (st != MM_OK) return st;
    if (!check_material(mat))
        return fail(MM_EINVAL, "material needs Ms > 0, A >= 0, alpha >= 0, gamma > 0, all finite");
    if (d_workspace && ws_bytes < p.total)
        return fail(MM_EINVAL, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, p.total);
    if (d_workspace && (reinterpret_cast<uintptr_t>(d_workspace) & 255))
        return fail(MM_EINVAL, "workspace must be 256-byte aligned");
    mm_sim* s = new mm_sim();
    s->p = p;
    s->mat = *mat;
    s->cell = grid->cell;
    s->flags = opt ? opt->flags : 0;
    s->stream = as_stream(stream);
    s->alpha = mat->alpha;
    s->hext[0] = s->hext[1] = s->hext[2] = 0.0;
    s->prof_kernel = -1;
    s->prof_every = 1;
    if (d_workspace) {
        s->ws = static_cast<char*>(d_workspace);
    } else {
        void* w = nullptr;
        hipError_t e = hipMalloc(&w, p.total);
        if (e != hipSuccess) {
            delete s;
            return fail(MM_ENOMEM, "hipMalloc(%zu): %s", p.total, hipGetErrorString(e));
        }
        s->ws = static_cast<char*>(w);
        s->own_ws = true;
    }
    hipError_t e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (s->own_ws) (void)hipFree(s->ws);
        delete s;
        return fail(MM_EHIP, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    // this device's copy of the static adjoint scratch (mm_backward_noalloc reports
    // a failure here; nothing else uses it)
    s->device = 0;
    s->scratch = nullptr;
    if ((e = hipGetDevice(&s->device)) != hipSuccess)
        s->scratch_err = std::string("hipGetDevice: ") + hipGetErrorString(e);
    else if (scratch_address(s->device, &s->scratch) != MM_OK)
        s->scratch_err = g_err;
    st = p.prec == MM_F32 ? build_kernel_spectrum<float>(s, s->stream)
                          : build_kernel_spectrum<double>(s, s->stream);
    if (st != MM_OK) {
        std::string keep = g_err;
        mm_destroy(s);
        g_err = keep;
        return st;
    }
    *out = s;
    return MM_OK;
}

mm_status mm_destroy(mm_sim* s)
{
    if (!s) return MM_OK;
    (void)hipStreamSynchronize(s->stream);
    drop_graph(s);
    drop_bwd_graphs(s);
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    if (s->own_ws) (void)hipFree(s->ws);
    delete s;
    return MM_OK;
}

mm_status mm_set_stream(mm_sim* s, void* stream)
{
    if (!s) return fail(MM_EINVAL, "sim is NULL");
    s->stream = as_stream(stream);
    return MM_OK;
}

mm_status mm_set_m(mm_sim* s, const void* m, int on_device)
{
    if (!s || !m) return fail(MM_EINVAL, "sim or m is NULL");
    return s->p.prec == MM_F32 ? set_m_impl<float>(s, m, on_device) : set_m_impl<double>(s, m, on_device);
}

mm_status mm_get_m(mm_sim* s, void* out, int on_device)
{
    if (!s || !out) return fail(MM_EINVAL, "sim or out is NULL");
    if (!s->has_m) return fail(MM_ESTATE, "m has not been set");
    const size_t bytes = 3 * (size_t)s->p.N * s->p.esz;
    HIP_TRY(hipMemcpyAsync(out, s->at<char>(s->p.o_mn), bytes,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->stream));
    if (!on_device) HIP_TRY(hipStreamSynchronize(s->stream));
    return MM_OK;
}

mm_status mm_set_hext(mm_sim* s, const double h[3])
{
    if (!s || !h) return fail(MM_EINVAL, "sim or h is NULL");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(h[a])) return fail(MM_EINVAL, "applied field must be finite");
    // captured steps hold the field as a kernel argument: a new value retires them
    for (int a = 0; a < 3; ++a) {
        if (s->hext[a] != h[a]) s->graph_valid = false;
        s->hext[a] = h[a];
    }
    return MM_OK;
}

mm_status mm_set_alpha(mm_sim* s, double alpha)
{
    if (!s) return fail(MM_EINVAL, "sim is NULL");
    if (!(alpha >= 0) || !std::isfinite(alpha)) return fail(MM_EINVAL, "alpha must be finite and >= 0");
    if (s->alpha != alpha) s->graph_valid = false;
    s->alpha = alpha;
    return MM_OK;
}

mm_status mm_set_ku_map(mm_sim* s, const void* ku, int on_device)
{
    if (!s) return fail(MM_EINVAL, "sim is NULL");
    // captured steps read the map from the handle's own buffer: only switching it on
    // or off retires them
    if (!ku) {
        if (s->has_ku_map) s->graph_valid = false;
        s->has_ku_map = false;
        return MM_OK;
    }
    const Plan& p = s->p;
    const size_t n = (size_t)p.N;
    const double f = 2.0 / (kMu0 * s->mat.Ms * s->mat.Ms);  // Ku -> reduced 2 Ku / (mu0 Ms^2)
    if (p.prec == MM_F32) {
        std::vector<float> h(n);
        if (on_device) {
            HIP_TRY(hipMemcpy(h.data(), ku, n * 4, hipMemcpyDeviceToHost));
        } else {
            memcpy(h.data(), ku, n * 4);
        }
        for (auto& v : h) {
            if (!std::isfinite(v)) return fail(MM_EINVAL, "Ku map must be finite");
            v = (float)(v * f);
        }
        HIP_TRY(hipMemcpyAsync(s->at<char>(p.o_ku), h.data(), n * 4, hipMemcpyHostToDevice, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    } else {
        std::vector<double> h(n);
        if (on_device) {
            HIP_TRY(hipMemcpy(h.data(), ku, n * 8, hipMemcpyDeviceToHost));
        } else {
            memcpy(h.data(), ku, n * 8);
        }
        for (auto& v : h) {
            if (!std::isfinite(v)) return fail(MM_EINVAL, "Ku map must be finite");
            v = v * f;
        }
        HIP_TRY(hipMemcpyAsync(s->at<char>(p.o_ku), h.data(), n * 8, hipMemcpyHostToDevice, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    if (!s->has_ku_map) s->graph_valid = false;
    s->has_ku_map = true;
    return MM_OK;
}

mm_status mm_step(mm_sim* s, int64_t nsteps, double dt)
{
    if (!s) return fail(MM_EINVAL, "sim is NULL");
    if (nsteps < 0) return fail(MM_EINVAL, "nsteps must be >= 0");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(MM_EINVAL, "dt must be finite and > 0");
    if (!s->has_m) return fail(MM_ESTATE, "mm_step before mm_set_m");
    return s->p.prec == MM_F32 ? step_impl<float>(s, nsteps, dt) : step_impl<double>(s, nsteps, dt);
}

mm_status mm_step_euler(mm_sim* s, int64_t nsteps, double dt)
{
    if (!s) return fail(MM_EINVAL, "sim is NULL");
    if (nsteps < 0) return fail(MM_EINVAL, "nsteps must be >= 0");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(MM_EINVAL, "dt must be finite and > 0");
    if (!s->has_m) return fail(MM_ESTATE, "mm_step_euler before mm_set_m");
    return s->p.prec == MM_F32 ? euler_steps<float>(s, nsteps, dt) : euler_steps<double>(s, nsteps, dt);
}

mm_status mm_run_schedule(mm_sim* s, const mm_segment* segs, int32_t nseg, int32_t method,
                          double dt, int64_t every, double* trace, int64_t trace_cap, int64_t* rows)
{
    if (rows) *rows = 0;
    if (!s) return fail(MM_EINVAL, "sim is NULL");
    if (nseg < 0 || (nseg > 0 && !segs)) return fail(MM_EINVAL, "segs is NULL or nseg < 0");
    if (method != MM_RK4 && method != MM_EULER) return fail(MM_EINVAL, "method must be MM_RK4 or MM_EULER");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(MM_EINVAL, "dt must be finite and > 0");
    if (every < 1) return fail(MM_EINVAL, "every must be >= 1");
    int64_t total = 0;
    for (int q = 0; q < nseg; ++q) {
        const mm_segment& g = segs[q];
        if (g.steps < 0 || g.steps > INT64_MAX - total) return fail(MM_EINVAL, "piece %d: bad step count", q);
        for (int c = 0; c < 3; ++c)
            if (!std::isfinite(g.h0[c]) || !std::isfinite(g.h1[c]))
                return fail(MM_EINVAL, "piece %d: applied field must be finite", q);
        if (!(g.alpha >= 0) || !std::isfinite(g.alpha))
            return fail(MM_EINVAL, "piece %d: alpha must be finite and >= 0", q);
        total += g.steps;
    }
    const int64_t due = total / every;
    if (due > 0 && (!trace || trace_cap < due))
        return fail(MM_EINVAL, "the trace needs %lld rows, trace_cap is %lld", (long long)due,
                    (long long)trace_cap);
    if (!s->has_m) return fail(MM_ESTATE, "mm_run_schedule before mm_set_m");
    return s->p.prec == MM_F32 ? schedule_impl<float>(s, segs, nseg, method, dt, every, trace, rows)
                               : schedule_impl<double>(s, segs, nseg, method, dt, every, trace, rows);
}

mm_status mm_get_field(mm_sim* s, int32_t term, void* out, int on_device)
{
    if (!s || !out) return fail(MM_EINVAL, "sim or out is NULL");
    if (term < 0 || term > 4) return fail(MM_EINVAL, "term must be 0..4");
    if (!s->has_m) return fail(MM_ESTATE, "m has not been set");
    return s->p.prec == MM_F32 ? field_impl<float>(s, term, out, on_device)
                               : field_impl<double>(s, term, out, on_device);
}

mm_status mm_get_energy(mm_sim* s, double out[5])
{
    if (!s || !out) return fail(MM_EINVAL, "sim or out is NULL");
    if (!s->has_m) return fail(MM_ESTATE, "m has not been set");
    double r[kRedSlots];
    mm_status st = s->p.prec == MM_F32 ? reduce_impl<float>(s, r) : reduce_impl<double>(s, r);
    if (st != MM_OK) return st;
    if (r[7] != 0.0) return fail(MM_ENONFINITE, "m holds %.0f non-finite cells", r[7]);
    const double Ms = s->mat.Ms, V = s->cell * s->cell * s->cell;
    out[0] = s->mat.A * s->cell * r[0];                // A delta sum over pairs |m_a - m_b|^2
    out[1] = 0.5 * kMu0 * Ms * Ms * V * r[1];          // sum Ku (my^2 + mz^2) V
    out[2] = -0.5 * kMu0 * Ms * Ms * V * r[2];         // -mu0/2 sum M.H_d V
    out[3] = -kMu0 * Ms * Ms * V * r[3];               // -mu0 sum M.H_ext V
    out[4] = out[0] + out[1] + out[2] + out[3];
    return MM_OK;
}

mm_status mm_get_mean_m(mm_sim* s, double out[3])
{
    if (!s || !out) return fail(MM_EINVAL, "sim or out is NULL");
    if (!s->has_m) return fail(MM_ESTATE, "m has not been set");
    double r[kRedSlots];
    const uint32_t keep = s->flags;
    s->flags |= MM_NO_DEMAG;  // the mean needs no field
    mm_status st = s->p.prec == MM_F32 ? reduce_impl<float>(s, r) : reduce_impl<double>(s, r);
    s->flags = keep;
    if (st != MM_OK) return st;
    if (r[7] != 0.0) return fail(MM_ENONFINITE, "m holds %.0f non-finite cells", r[7]);
    for (int a = 0; a < 3; ++a) out[a] = r[4 + a] / (double)s->p.N;
    return MM_OK;
}

mm_status mm_get_max_torque(mm_sim* s, double* out)
{
    if (!s || !out) return fail(MM_EINVAL, "sim or out is NULL");
    if (!s->has_m) return fail(MM_ESTATE, "m has not been set");
    double r[kRedSlots];
    mm_status st = s->p.prec == MM_F32 ? reduce_impl<float>(s, r) : reduce_impl<double>(s, r);
    if (st != MM_OK) return st;
    if (r[7] != 0.0) return fail(MM_ENONFINITE, "m holds %.0f non-finite cells", r[7]);
    *out = s->mat.Ms * r[8];  // reduced torque |m x h| -> A/m
    return MM_OK;
}

mm_status mm_get_plan(mm_sim* s, mm_plan_info* out)
{
    if (!s || !out) return fail(MM_EINVAL, "sim or out is NULL");
    out->px = s->p.Px;
    out->py = s->p.Py;
    out->pz = s->p.Pz;
    out->hx = s->p.hx;
    out->ncomp = s->p.ncomp;
    out->threads = s->p.nt;
    out->spectrum_elems = (int64_t)s->p.kplanes * s->p.oct_elems;
    out->passes = s->p.wg1 ? 1 : ((s->p.three_d && !s->p.yz && !s->p.zd) ? 5 : 3);
    out->kernel_imag_ratio = s->imag_ratio;
    out->generic_fft = (s->flags & MM_GENERIC_FFT) ? 1 : 0;
    out->tuned = s->tuned;
    out->candidates = s->tune_candidates;
    out->tuned_demag_ms = s->tuned_ms;
    out->x_lines = s->p.xl;
    out->x_lines_inv = s->p.xl_inv;
    out->two_plane = s->p.zd ? 1 : 0;
    out->fused_stage = s->p.fs ? 1 : 0;
    return MM_OK;
}

mm_status mm_get_kernel_spectrum(mm_sim* s, void* out, int on_device)
{
    if (!s || !out) return fail(MM_EINVAL, "sim or out is NULL");
    if (s->flags & MM_NO_DEMAG) return fail(MM_ESTATE, "handle was created without demag");
    const size_t bytes = (size_t)s->p.kplanes * s->p.oct_elems * s->p.esz;
    HIP_TRY(hipMemcpyAsync(out, s->at<char>(s->p.o_kern), bytes,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return MM_OK;
}

mm_status mm_demag_tensor(int32_t nx, int32_t ny, int32_t nz, double* d_out, void* stream)
{
    if (nx < 1 || ny < 1 || nz < 1 || !d_out) return fail(MM_EINVAL, "dims must be >= 1 and d_out non-NULL");
    if ((int64_t)(2 * nx - 1) * (2 * ny - 1) * (2 * nz - 1) > ((int64_t)1 << 34))
        return fail(MM_ENOTSUP, "tensor table too large");
    HIP_TRY(launch_tensor_table(d_out, 0, nx, ny, nz, as_stream(stream)));
    return MM_OK;
}

mm_status mm_demag_tensor_newell(int32_t nx, int32_t ny, int32_t nz, double* d_out, void* stream)
{
    if (nx < 1 || ny < 1 || nz < 1 || !d_out) return fail(MM_EINVAL, "dims must be >= 1 and d_out non-NULL");
    if ((int64_t)(2 * nx - 1) * (2 * ny - 1) * (2 * nz - 1) > ((int64_t)1 << 34))
        return fail(MM_ENOTSUP, "tensor table too large");
    HIP_TRY(launch_tensor_table(d_out, 1, nx, ny, nz, as_stream(stream)));
    return MM_OK;
}

mm_status mm_rollout(mm_sim* s, int64_t nsteps, double dt, int64_t ckpt_every, void* d_ckpt)
{
    if (!s || !d_ckpt) return fail(MM_EINVAL, "sim or checkpoint buffer is NULL");
    if (nsteps < 1 || ckpt_every < 1) return fail(MM_EINVAL, "nsteps and ckpt_every must be >= 1");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(MM_EINVAL, "dt must be finite and > 0");
    if (!s->has_m) return fail(MM_ESTATE, "mm_rollout before mm_set_m");
    return s->p.prec == MM_F32 ? rollout_impl<float>(s, nsteps, dt, ckpt_every, (float*)d_ckpt)
                               : rollout_impl<double>(s, nsteps, dt, ckpt_every, (double*)d_ckpt);
}

mm_status mm_normalize_backward(mm_sim* s, const void* d_v, const void* d_gu, void* d_gv)
{
    if (!s || !d_v || !d_gu || !d_gv) return fail(MM_EINVAL, "NULL argument");
    if (s->p.prec == MM_F32)
        HIP_TRY(launch_normalize_vjp<float>(static_cast<const float*>(d_v), static_cast<const float*>(d_gu),
                                            static_cast<float*>(d_gv), s->p.N, s->stream));
    else
        HIP_TRY(launch_normalize_vjp<double>(static_cast<const double*>(d_v), static_cast<const double*>(d_gu),
                                             static_cast<double*>(d_gv), s->p.N, s->stream));
    return MM_OK;
}

mm_status mm_adjoint_workspace_query(mm_sim* s, int64_t ckpt_every, size_t* bytes)
{
    if (!s || !bytes) return fail(MM_EINVAL, "sim or bytes is NULL");
    if (ckpt_every < 1) return fail(MM_EINVAL, "ckpt_every must be >= 1");
    *bytes = adj_bytes(s->p, ckpt_every);
    return MM_OK;
}

mm_status mm_backward(mm_sim* s, int64_t nsteps, double dt, int64_t ckpt_every, const void* d_ckpt,
                      const void* d_lam_final, double* d_dku, void* d_dm0, void* d_adj_ws,
                      size_t adj_ws_bytes)
{
    if (!s || !d_ckpt || !d_lam_final || !d_dku || !d_adj_ws)
        return fail(MM_EINVAL, "NULL argument");
    if (nsteps < 1 || ckpt_every < 1) return fail(MM_EINVAL, "nsteps and ckpt_every must be >= 1");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(MM_EINVAL, "dt must be finite and > 0");
    if (!s->has_m) return fail(MM_ESTATE, "mm_backward before mm_set_m");
    if (adj_ws_bytes < adj_bytes(s->p, ckpt_every))
        return fail(MM_EINVAL, "adjoint workspace of %zu bytes is smaller than the %zu needed", adj_ws_bytes,
                    adj_bytes(s->p, ckpt_every));
    if (reinterpret_cast<uintptr_t>(d_adj_ws) & 255) return fail(MM_EINVAL, "adjoint workspace must be 256-byte aligned");
    return s->p.prec == MM_F32
               ? backward_impl<float>(s, nsteps, dt, ckpt_every, (const float*)d_ckpt,
                                      (const float*)d_lam_final, d_dku, (float*)d_dm0, (char*)d_adj_ws, true)
               : backward_impl<double>(s, nsteps, dt, ckpt_every, (const double*)d_ckpt,
                                       (const double*)d_lam_final, d_dku, (double*)d_dm0,
                                       (char*)d_adj_ws, true);
}

mm_status mm_backward_noalloc(mm_sim* s, int64_t nsteps, double dt, int64_t ckpt_every, const void* d_ckpt,
                              const void* d_lam_final, double* d_dku, void* d_dm0)
{
    if (!s || !d_ckpt || !d_lam_final || !d_dku) return fail(MM_EINVAL, "NULL argument");
    if (nsteps < 1 || ckpt_every < 1) return fail(MM_EINVAL, "nsteps and ckpt_every must be >= 1");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(MM_EINVAL, "dt must be finite and > 0");
    if (!s->has_m) return fail(MM_ESTATE, "mm_backward_noalloc before mm_set_m");
    const size_t need = adj_bytes(s->p, ckpt_every);
    if (need > kNoAllocScratchBytes)
        return fail(MM_EINVAL,
                    "ckpt_every %lld needs %zu bytes of adjoint scratch; the static scratch holds %zu "
                    "(use a shorter checkpoint interval or mm_backward)",
                    (long long)ckpt_every, need, kNoAllocScratchBytes);
    if (!s->scratch) return fail(MM_EHIP, "static scratch unavailable: %s", s->scratch_err.c_str());
    return s->p.prec == MM_F32
               ? backward_impl<float>(s, nsteps, dt, ckpt_every, (const float*)d_ckpt,
                                      (const float*)d_lam_final, d_dku, (float*)d_dm0, s->scratch, false)
               : backward_impl<double>(s, nsteps, dt, ckpt_every, (const double*)d_ckpt,
                                       (const double*)d_lam_final, d_dku, (double*)d_dm0, s->scratch, false);
}

mm_status mm_batch_workspace_query(int32_t n, const mm_grid* grids, const mm_options* opt,
                                   size_t* bytes)
{
    if (!bytes) return fail(MM_EINVAL, "bytes is NULL");
    BatchLayout L;
    mm_status st = batch_layout(n, grids, opt, &L);
    if (st != MM_OK) return st;
    *bytes = L.total;
    if (opt && (opt->flags & MM_AUTOTUNE))  // room for whichever layout wins
        for (const mm_options& c : batch_tune_candidates(n, grids, opt)) {
            BatchLayout Q;
            if (batch_layout(n, grids, &c, &Q) == MM_OK) *bytes = std::max(*bytes, Q.total);
        }
    return MM_OK;
}

// The batch on a layout: descriptors, tile prefix sums and size classes
// uploaded; with spectra, each grid's kernel spectrum and twiddles too (the
// timing runs of the autotuner need neither).
static mm_status batch_build(int32_t n, const mm_grid* grids, const mm_material* mat,
                             const double* hext, const mm_options* opt, void* d_workspace,
                             size_t ws_bytes, void* stream, bool spectra, mm_batch** out)
{
    *out = nullptr;
    if (!mat) return fail(MM_EINVAL, "material is NULL");
    BatchLayout L;
    mm_status st = batch_layout(n, grids, opt, &L);
    if (st != MM_OK) return st;
    const bool per_grid = opt && (opt->flags & MM_PER_GRID_MATERIAL);
    std::vector<mm_material> mats(n);
    for (int s = 0; s < n; ++s) {
        mats[s] = per_grid ? mat[s] : mat[0];
        if (!check_material(&mats[s]))
            return fail(MM_EINVAL, "material of grid %d needs Ms > 0, A >= 0, alpha >= 0, gamma > 0, all finite",
                        s);
    }
    if (hext)
        for (int q = 0; q < 3 * n; ++q)
            if (!std::isfinite(hext[q])) return fail(MM_EINVAL, "applied fields must be finite");
    if (d_workspace && ws_bytes < L.total)
        return fail(MM_EINVAL, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, L.total);
    if (d_workspace && (reinterpret_cast<uintptr_t>(d_workspace) & 255))
        return fail(MM_EINVAL, "workspace must be 256-byte aligned");
    mm_batch* b = new mm_batch();
    b->n = n;
    b->mats = mats;
    b->flags = opt ? opt->flags : 0;
    b->stream = as_stream(stream);
    b->desc_dt = 0.0;  // no dt yet: the first step fills gdt
    for (int s = 0; s < n; ++s) {
        BatchDesc& d = L.desc[s];
        const mm_material& m = mats[s];
        const double Ms = m.Ms;
        for (int a = 0; a < 3; ++a) d.hred[a] = hext ? hext[3 * s + a] / Ms : 0.0;
        d.cex = 2.0 * m.A / (kMu0 * Ms * Ms * grids[s].cell * grids[s].cell);
        d.can = 2.0 * m.Ku / (kMu0 * Ms * Ms);
        d.alpha = m.alpha;
        d.gdt = 0.0;
    }
    b->L = std::move(L);
    const BatchLayout& BL = b->L;
    auto bail = [&](mm_status e) {
        std::string keep = g_err;
        mm_batch_destroy(b);
        g_err = keep;
        return e;
    };
    if (d_workspace) {
        b->ws = static_cast<char*>(d_workspace);
    } else {
        void* w = nullptr;
        hipError_t e = hipMalloc(&w, BL.total);
        if (e != hipSuccess) {
            delete b;
            return fail(MM_ENOMEM, "hipMalloc(%zu): %s", BL.total, hipGetErrorString(e));
        }
        b->ws = static_cast<char*>(w);
        b->own_ws = true;
    }
    hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(fail(MM_EHIP, "hipStreamCreate: %s", hipGetErrorString(e)));
    hipStream_t hs = b->stream;
    e = hipMemcpyAsync(b->at<char>(BL.o_desc), BL.desc.data(), n * sizeof(BatchDesc),
                       hipMemcpyHostToDevice, hs);
    if (e != hipSuccess) return bail(fail(MM_EHIP, "descriptor upload: %s", hipGetErrorString(e)));
    std::vector<int> pre(4 * (size_t)(n + 1));
    for (int q = 0; q < 4; ++q)
        for (int s = 0; s <= n; ++s) pre[q * (n + 1) + s] = BL.prefix[q][s];
    e = hipMemcpyAsync(b->at<char>(BL.o_prefix), pre.data(), pre.size() * sizeof(int),
                       hipMemcpyHostToDevice, hs);
    std::vector<int> cints((size_t)std::max<int64_t>(BL.class_ints, 1), 0);
    for (const BatchClassHost& c : BL.classes) {
        std::copy(c.members.begin(), c.members.end(), cints.begin() + c.off);
        std::copy(c.prefix.begin(), c.prefix.end(), cints.begin() + c.off + c.members.size());
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->at<char>(BL.o_classes), cints.data(), cints.size() * sizeof(int),
                           hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return bail(fail(MM_EHIP, "prefix upload: %s", hipGetErrorString(e)));
    if (!spectra) {
        *out = b;
        return MM_OK;
    }
    // kernel spectra and twiddles: one single-grid setup per grid on the scratch region
    mm_options o = opt ? *opt : mm_options{};
    o.threads = 256;
    o.flags &= ~(uint32_t)MM_USE_GRAPH;
    if (BL.plan_generic) o.flags |= MM_GENERIC_FFT;  // the same plans (no two-plane schedule)
    for (int s = 0; s < n; ++s) {
        const Plan& p = BL.plans[s];
        const BatchDesc& d = BL.desc[s];
        mm_sim* t = nullptr;
        mm_options og = o;  // the grid's padded sizes as the layout planned them
        og.px = BL.pad[s][0];
        og.py = BL.pad[s][1];
        mm_status r = mm_create(&grids[s], &b->mats[s], &og, b->at<char>(BL.o_scratch), BL.scratch, stream, &t);
        if (r != MM_OK) return bail(r);
        const size_t esz = BL.esz;
        hipError_t ce = hipMemcpyAsync(b->at<char>(BL.o_kern) + d.koff * esz, t->at<char>(p.o_kern),
                                       (size_t)p.kplanes * p.oct_elems * esz, hipMemcpyDeviceToDevice, hs);
        const size_t cz = 2 * esz;
        if (ce == hipSuccess)
            ce = hipMemcpyAsync(b->at<char>(BL.o_tw) + d.twx * cz, t->at<char>(p.o_twx), p.Px * cz,
                                hipMemcpyDeviceToDevice, hs);
        if (ce == hipSuccess)
            ce = hipMemcpyAsync(b->at<char>(BL.o_tw) + d.twy * cz, t->at<char>(p.o_twy), p.Py * cz,
                                hipMemcpyDeviceToDevice, hs);
        if (ce == hipSuccess)
            ce = hipMemcpyAsync(b->at<char>(BL.o_tw) + d.twz * cz, t->at<char>(p.o_twz), p.Pz * cz,
                                hipMemcpyDeviceToDevice, hs);
        mm_destroy(t);  // waits for the stream, so the scratch is free for the next grid
        if (ce != hipSuccess) return bail(fail(MM_EHIP, "spectrum copy: %s", hipGetErrorString(ce)));
    }
    *out = b;
    return MM_OK;
}

mm_status mm_batch_create(int32_t n, const mm_grid* grids, const mm_material* mat,
                          const double* hext, const mm_options* opt, void* d_workspace,
                          size_t ws_bytes, void* stream, mm_batch** out)
{
    if (!out) return fail(MM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!opt || !(opt->flags & MM_AUTOTUNE) || (opt->flags & MM_NO_DEMAG))
        return batch_build(n, grids, mat, hext, opt, d_workspace, ws_bytes, stream, true, out);
    // MM_AUTOTUNE: time one field evaluation of every candidate layout on
    // zero-filled data, then build the fastest with its spectra.  The first
    // candidate is the default layout: its argument errors go to the caller;
    // a later candidate that cannot be built (a padded length beyond the
    // passes, a workspace sized without MM_AUTOTUNE) is skipped.
    const std::vector<mm_options> cands = batch_tune_candidates(n, grids, opt);
    if (cands.empty()) {
        BatchLayout L;
        mm_status st = batch_layout(n, grids, opt, &L);
        return st != MM_OK ? st : fail(MM_ENOTSUP, "no layout of this batch could be built");
    }
    double best_ms = 1e300;
    size_t best = 0;
    int ncand = 0;
    for (size_t i = 0; i < cands.size(); ++i) {
        mm_batch* t = nullptr;
        mm_status r = batch_build(n, grids, mat, hext, &cands[i], d_workspace, ws_bytes, stream, false, &t);
        if (r != MM_OK) {
            if (i == 0) return r;
            continue;
        }
        double ms = 0.0;
        r = t->L.prec == MM_F32 ? time_batch_demag<float>(t, &ms) : time_batch_demag<double>(t, &ms);
        std::string keep = g_err;
        mm_batch_destroy(t);
        g_err = keep;
        if (r != MM_OK) return r;
        ++ncand;
        if (ms < best_ms) {
            best_ms = ms;
            best = i;
        }
    }
    mm_status r = batch_build(n, grids, mat, hext, &cands[best], d_workspace, ws_bytes, stream, true, out);
    if (r == MM_OK) {
        (*out)->tuned = 1;
        (*out)->tune_candidates = ncand;
        (*out)->tuned_ms = best_ms;
    }
    return r;
}

mm_status mm_batch_get_info(mm_batch* b, mm_batch_info* out)
{
    if (!b || !out) return fail(MM_EINVAL, "NULL argument");
    memset(out, 0, sizeof *out);
    out->cells = b->L.cells;
    out->n = b->n;
    out->pow2_pad = (b->flags & MM_POW2_PAD) ? 1 : 0;
    out->fast_pad = (b->flags & MM_FAST_PAD) ? 1 : 0;
    out->size_classes = b->L.fast ? 1 : 0;
    out->tuned = b->tuned;
    out->tune_candidates = b->tune_candidates;
    out->tuned_ms = b->tuned_ms;
    out->workspace_bytes = b->L.total;
    return MM_OK;
}

mm_status mm_batch_get_grid_plan(mm_batch* b, int32_t i, mm_plan_info* out)
{
    if (!b || !out) return fail(MM_EINVAL, "NULL argument");
    if (i < 0 || i >= b->n) return fail(MM_EINVAL, "grid index %d outside 0..%d", i, b->n - 1);
    const Plan& p = b->L.plans[i];
    memset(out, 0, sizeof *out);
    out->px = p.Px;
    out->py = p.Py;
    out->pz = p.Pz;
    out->hx = p.hx;
    out->ncomp = p.ncomp;
    out->threads = p.nt;
    out->spectrum_elems = (int64_t)p.kplanes * p.oct_elems;
    out->passes = (p.three_d && !p.zd) ? 5 : 3;
    out->generic_fft = b->L.fast ? 0 : 1;
    out->x_lines = p.xl;
    out->x_lines_inv = p.xl_inv;
    out->two_plane = p.zd ? 1 : 0;
    return MM_OK;
}

mm_status mm_batch_destroy(mm_batch* b)
{
    if (!b) return MM_OK;
    (void)hipStreamSynchronize(b->stream);
    batch_drop_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->own_ws) (void)hipFree(b->ws);
    delete b;
    return MM_OK;
}

mm_status mm_batch_set_m(mm_batch* b, const void* m, int on_device)
{
    if (!b || !m) return fail(MM_EINVAL, "batch or m is NULL");
    return b->L.prec == MM_F32 ? batch_set_m_impl<float>(b, m, on_device)
                               : batch_set_m_impl<double>(b, m, on_device);
}

mm_status mm_batch_get_m(mm_batch* b, void* out, int on_device)
{
    if (!b || !out) return fail(MM_EINVAL, "batch or out is NULL");
    if (!b->has_m) return fail(MM_ESTATE, "m has not been set");
    HIP_TRY(hipMemcpyAsync(out, b->at<char>(b->L.o_mn), (size_t)b->L.vec_elems * b->L.esz,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, b->stream));
    if (!on_device) HIP_TRY(hipStreamSynchronize(b->stream));
    return MM_OK;
}

mm_status mm_batch_get_field(mm_batch* b, int32_t term, void* out, int on_device)
{
    if (!b || !out) return fail(MM_EINVAL, "batch or out is NULL");
    if (term < 0 || term > 4) return fail(MM_EINVAL, "term must be 0..4");
    if (!b->has_m) return fail(MM_ESTATE, "m has not been set");
    return b->L.prec == MM_F32 ? batch_field_impl<float>(b, term, out, on_device)
                               : batch_field_impl<double>(b, term, out, on_device);
}

mm_status mm_batch_step(mm_batch* b, int64_t nsteps, double dt)
{
    if (!b) return fail(MM_EINVAL, "batch is NULL");
    if (nsteps < 0) return fail(MM_EINVAL, "nsteps must be >= 0");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(MM_EINVAL, "dt must be finite and > 0");
    if (!b->has_m) return fail(MM_ESTATE, "mm_batch_step before mm_batch_set_m");
    return b->L.prec == MM_F32 ? batch_step_impl<float>(b, nsteps, dt) : batch_step_impl<double>(b, nsteps, dt);
}

mm_status mm_batch_set_stream(mm_batch* b, void* stream)
{
    if (!b) return fail(MM_EINVAL, "batch is NULL");
    b->stream = as_stream(stream);
    return MM_OK;
}

mm_status mm_batch_cells(mm_batch* b, int64_t* total_cells)
{
    if (!b || !total_cells) return fail(MM_EINVAL, "NULL argument");
    *total_cells = b->L.cells;
    return MM_OK;
}

mm_status mm_profile_begin(mm_sim* s, int32_t kernel)
{
    if (!s) return fail(MM_EINVAL, "sim is NULL");
    if (kernel < 0 || kernel >= KCOUNT) return fail(MM_EINVAL, "kernel id must be 0..5");
    s->prof_kernel = kernel;
    s->prof_seen = 0;
    s->prof_armed = false;
    s->ev_used = 0;
    return MM_OK;
}

mm_status mm_profile_sample(mm_sim* s, int32_t every)
{
    if (!s) return fail(MM_EINVAL, "sim is NULL");
    if (every < 1) return fail(MM_EINVAL, "every must be >= 1");
    s->prof_every = every;
    return MM_OK;
}

mm_status mm_profile_end(mm_sim* s, double* total_ms, int64_t* launches)
{
    if (!s || !total_ms || !launches) return fail(MM_EINVAL, "NULL argument");
    if (s->prof_kernel < 0) return fail(MM_ESTATE, "no profile open");
    HIP_TRY(hipStreamSynchronize(s->stream));
    double tot = 0.0;
    for (size_t q = 0; q + 1 < s->ev_used; q += 2) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, s->ev[q], s->ev[q + 1]));
        tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)(s->ev_used / 2);
    s->prof_kernel = -1;
    s->ev_used = 0;
    return MM_OK;
}

const char* mm_kernel_name(int32_t kernel)
{
    static const char* names[KCOUNT] = {"k_row_r2c", "k_col_fft(fwd)", "k_kspace", "k_col_fft(inv)",
                                        "k_row_c2r", "k_llg_stage"};
    return (kernel >= 0 && kernel < KCOUNT) ? names[kernel] : "unknown";
}

const char* mm_status_string(mm_status s)
{
    switch (s) {
    case MM_OK: return "MM_OK";
    case MM_EINVAL: return "MM_EINVAL";
    case MM_ENOMEM: return "MM_ENOMEM";
    case MM_EHIP: return "MM_EHIP";
    case MM_ESTATE: return "MM_ESTATE";
    case MM_ENOTSUP: return "MM_ENOTSUP";
    case MM_ENONFINITE: return "MM_ENONFINITE";
    }
    return "unknown";
}

const char* mm_last_error(void) { return g_err.c_str(); }

}  // extern "C"
