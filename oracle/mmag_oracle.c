/*
 * mmag_oracle.c -- plain, slow, FP64 CPU reference of the finite-difference
 * micromagnetic step.  TEST INFRASTRUCTURE ONLY: it is loaded by the tests,
 * by the smoke check and by the CPU-baseline leg of the benchmark, never by the
 * product path, and it shares no code with the HIP library.
 *
 * Every quantity follows the paper (Zhu, "Accelerate micromagnetic simulations
 * with GPU programming in MATLAB", arXiv:1501.07293) written out plainly:
 *   - demag tensor: Sec. 2.3, Eqs. 10-11 (eight-corner sums), origin included;
 *   - demag field: Eqs. 12-13 as a direct O(N^2) sum (no FFT);
 *   - exchange:    Sec. 2.1, Eq. 5 with the Neumann rule of Eqs. 6-7;
 *   - anisotropy:  Sec. 2.2, Eq. 8, easy axis x, x component only (Listing 2);
 *   - LLG:         Eq. 2 in Landau-Lifshitz form, gamma multiplying H in A/m;
 *   - integrator:  classical RK4 with one renormalisation per step
 *                  (the renormalisation of the appendix script);
 *   - energies:    Eq. 1 term by term;
 *   - periodic axes (optional): the boundary the paper contrasts with zero
 *                  padding (Sec. 2.3): the exchange stencil wraps around, and
 *                  the demag sum runs over the minimum image of each source
 *                  and `images` further images on each side (see
 *                  or_tensor_table_periodic for the exact reading).
 *
 * Units are SI: m is a unit vector per cell, M = Ms m, fields in A/m, energy
 * in J.  Layout: planar [3][nz][ny][nx], x fastest.  Cell c = (i,j,k) has
 * linear index (k*ny + j)*nx + i.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846264338327950288
#define OR_MU0 (4.0e-7 * OR_PI)

typedef struct {
    int32_t nx, ny, nz;
    double cell;        /* edge delta of the cubic cell, m */
    double Ms;          /* saturation magnetisation, A/m */
    double A;           /* exchange constant, J/m */
    double Ku;          /* uniaxial anisotropy, J/m^3 (used when ku_map is NULL) */
    double alpha;       /* damping */
    double gamma;       /* gyromagnetic ratio multiplying H in A/m, m/(A s) */
    double hext[3];     /* applied field, A/m */
    const double *ku_map; /* optional per-cell Ku, N values, J/m^3 */
    int32_t demag;      /* 0 switches the demag term off */
    int32_t periodic[3]; /* per axis x, y, z: 1 = periodic */
    int32_t images;     /* periodic axes: images on each side beyond the minimum image */
} or_params;

void or_newell_point(int32_t I, int32_t J, int32_t K, double out[6]);

/* ------------------------------------------------------------------------ */
/* ln(Z + r) with r = |(X,Y,Z)|.  For Z < 0 the sum Z + r cancels; the identity
 * Z + r = (X^2 + Y^2) / (r - Z) gives the same number without cancellation.
 * X, Y, Z are half-integers here, so X^2 + Y^2 > 0.                          */
static double log_z_plus_r(double X, double Y, double Z, double r)
{
    if (Z >= 0.0) return log(Z + r);
    return log((X * X + Y * Y) / (r - Z));
}

/* Demag tensor, Eqs. 10-11.  (I,J,K) is the integer offset source-observer in
 * cells; the result is dimensionless (independent of delta).  The sums run
 * over i,j,k in {0,1} (the listing's loop bounds; the equation's lower limit 1
 * on i is read as 0).  Output order: xx, xy, xz, yy, yz, zz.  Kxz and Kyz are
 * the permutations of Eq. 11 with ln(Y+r) and ln(X+r).                       */
void or_tensor_point(int32_t I, int32_t J, int32_t K, double out[6])
{
    double sxx = 0, syy = 0, szz = 0, sxy = 0, sxz = 0, syz = 0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k) {
                double X = I + i - 0.5, Y = J + j - 0.5, Z = K + k - 0.5;
                double r = sqrt(X * X + Y * Y + Z * Z);
                double s = ((i + j + k) & 1) ? -1.0 : 1.0;
                sxx += s * atan(Y * Z / (X * r));
                syy += s * atan(X * Z / (Y * r));
                szz += s * atan(X * Y / (Z * r));
                sxy += s * log_z_plus_r(X, Y, Z, r);
                sxz += s * log_z_plus_r(X, Z, Y, r);
                syz += s * log_z_plus_r(Y, Z, X, r);
            }
    double pf = 1.0 / (4.0 * OR_PI);
    out[0] = pf * sxx;
    out[1] = -pf * sxy;
    out[2] = -pf * sxz;
    out[3] = pf * syy;
    out[4] = -pf * syz;
    out[5] = pf * szz;
}

/* Table of all offsets |I|<nx, |J|<ny, |K|<nz:
 * out[c][K+nz-1][J+ny-1][I+nx-1], c in the order of or_tensor_point. */
void or_tensor_table(int32_t nx, int32_t ny, int32_t nz, double *out)
{
    int64_t tx = 2 * nx - 1, ty = 2 * ny - 1, tz = 2 * nz - 1;
    int64_t plane = tx * ty * tz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t kk = 0; kk < tz; ++kk)
        for (int64_t jj = 0; jj < ty; ++jj)
            for (int64_t ii = 0; ii < tx; ++ii) {
                double v[6];
                or_tensor_point((int32_t)(ii - (nx - 1)), (int32_t)(jj - (ny - 1)),
                                (int32_t)(kk - (nz - 1)), v);
                int64_t idx = (kk * ty + jj) * tx + ii;
                for (int c = 0; c < 6; ++c) out[c * plane + idx] = v[c];
            }
}

/* Periodic table.  Along an open axis of n cells the entries are the offsets
 * d = t - (n - 1), t in [0, 2n - 1), as in or_tensor_table.  Along a periodic
 * axis of period n the entry t in [0, n) stands for every offset d = t (mod n)
 * and holds the sum over images: the representative of t nearest to zero
 * (t if 2t < n, t - n if 2t > n; for 2t = n both t and t - n, each with weight
 * 1/2, so that the entry keeps the parity of the tensor component) plus
 * `images` multiples of n on either side of it.  The entry is the weighted sum
 * of the tensor over the product of the per-axis offset lists.  kind 0: Eqs.
 * 10-11; kind 1: Newell's cell-averaged tensor.  Output [6][tz][ty][tx].     */
static int axis_offsets(int n, int periodic, int images, int t, int *off, double *w)
{
    if (!periodic) {
        off[0] = t - (n - 1);
        w[0] = 1.0;
        return 1;
    }
    int reps[2], nr = 0;
    double rw = 1.0;
    if (2 * t < n) {
        reps[nr++] = t;
    } else if (2 * t > n) {
        reps[nr++] = t - n;
    } else {
        reps[nr++] = t;
        reps[nr++] = t - n;
        rw = 0.5;
    }
    int k = 0;
    for (int r = 0; r < nr; ++r)
        for (int j = -images; j <= images; ++j) {
            off[k] = reps[r] + j * n;
            w[k] = rw;
            ++k;
        }
    return k;
}

void or_tensor_table_periodic(int32_t nx, int32_t ny, int32_t nz, const int32_t periodic[3],
                              int32_t images, int32_t kind, double *out)
{
    const int64_t tx = periodic[0] ? nx : 2 * nx - 1, ty = periodic[1] ? ny : 2 * ny - 1;
    const int64_t tz = periodic[2] ? nz : 2 * nz - 1, plane = tx * ty * tz;
    const int cap = 2 * (2 * images + 1);
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
    for (int64_t kk = 0; kk < tz; ++kk)
        for (int64_t jj = 0; jj < ty; ++jj) {
            int ox[cap], oy[cap], oz[cap];
            double wx[cap], wy[cap], wz[cap];
            int nzo = axis_offsets(nz, periodic[2], images, (int)kk, oz, wz);
            int nyo = axis_offsets(ny, periodic[1], images, (int)jj, oy, wy);
            for (int64_t ii = 0; ii < tx; ++ii) {
                int nxo = axis_offsets(nx, periodic[0], images, (int)ii, ox, wx);
                double acc[6] = {0, 0, 0, 0, 0, 0};
                for (int c = 0; c < nzo; ++c)
                    for (int b = 0; b < nyo; ++b)
                        for (int a = 0; a < nxo; ++a) {
                            double v[6];
                            if (kind == 1) or_newell_point(ox[a], oy[b], oz[c], v);
                            else or_tensor_point(ox[a], oy[b], oz[c], v);
                            double w = wx[a] * wy[b] * wz[c];
                            for (int q = 0; q < 6; ++q) acc[q] += w * v[q];
                        }
                int64_t idx = (kk * ty + jj) * tx + ii;
                for (int q = 0; q < 6; ++q) out[q * plane + idx] = acc[q];
            }
        }
}

/* ------------------------------------------------------------------------ */
/* Demag field, Eqs. 12-13, direct sum: H_a(o) = Ms sum_s sum_b K_ab(s-o) m_b(s).
 * table: from or_tensor_table for the same grid (or_tensor_table_periodic when
 * an axis is periodic; its entry along a periodic axis is (s - o) mod n).
 * obs: optional list of observation cell indices (nobs of them); H then holds
 * [3][nobs].  With obs == NULL every cell is an observer and H is [3][N].    */
static int64_t table_index(int64_t d, int64_t n, int periodic)
{
    return periodic ? ((d % n) + n) % n : d + n - 1;
}

void or_demag(const or_params *p, const double *m, const double *table,
              const int64_t *obs, int64_t nobs, double *H)
{
    const int64_t nx = p->nx, ny = p->ny, nz = p->nz, N = nx * ny * nz;
    const int px = p->periodic[0], py = p->periodic[1], pz = p->periodic[2];
    const int64_t tx = px ? nx : 2 * nx - 1, ty = py ? ny : 2 * ny - 1, tz = pz ? nz : 2 * nz - 1;
    const int64_t plane = tx * ty * tz;
    const double *mx = m, *my = m + N, *mz = m + 2 * N;
    int64_t nout = obs ? nobs : N;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nout; ++q) {
        int64_t o = obs ? obs[q] : q;
        int64_t oi = o % nx, oj = (o / nx) % ny, ok = o / (nx * ny);
        double hx = 0, hy = 0, hz = 0;
        for (int64_t sk = 0; sk < nz; ++sk)
            for (int64_t sj = 0; sj < ny; ++sj)
                for (int64_t si = 0; si < nx; ++si) {
                    int64_t s = (sk * ny + sj) * nx + si;
                    int64_t t = (table_index(sk - ok, nz, pz) * ty + table_index(sj - oj, ny, py)) * tx
                              + table_index(si - oi, nx, px);
                    double kxx = table[t], kxy = table[plane + t], kxz = table[2 * plane + t];
                    double kyy = table[3 * plane + t], kyz = table[4 * plane + t];
                    double kzz = table[5 * plane + t];
                    double ax = mx[s], ay = my[s], az = mz[s];
                    hx += kxx * ax + kxy * ay + kxz * az;
                    hy += kxy * ax + kyy * ay + kyz * az;
                    hz += kxz * ax + kyz * ay + kzz * az;
                }
        H[q] = p->Ms * hx;
        H[nout + q] = p->Ms * hy;
        H[2 * nout + q] = p->Ms * hz;
    }
}

/* Exchange field, Eq. 5 with Eqs. 6-7: a missing neighbour is the cell itself,
 * so it contributes nothing; H = 2A/(mu0 Ms delta^2) sum_nb (m_nb - m_c).
 * Along a periodic axis no neighbour is missing: the first and last cells are
 * neighbours.                                                                */
void or_exchange(const or_params *p, const double *m, double *H)
{
    const int64_t nx = p->nx, ny = p->ny, nz = p->nz, N = nx * ny * nz;
    const double pref = 2.0 * p->A / (OR_MU0 * p->Ms * p->cell * p->cell);
    const int px = p->periodic[0], py = p->periodic[1], pz = p->periodic[2];
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        for (int a = 0; a < 3; ++a) {
            const double *u = m + a * N;
            double mc = u[c], acc = 0.0;
            if (i > 0) acc += u[c - 1] - mc;
            else if (px) acc += u[c + nx - 1] - mc;
            if (i < nx - 1) acc += u[c + 1] - mc;
            else if (px) acc += u[c - (nx - 1)] - mc;
            if (j > 0) acc += u[c - nx] - mc;
            else if (py) acc += u[c + nx * (ny - 1)] - mc;
            if (j < ny - 1) acc += u[c + nx] - mc;
            else if (py) acc += u[c - nx * (ny - 1)] - mc;
            if (k > 0) acc += u[c - nx * ny] - mc;
            else if (pz) acc += u[c + nx * ny * (nz - 1)] - mc;
            if (k < nz - 1) acc += u[c + nx * ny] - mc;
            else if (pz) acc += u[c - nx * ny * (nz - 1)] - mc;
            H[a * N + c] = pref * acc;
        }
    }
}

/* Anisotropy field, Eq. 8: x component 2 Ku/(mu0 Ms) m_x, y and z zero. */
void or_anisotropy(const or_params *p, const double *m, double *H)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    for (int64_t c = 0; c < N; ++c) {
        double ku = p->ku_map ? p->ku_map[c] : p->Ku;
        H[c] = 2.0 * ku / (OR_MU0 * p->Ms) * m[c];
        H[N + c] = 0.0;
        H[2 * N + c] = 0.0;
    }
}

/* Effective field, Eq. 3.  Any of the per-term outputs may be NULL; heff
 * (the sum) may be NULL too.  Each buffer is [3][N].                         */
void or_heff(const or_params *p, const double *m, const double *table,
             double *h_exch, double *h_anis, double *h_demag, double *heff)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    double *ex = (double *)malloc(sizeof(double) * 3 * N);
    double *an = (double *)malloc(sizeof(double) * 3 * N);
    double *dm = (double *)calloc(3 * N, sizeof(double));
    or_exchange(p, m, ex);
    or_anisotropy(p, m, an);
    if (p->demag) or_demag(p, m, table, NULL, 0, dm);
    if (h_exch) memcpy(h_exch, ex, sizeof(double) * 3 * N);
    if (h_anis) memcpy(h_anis, an, sizeof(double) * 3 * N);
    if (h_demag) memcpy(h_demag, dm, sizeof(double) * 3 * N);
    if (heff)
        for (int a = 0; a < 3; ++a)
            for (int64_t c = 0; c < N; ++c)
                heff[a * N + c] = ex[a * N + c] + an[a * N + c] + dm[a * N + c] + p->hext[a];
    free(ex);
    free(an);
    free(dm);
}

/* LLG right-hand side, Eq. 2 for the unit vector m:
 * dm/dt = -gamma/(1+alpha^2) [ m x H + alpha m x (m x H) ].                 */
void or_llg_rhs(const or_params *p, const double *m, const double *heff, double *dmdt)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    const double g = p->gamma / (1.0 + p->alpha * p->alpha);
    for (int64_t c = 0; c < N; ++c) {
        double mx = m[c], my = m[N + c], mz = m[2 * N + c];
        double hx = heff[c], hy = heff[N + c], hz = heff[2 * N + c];
        double tx = my * hz - mz * hy, ty = mz * hx - mx * hz, tz = mx * hy - my * hx;
        double dx = my * tz - mz * ty, dy = mz * tx - mx * tz, dz = mx * ty - my * tx;
        dmdt[c] = -g * (tx + p->alpha * dx);
        dmdt[N + c] = -g * (ty + p->alpha * dy);
        dmdt[2 * N + c] = -g * (tz + p->alpha * dz);
    }
}

/* f(m) = RHS at the effective field of m. */
static void rhs_of(const or_params *p, const double *m, const double *table,
                   double *heff, double *out)
{
    or_heff(p, m, table, NULL, NULL, NULL, heff);
    or_llg_rhs(p, m, heff, out);
}

/* Classical RK4, nsteps steps of dt; m (in/out) is renormalised per cell once
 * at the end of every step (stage states are not normalised).              */
void or_rk4(const or_params *p, double *m, const double *table, double dt, int64_t nsteps)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz, L = 3 * N;
    double *k1 = (double *)malloc(sizeof(double) * L);
    double *k2 = (double *)malloc(sizeof(double) * L);
    double *k3 = (double *)malloc(sizeof(double) * L);
    double *k4 = (double *)malloc(sizeof(double) * L);
    double *ms = (double *)malloc(sizeof(double) * L);
    double *h = (double *)malloc(sizeof(double) * L);
    for (int64_t n = 0; n < nsteps; ++n) {
        rhs_of(p, m, table, h, k1);
        for (int64_t q = 0; q < L; ++q) ms[q] = m[q] + 0.5 * dt * k1[q];
        rhs_of(p, ms, table, h, k2);
        for (int64_t q = 0; q < L; ++q) ms[q] = m[q] + 0.5 * dt * k2[q];
        rhs_of(p, ms, table, h, k3);
        for (int64_t q = 0; q < L; ++q) ms[q] = m[q] + dt * k3[q];
        rhs_of(p, ms, table, h, k4);
        for (int64_t q = 0; q < L; ++q)
            m[q] = m[q] + dt / 6.0 * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
        for (int64_t c = 0; c < N; ++c) {
            double nrm = sqrt(m[c] * m[c] + m[N + c] * m[N + c] + m[2 * N + c] * m[2 * N + c]);
            m[c] /= nrm;
            m[N + c] /= nrm;
            m[2 * N + c] /= nrm;
        }
    }
    free(k1);
    free(k2);
    free(k3);
    free(k4);
    free(ms);
    free(h);
}

/* Energies of Eq. 1 in J: out = {exchange, anisotropy, demag, zeeman, total}.
 * Exchange is summed over face-neighbour pairs, A delta |m_a - m_b|^2, which
 * is the discrete form of A (grad m)^2 consistent with Eq. 5; anisotropy uses
 * Ku (m_y^2 + m_z^2); demag -mu0/2 M.H_d; Zeeman -mu0 M.H_ext, each times the
 * cell volume.                                                              */
void or_energy(const or_params *p, const double *m, const double *table, double out[5])
{
    const int64_t nx = p->nx, ny = p->ny, nz = p->nz, N = nx * ny * nz;
    const double V = p->cell * p->cell * p->cell;
    double eex = 0, ean = 0, ed = 0, ez = 0;
    const int px = p->periodic[0], py = p->periodic[1], pz = p->periodic[2];
    for (int64_t c = 0; c < N; ++c) {
        int64_t i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        /* each neighbour pair once, towards +x, +y, +z; along a periodic axis the
         * last cell pairs with the first (the pairs of the wrapped stencil)     */
        int64_t nb[3] = {i < nx - 1 ? c + 1 : (px ? c - (nx - 1) : -1),
                         j < ny - 1 ? c + nx : (py ? c - nx * (ny - 1) : -1),
                         k < nz - 1 ? c + nx * ny : (pz ? c - nx * ny * (nz - 1) : -1)};
        for (int d = 0; d < 3; ++d) {
            if (nb[d] < 0) continue;
            for (int a = 0; a < 3; ++a) {
                double df = m[a * N + nb[d]] - m[a * N + c];
                eex += p->A * p->cell * df * df;
            }
        }
        double ku = p->ku_map ? p->ku_map[c] : p->Ku;
        ean += ku * V * (m[N + c] * m[N + c] + m[2 * N + c] * m[2 * N + c]);
        for (int a = 0; a < 3; ++a) ez += -OR_MU0 * V * p->Ms * m[a * N + c] * p->hext[a];
    }
    if (p->demag) {
        double *hd = (double *)malloc(sizeof(double) * 3 * N);
        or_demag(p, m, table, NULL, 0, hd);
        for (int64_t q = 0; q < 3 * N; ++q) ed += -0.5 * OR_MU0 * V * p->Ms * m[q] * hd[q];
        free(hd);
    }
    out[0] = eex;
    out[1] = ean;
    out[2] = ed;
    out[3] = ez;
    out[4] = eex + ean + ed + ez;
}

/* Mean of m over the cells (the appendix script's periodic output). */
void or_mean_m(const or_params *p, const double *m, double out[3])
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    for (int a = 0; a < 3; ++a) {
        double s = 0;
        for (int64_t c = 0; c < N; ++c) s += m[a * N + c];
        out[a] = s / (double)N;
    }
}

/* Largest torque over the cells: max_c |m_c x H_eff,c| in A/m, with H_eff the
 * full effective field of Eq. 3 at m (the quantity whose vanishing marks an
 * equilibrium of Eq. 2; used as a relaxation criterion).                     */
double or_max_torque(const or_params *p, const double *m, const double *table)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    double *h = (double *)malloc(sizeof(double) * 3 * N);
    or_heff(p, m, table, NULL, NULL, NULL, h);
    double best = 0.0;
    for (int64_t c = 0; c < N; ++c) {
        double mx = m[c], my = m[N + c], mz = m[2 * N + c];
        double hx = h[c], hy = h[N + c], hz = h[2 * N + c];
        double tx = my * hz - mz * hy, ty = mz * hx - mx * hz, tz = mx * hy - my * hx;
        double t = sqrt(tx * tx + ty * ty + tz * tz);
        if (t > best) best = t;
    }
    free(h);
    return best;
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint of nsteps RK4 steps with renormalisation (test infrastructure
 * for the gradient of a loss of the final state).  With the effective field
 * H(m) = L m + H_ext (L symmetric: exchange Laplacian with the Neumann rule,
 * diagonal anisotropy, symmetric demag tensor) and
 *   f(m) = -g [ m x H + alpha m x (m x H) ],   g = gamma / (1 + alpha^2),
 * the transpose Jacobian applied to a covector lam is
 *   (df/dm)^T lam = -g [ H x lam + alpha ((m x H) x lam + H x (lam x m)) ] + L nu,
 *   nu = -g [ lam x m + alpha (lam x m) x m ],
 * and the anisotropy map enters through dH_x/dKu(c) = 2 m_x(c) / (mu0 Ms), so
 * dLoss/dKu(c) collects nu_x(c) m_x(c) 2 / (mu0 Ms) over every stage.
 * lam_final = dLoss/dm at the final state; outputs dku (N) and dm0 ([3][N]),
 * either may be NULL.  Stores every stage of every step (small grids only). */
static void cross3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* out = (df/dm)^T lam at (m, H); nu_out = nu (both [3][N]). */
static void rhs_vjp(const or_params *p, const double *m, const double *H, const double *lam,
                    const double *table, double *out, double *nu_out)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    const double g = p->gamma / (1.0 + p->alpha * p->alpha);
    for (int64_t c = 0; c < N; ++c) {
        double mm[3] = {m[c], m[N + c], m[2 * N + c]};
        double hh[3] = {H[c], H[N + c], H[2 * N + c]};
        double ll[3] = {lam[c], lam[N + c], lam[2 * N + c]};
        double mxh[3], t1[3], t2[3], lxm[3], t3[3], t4[3];
        cross3(hh, ll, t1);        /* H x lam */
        cross3(mm, hh, mxh);       /* m x H */
        cross3(mxh, ll, t2);       /* (m x H) x lam */
        cross3(ll, mm, lxm);       /* lam x m */
        cross3(hh, lxm, t3);       /* H x (lam x m) */
        cross3(lxm, mm, t4);       /* (lam x m) x m */
        for (int a = 0; a < 3; ++a) {
            out[a * N + c] = -g * (t1[a] + p->alpha * (t2[a] + t3[a]));
            nu_out[a * N + c] = -g * (lxm[a] + p->alpha * t4[a]);
        }
    }
    /* + L nu: the field operator without the applied field, applied to nu */
    or_params q = *p;
    q.hext[0] = q.hext[1] = q.hext[2] = 0.0;
    double *Lnu = (double *)malloc(sizeof(double) * 3 * N);
    or_heff(&q, nu_out, table, NULL, NULL, NULL, Lnu);
    for (int64_t k = 0; k < 3 * N; ++k) out[k] += Lnu[k];
    free(Lnu);
}

void or_rk4_adjoint(const or_params *p, const double *m0, const double *table, double dt,
                    int64_t nsteps, const double *lam_final, double *dku, double *dm0)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz, L = 3 * N;
    /* forward: every stage state and its field */
    double *ms = (double *)malloc(sizeof(double) * L * 4 * nsteps);  /* m_n, m2, m3, m4 */
    double *hs = (double *)malloc(sizeof(double) * L * 4 * nsteps);
    double *mend = (double *)malloc(sizeof(double) * L * (nsteps + 1));
    double *k = (double *)malloc(sizeof(double) * L * 4);
    memcpy(mend, m0, sizeof(double) * L);
    for (int64_t n = 0; n < nsteps; ++n) {
        double *S = ms + 4 * n * L, *Hh = hs + 4 * n * L;
        const double *mn = mend + n * L;
        memcpy(S, mn, sizeof(double) * L);
        const double cf[3] = {0.5, 0.5, 1.0};
        for (int s = 0; s < 4; ++s) {
            or_heff(p, S + s * L, table, NULL, NULL, NULL, Hh + s * L);
            or_llg_rhs(p, S + s * L, Hh + s * L, k + s * L);
            if (s < 3)
                for (int64_t q = 0; q < L; ++q) S[(s + 1) * L + q] = mn[q] + cf[s] * dt * k[s * L + q];
        }
        double *mnext = mend + (n + 1) * L;
        for (int64_t q = 0; q < L; ++q)
            mnext[q] = mn[q] + dt / 6.0 * (k[q] + 2 * k[L + q] + 2 * k[2 * L + q] + k[3 * L + q]);
        for (int64_t c = 0; c < N; ++c) {
            double nrm = sqrt(mnext[c] * mnext[c] + mnext[N + c] * mnext[N + c] +
                              mnext[2 * N + c] * mnext[2 * N + c]);
            for (int a = 0; a < 3; ++a) mnext[a * N + c] /= nrm;
        }
    }
    /* reverse */
    double *lam = (double *)malloc(sizeof(double) * L);
    double *mu = (double *)malloc(sizeof(double) * L);
    double *dF = (double *)malloc(sizeof(double) * L);
    double *a = (double *)malloc(sizeof(double) * L);
    double *nu = (double *)malloc(sizeof(double) * L);
    double *acc = (double *)malloc(sizeof(double) * L);
    double *mstar = (double *)malloc(sizeof(double) * L);
    memcpy(lam, lam_final, sizeof(double) * L);
    if (dku) memset(dku, 0, sizeof(double) * N);
    const double kfac = 2.0 / (OR_MU0 * p->Ms);
    for (int64_t n = nsteps - 1; n >= 0; --n) {
        double *S = ms + 4 * n * L, *Hh = hs + 4 * n * L;
        const double *mn = mend + n * L;
        for (int s = 0; s < 4; ++s) or_llg_rhs(p, S + s * L, Hh + s * L, k + s * L);
        for (int64_t q = 0; q < L; ++q)
            mstar[q] = mn[q] + dt / 6.0 * (k[q] + 2 * k[L + q] + 2 * k[2 * L + q] + k[3 * L + q]);
        /* renormalisation: mp = mstar / norm, so mu = (lam - (lam . mp) mp) / norm */
        for (int64_t c = 0; c < N; ++c) {
            double nrm = sqrt(mstar[c] * mstar[c] + mstar[N + c] * mstar[N + c] +
                              mstar[2 * N + c] * mstar[2 * N + c]);
            double mp[3] = {mstar[c] / nrm, mstar[N + c] / nrm, mstar[2 * N + c] / nrm};
            double dot = lam[c] * mp[0] + lam[N + c] * mp[1] + lam[2 * N + c] * mp[2];
            for (int d = 0; d < 3; ++d) mu[d * N + c] = (lam[d * N + c] - dot * mp[d]) / nrm;
        }
        /* m* = m_n + (F1 + 2F2 + 2F3 + F4)/6 with F_s = dt f(m_s);
         * m2 = m_n + F1/2, m3 = m_n + F2/2, m4 = m_n + F3. */
        memcpy(acc, mu, sizeof(double) * L);
        for (int64_t q = 0; q < L; ++q) dF[q] = mu[q] / 6.0;
        for (int s = 3; s >= 0; --s) {
            rhs_vjp(p, S + s * L, Hh + s * L, dF, table, a, nu);
            for (int64_t q = 0; q < L; ++q) a[q] *= dt;
            if (dku)
                for (int64_t c = 0; c < N; ++c) dku[c] += dt * nu[c] * S[s * L + c] * kfac;
            for (int64_t q = 0; q < L; ++q) acc[q] += a[q];
            if (s == 3)
                for (int64_t q = 0; q < L; ++q) dF[q] = 2.0 * mu[q] / 6.0 + a[q];
            else if (s == 2)
                for (int64_t q = 0; q < L; ++q) dF[q] = 2.0 * mu[q] / 6.0 + 0.5 * a[q];
            else if (s == 1)
                for (int64_t q = 0; q < L; ++q) dF[q] = mu[q] / 6.0 + 0.5 * a[q];
        }
        memcpy(lam, acc, sizeof(double) * L);
    }
    if (dm0) memcpy(dm0, lam, sizeof(double) * L);
    free(ms);
    free(hs);
    free(mend);
    free(k);
    free(lam);
    free(mu);
    free(dF);
    free(a);
    free(nu);
    free(acc);
    free(mstar);
}

/* Explicit Euler with renormalisation, the integrator of the appendix script:
 * m <- (m + dt f(m)) / |m + dt f(m)| per cell, nsteps times. */
void or_euler(const or_params *p, double *m, const double *table, double dt, int64_t nsteps)
{
    const int64_t N = (int64_t)p->nx * p->ny * p->nz, L = 3 * N;
    double *k = (double *)malloc(sizeof(double) * L);
    double *h = (double *)malloc(sizeof(double) * L);
    for (int64_t n = 0; n < nsteps; ++n) {
        rhs_of(p, m, table, h, k);
        for (int64_t q = 0; q < L; ++q) m[q] += dt * k[q];
        for (int64_t c = 0; c < N; ++c) {
            double nrm = sqrt(m[c] * m[c] + m[N + c] * m[N + c] + m[2 * N + c] * m[2 * N + c]);
            m[c] /= nrm;
            m[N + c] /= nrm;
            m[2 * N + c] /= nrm;
        }
    }
    free(k);
    free(h);
}
