/*
 * newell_oracle.c -- the cell-averaged demag tensor of Newell, Williams and
 * Dunlop (J. Geophys. Res. 98, 9551, 1993), the alternative to the paper's
 * point-field tensor that Sec. 2.3 cites.  TEST INFRASTRUCTURE ONLY (part of
 * the oracle library; never used by the product path).
 *
 * For two cubic cells of unit edge at integer offset (X, Y, Z), the xx entry
 * of the averaged tensor N is (1/4pi) times the second difference, in all
 * three directions, of Newell's function f:
 *     sum over i, j, k in {-1, 0, 1} of w_i w_j w_k f(X+i, Y+j, Z+k),
 *     w_0 = 2, w_(+-1) = -1;
 * the xy entry is the same sum over Newell's g.  yy, zz follow from f with
 * the axes permuted, xz and yz from g (f is symmetric in its last two
 * arguments, g in its first two).  With H = -N M, the tensor that multiplies
 * M in the convention of Eqs. 12-13 is K = -N.
 *
 * The 27-term sums cancel catastrophically at large offsets (f grows as r^3,
 * the result falls as r^-3), so everything is evaluated in binary128
 * (__float128, libquadmath): at |offset| = 1000 cells it still holds ~16
 * significant digits.  The result is returned in FP64.
 */
#include <quadmath.h>
#include <stdint.h>

typedef __float128 q;

/* Newell's f; even in each argument. */
static q newell_f(q x, q y, q z)
{
    x = fabsq(x);
    y = fabsq(y);
    z = fabsq(z);
    const q x2 = x * x, y2 = y * y, z2 = z * z, R = sqrtq(x2 + y2 + z2);
    q s = (2 * x2 - y2 - z2) * R / 6;
    if (y > 0 && x2 + z2 > 0) s += y / 2 * (z2 - x2) * asinhq(y / sqrtq(x2 + z2));
    if (z > 0 && x2 + y2 > 0) s += z / 2 * (y2 - x2) * asinhq(z / sqrtq(x2 + y2));
    if (x > 0 && y > 0 && z > 0) s -= x * y * z * atanq(y * z / (x * R));
    return s;
}

/* Newell's g; odd in x and in y, even in z. */
static q newell_g(q x, q y, q z)
{
    const q sgn = ((x < 0) != (y < 0)) ? -1 : 1;
    x = fabsq(x);
    y = fabsq(y);
    z = fabsq(z);
    const q x2 = x * x, y2 = y * y, z2 = z * z, R = sqrtq(x2 + y2 + z2);
    q s = -x * y * R / 3;
    if (z > 0 && x2 + y2 > 0) s += x * y * z * asinhq(z / sqrtq(x2 + y2));
    if (x > 0 && y2 + z2 > 0) s += y / 6 * (3 * z2 - y2) * asinhq(x / sqrtq(y2 + z2));
    if (y > 0 && x2 + z2 > 0) s += x / 6 * (3 * z2 - x2) * asinhq(y / sqrtq(x2 + z2));
    if (x > 0 && y > 0 && z > 0) {
        s -= z2 * z / 6 * atanq(x * y / (z * R));
        s -= z * y2 / 2 * atanq(x * z / (y * R));
        s -= z * x2 / 2 * atanq(y * z / (x * R));
    }
    return sgn * s;
}

/* sum_{ijk} w_i w_j w_k F(a + i, b + j, c + k) / (4 pi) */
static q second_difference(q (*F)(q, q, q), q a, q b, q c)
{
    static const int w[3] = {-1, 2, -1};
    q s = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                s += (q)(w[i] * w[j] * w[k]) * F(a + (i - 1), b + (j - 1), c + (k - 1));
    return s / (4 * M_PIq);
}

/* K = -N at integer offset (I, J, K): {xx, xy, xz, yy, yz, zz}. */
void or_newell_point(int32_t I, int32_t J, int32_t K, double out[6])
{
    const q X = I, Y = J, Z = K;
    out[0] = -(double)second_difference(newell_f, X, Y, Z);
    out[1] = -(double)second_difference(newell_g, X, Y, Z);
    out[2] = -(double)second_difference(newell_g, X, Z, Y);
    out[3] = -(double)second_difference(newell_f, Y, X, Z);
    out[4] = -(double)second_difference(newell_g, Y, Z, X);
    out[5] = -(double)second_difference(newell_f, Z, X, Y);
}

/* The table over all offsets of an nx x ny x nz grid, layout of or_tensor_table:
 * [6][2nz-1][2ny-1][2nx-1], offset (I, J, K) at index (K+nz-1, J+ny-1, I+nx-1). */
void or_newell_table(int32_t nx, int32_t ny, int32_t nz, double *out)
{
    const int64_t sx = 2 * nx - 1, sy = 2 * ny - 1, sz = 2 * nz - 1;
    const int64_t plane = sx * sy * sz;
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int32_t K = -(nz - 1); K <= nz - 1; ++K)
        for (int32_t J = -(ny - 1); J <= ny - 1; ++J)
            for (int32_t I = -(nx - 1); I <= nx - 1; ++I) {
                double t[6];
                or_newell_point(I, J, K, t);
                const int64_t o = ((int64_t)(K + nz - 1) * sy + (J + ny - 1)) * sx + (I + nx - 1);
                for (int c = 0; c < 6; ++c) out[c * plane + o] = t[c];
            }
}
