// mm_tensor.hip -- one-time setup in FP64: the demag tensor of Sec. 2.3
// (Eqs. 10-11, Nakatani's point-field form, origin included), twiddle tables,
// and the real octant of the kernel spectrum.
#include "mm_common.hpp"
#include "mm_kernels.hpp"

namespace mm {

// ln(Z + r); for Z < 0 use Z + r = (X^2 + Y^2) / (r - Z), which does not cancel.
__device__ inline double log_z_plus_r(double X, double Y, double Z, double r)
{
    return Z >= 0.0 ? log(Z + r) : log((X * X + Y * Y) / (r - Z));
}

// Component comp (0..5 = xx, xy, xz, yy, yz, zz) at offset (I,J,K) = source -
// observer, in units of the cell edge: the eight-corner alternating sums of
// Eq. 10 (atan terms, diagonal) and Eq. 11 (log terms, off-diagonal, with the
// minus sign), over corners i,j,k in {0,1}.  Integer offsets give the paper's
// tensor; real ones the point field at a shifted observer (used below).
__device__ double tensor_component(int comp, double I, double J, double K)
{
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const double X = I + i - 0.5, Y = J + j - 0.5, Z = K + k - 0.5;
                const double r = sqrt(X * X + Y * Y + Z * Z);
                double t;
                switch (comp) {
                case 0: t = atan(Y * Z / (X * r)); break;
                case 1: t = log_z_plus_r(X, Y, Z, r); break;
                case 2: t = log_z_plus_r(X, Z, Y, r); break;
                case 3: t = atan(X * Z / (Y * r)); break;
                case 4: t = log_z_plus_r(Y, Z, X, r); break;
                default: t = atan(X * Y / (Z * r)); break;
                }
                s += ((i + j + k) & 1) ? -t : t;
            }
    const double pf = 0.079577471545947667884;  // 1 / (4 pi)
    return (comp == 0 || comp == 3 || comp == 5) ? pf * s : -pf * s;
}

// ---- Newell's cell-averaged tensor (Newell, Williams and Dunlop 1993; the
// alternative Sec. 2.3 cites), in the sign convention above (K = -N).
// Near the origin: the 27-point second difference of Newell's f (diagonal) and
// g (off-diagonal) in FP64.  That sum cancels as (r / delta)^6 in relative
// terms, so from a (Euclidean) distance of kNewellFar cells on, the average of
// the point field above over the observer's cell is taken instead, by 4-point
// Gauss-Legendre quadrature per axis; both parts stay within ~2e-10 of the
// exact averaged tensor.
constexpr int kNewellFar = 8;

__device__ double newell_f(double x, double y, double z)
{
    x = fabs(x);
    y = fabs(y);
    z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z, R = sqrt(x2 + y2 + z2);
    double s = (2.0 * x2 - y2 - z2) * R / 6.0;
    if (y > 0.0 && x2 + z2 > 0.0) s += 0.5 * y * (z2 - x2) * asinh(y / sqrt(x2 + z2));
    if (z > 0.0 && x2 + y2 > 0.0) s += 0.5 * z * (y2 - x2) * asinh(z / sqrt(x2 + y2));
    if (x > 0.0 && y > 0.0 && z > 0.0) s -= x * y * z * atan(y * z / (x * R));
    return s;
}

__device__ double newell_g(double x, double y, double z)
{
    const double sgn = ((x < 0.0) != (y < 0.0)) ? -1.0 : 1.0;
    x = fabs(x);
    y = fabs(y);
    z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z, R = sqrt(x2 + y2 + z2);
    double s = -x * y * R / 3.0;
    if (z > 0.0 && x2 + y2 > 0.0) s += x * y * z * asinh(z / sqrt(x2 + y2));
    if (x > 0.0 && y2 + z2 > 0.0) s += y / 6.0 * (3.0 * z2 - y2) * asinh(x / sqrt(y2 + z2));
    if (y > 0.0 && x2 + z2 > 0.0) s += x / 6.0 * (3.0 * z2 - x2) * asinh(y / sqrt(x2 + z2));
    if (x > 0.0 && y > 0.0 && z > 0.0) {
        s -= z2 * z / 6.0 * atan(x * y / (z * R));
        s -= 0.5 * z * y2 * atan(x * z / (y * R));
        s -= 0.5 * z * x2 * atan(y * z / (x * R));
    }
    return sgn * s;
}

// (1 / 4 pi) sum_{i,j,k in -1..1} w_i w_j w_k F(a+i, b+j, c+k), w = (-1, 2, -1)
template <bool G>
__device__ double newell_sum(double a, double b, double c)
{
    double s = 0.0;
    for (int i = -1; i <= 1; ++i)
        for (int j = -1; j <= 1; ++j)
            for (int k = -1; k <= 1; ++k) {
                const double w = (i ? -1.0 : 2.0) * (j ? -1.0 : 2.0) * (k ? -1.0 : 2.0);
                s += w * (G ? newell_g(a + i, b + j, c + k) : newell_f(a + i, b + j, c + k));
            }
    return 0.079577471545947667884 * s;
}

__device__ double newell_component(int comp, int I, int J, int K)
{
    if (I * I + J * J + K * K < kNewellFar * kNewellFar) {
        const double X = I, Y = J, Z = K;
        switch (comp) {
        case 0: return -newell_sum<false>(X, Y, Z);
        case 1: return -newell_sum<true>(X, Y, Z);
        case 2: return -newell_sum<true>(X, Z, Y);
        case 3: return -newell_sum<false>(Y, X, Z);
        case 4: return -newell_sum<true>(Y, Z, X);
        default: return -newell_sum<false>(Z, X, Y);
        }
    }
    // nodes and weights of 4-point Gauss-Legendre on [-1/2, 1/2]
    const double u[4] = {-0.43056815579702629, -0.16999052179242813, 0.16999052179242813,
                         0.43056815579702629};
    const double w[4] = {0.17392742256872693, 0.32607257743127307, 0.32607257743127307,
                         0.17392742256872693};
    double s = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c)
                s += w[a] * w[b] * w[c] * tensor_component(comp, I + u[a], J + u[b], K + u[c]);
    return s;
}

// kind 0: Eqs. 10-11 (the paper's tensor); kind 1: Newell's averaged tensor
__device__ inline double tensor_value(int kind, int comp, int I, int J, int K)
{
    return kind ? newell_component(comp, I, J, K) : tensor_component(comp, I, J, K);
}

// Wrapped offset of padded index q along an axis of n cells padded to P >= 2n-1:
// q < n -> q; q > P - n -> q - P; otherwise no offset (the entry is zero).
__device__ inline bool wrap_offset(int q, int n, int P, int* d)
{
    if (q < n) {
        *d = q;
        return true;
    }
    if (q > P - n) {
        *d = q - P;
        return true;
    }
    return false;
}

// Offsets one padded index stands for along an axis.  Open axis: the wrapped
// offset (or none).  Periodic axis (P = n): index t stands for every offset
// t + j n; the representative nearest zero is t (2t < n) or t - n (2t > n);
// at 2t = n both, weight 1/2 each, which keeps the parity of each tensor
// component under t -> n - t.  `images` multiples of n on either side of each
// representative are added.
struct AxisSet {
    int rep[2];
    int nrep;
    double w;
    int period, images;
};

__device__ inline bool axis_set(int q, int n, int P, bool periodic, int images, AxisSet* a)
{
    a->period = n;
    a->w = 1.0;
    a->nrep = 1;
    a->images = 0;
    if (!periodic) return wrap_offset(q, n, P, &a->rep[0]);
    a->images = images;
    if (2 * q < n) {
        a->rep[0] = q;
    } else if (2 * q > n) {
        a->rep[0] = q - n;
    } else {
        a->rep[0] = q;
        a->rep[1] = q - n;
        a->nrep = 2;
        a->w = 0.5;
    }
    return true;
}

__global__ void k_tensor_wrapped(double* out, int kind, int comp, int nx, int ny, int nz, int Px,
                                 int Py, int Pz, int per, int images)
{
    const int64_t total = (int64_t)Px * Py * Pz;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int qx = (int)(q % Px);
        const int qy = (int)((q / Px) % Py);
        const int qz = (int)(q / ((int64_t)Px * Py));
        AxisSet ax, ay, az;
        double v = 0.0;
        if (axis_set(qx, nx, Px, per & 1, images, &ax) && axis_set(qy, ny, Py, per & 2, images, &ay) &&
            axis_set(qz, nz, Pz, per & 4, images, &az)) {
            const double w = ax.w * ay.w * az.w;
            for (int rz = 0; rz < az.nrep; ++rz)
                for (int jz = -az.images; jz <= az.images; ++jz)
                    for (int ry = 0; ry < ay.nrep; ++ry)
                        for (int jy = -ay.images; jy <= ay.images; ++jy)
                            for (int rx = 0; rx < ax.nrep; ++rx)
                                for (int jx = -ax.images; jx <= ax.images; ++jx)
                                    v += w * tensor_value(kind, comp, ax.rep[rx] + jx * ax.period,
                                                          ay.rep[ry] + jy * ay.period,
                                                          az.rep[rz] + jz * az.period);
        }
        out[q] = v;
    }
}

__global__ void k_tensor_table(double* out, int kind, int nx, int ny, int nz)
{
    const int tx = 2 * nx - 1, ty = 2 * ny - 1, tz = 2 * nz - 1;
    const int64_t plane = (int64_t)tx * ty * tz;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < plane;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int I = (int)(q % tx) - (nx - 1);
        const int J = (int)((q / tx) % ty) - (ny - 1);
        const int K = (int)(q / ((int64_t)tx * ty)) - (nz - 1);
        for (int c = 0; c < 6; ++c) out[c * plane + q] = tensor_value(kind, c, I, J, K);
    }
}

template <typename T>
__global__ void k_twiddles(cpx<T>* tw, int P)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P) return;
    double s, c;
    sincospi(2.0 * (double)t / (double)P, &s, &c);
    tw[t] = cpx<T>{(T)c, (T)(-s)};
}

__device__ inline void atomic_max_pos(unsigned long long* a, double v)
{
    // non-negative doubles order like their bit patterns
    atomicMax(a, (unsigned long long)__double_as_longlong(v));
}

template <typename T>
__global__ void k_octant(T* out, const cpx<double>* spec, int hx, int Py, int Pz, int64_t sx,
                         double scale, unsigned long long* stats)
{
    const int oy = Py / 2 + 1, oz = Pz / 2 + 1;
    const int64_t total = (int64_t)oz * oy * hx;
    double im_max = 0.0, re_max = 0.0;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int ky = (int)(q % oy);
        const int kx = (int)((q / oy) % hx);
        const int kz = (int)(q / ((int64_t)hx * oy));
        const cpx<double> v = spec[((int64_t)kz * Py + ky) * sx + kx];
        out[q] = (T)(v.re * scale);
        im_max = fmax(im_max, fabs(v.im * scale));
        re_max = fmax(re_max, fabs(v.re * scale));
    }
    // one atomic per wave: reduce across the wave first
    for (int off = 32; off > 0; off >>= 1) {
        im_max = fmax(im_max, __shfl_xor(im_max, off));
        re_max = fmax(re_max, __shfl_xor(re_max, off));
    }
    if ((threadIdx.x & 63) == 0) {
        atomic_max_pos(&stats[0], im_max);
        atomic_max_pos(&stats[1], re_max);
    }
}

// Coefficient planes of the two-plane schedule (nz = 2) from the FP64 3-D
// spectrum of one component padded to Pz = 4 along z.  With K^(d) the 2-D
// spectrum of the tensor plane at z offset d, the z transform gives
// S(kz) = K^(0) + K^(1) (-i)^kz + K^(-1) i^kz.  Components even in z (xx, xy,
// yy, zz: K^(-1) = K^(1)): K^(0) = S(1), K^(1) = (S(0) - S(2)) / 4.  Odd in z
// (xz, yz: K^(0) = 0, K^(-1) = -K^(1) = -i s): S(1) = 2 s, the plane stores s.
// comp: 0 xx, 1 xy, 2 xz, 3 yy, 4 yz, 5 zz; out: that component's first plane
// (planes of hx (Py/2+1) values, ky fastest); scale = 1 / (Px Py).
template <typename T>
__global__ void k_table_z2(T* out, const cpx<double>* spec, int comp, int hx, int Py, int64_t sx,
                           double scale, unsigned long long* stats)
{
    const int oy = Py / 2 + 1;
    const int64_t plane = (int64_t)hx * oy;
    const bool odd = comp == 2 || comp == 4;
    double im_max = 0.0, re_max = 0.0;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < plane;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int ky = (int)(q % oy);
        const int kx = (int)(q / oy);
        const cpx<double> s0 = spec[((int64_t)0 * Py + ky) * sx + kx];
        const cpx<double> s1 = spec[((int64_t)1 * Py + ky) * sx + kx];
        const cpx<double> s2 = spec[((int64_t)2 * Py + ky) * sx + kx];
        if (odd) {
            out[q] = (T)(0.5 * s1.re * scale);
            im_max = fmax(im_max, fmax(fabs(s1.im), fmax(fabs(s0.re), fabs(s2.re))) * scale);
            re_max = fmax(re_max, fabs(s1.re * scale));
        } else {
            out[q] = (T)(s1.re * scale);
            out[plane + q] = (T)(0.25 * (s0.re - s2.re) * scale);
            im_max = fmax(im_max, fmax(fabs(s0.im), fmax(fabs(s1.im), fabs(s2.im))) * scale);
            re_max = fmax(re_max, fmax(fabs(s0.re), fabs(s2.re)) * scale);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        im_max = fmax(im_max, __shfl_xor(im_max, off));
        re_max = fmax(re_max, __shfl_xor(re_max, off));
    }
    if ((threadIdx.x & 63) == 0) {
        atomic_max_pos(&stats[0], im_max);
        atomic_max_pos(&stats[1], re_max);
    }
}

static int grid_for(int64_t n, int block)
{
    int64_t g = (n + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_tensor_wrapped(double* out, int kind, int comp, int nx, int ny, int nz, int Px,
                                 int Py, int Pz, int per, int images, hipStream_t s)
{
    const int64_t total = (int64_t)Px * Py * Pz;
    hipLaunchKernelGGL(k_tensor_wrapped, dim3(grid_for(total, 256)), dim3(256), 0, s, out, kind, comp,
                       nx, ny, nz, Px, Py, Pz, per, images);
    return hipGetLastError();
}

hipError_t launch_tensor_table(double* out, int kind, int nx, int ny, int nz, hipStream_t s)
{
    const int64_t total = (int64_t)(2 * nx - 1) * (2 * ny - 1) * (2 * nz - 1);
    hipLaunchKernelGGL(k_tensor_table, dim3(grid_for(total, 256)), dim3(256), 0, s, out, kind, nx, ny,
                       nz);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_twiddles(void* tw, int P, hipStream_t s)
{
    hipLaunchKernelGGL(k_twiddles<T>, dim3((P + 255) / 256), dim3(256), 0, s, (cpx<T>*)tw, P);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_octant(void* out, const void* spec, int hx, int Py, int Pz, int64_t sx,
                         double scale, unsigned long long* stats, hipStream_t s)
{
    const int64_t total = (int64_t)(Pz / 2 + 1) * (Py / 2 + 1) * hx;
    hipLaunchKernelGGL(k_octant<T>, dim3(grid_for(total, 256)), dim3(256), 0, s, (T*)out,
                       (const cpx<double>*)spec, hx, Py, Pz, sx, scale, stats);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_table_z2(void* out, const void* spec, int comp, int hx, int Py, int64_t sx,
                           double scale, unsigned long long* stats, hipStream_t s)
{
    const int64_t total = (int64_t)(Py / 2 + 1) * hx;
    hipLaunchKernelGGL(k_table_z2<T>, dim3(grid_for(total, 256)), dim3(256), 0, s, (T*)out,
                       (const cpx<double>*)spec, comp, hx, Py, sx, scale, stats);
    return hipGetLastError();
}

template hipError_t launch_table_z2<float>(void*, const void*, int, int, int, int64_t, double,
                                           unsigned long long*, hipStream_t);
template hipError_t launch_table_z2<double>(void*, const void*, int, int, int, int64_t, double,
                                            unsigned long long*, hipStream_t);
template hipError_t launch_twiddles<float>(void*, int, hipStream_t);
template hipError_t launch_twiddles<double>(void*, int, hipStream_t);
template hipError_t launch_octant<float>(void*, const void*, int, int, int, int64_t, double,
                                         unsigned long long*, hipStream_t);
template hipError_t launch_octant<double>(void*, const void*, int, int, int, int64_t, double,
                                          unsigned long long*, hipStream_t);

}  // namespace mm
