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

// Component comp (0..5 = xx, xy, xz, yy, yz, zz) at integer offset
// (I,J,K) = source - observer, in units of the cell edge: the eight-corner
// alternating sums of Eq. 10 (atan terms, diagonal) and Eq. 11 (log terms,
// off-diagonal, with the minus sign), over corners i,j,k in {0,1}.
__device__ double tensor_component(int comp, int I, int J, int K)
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

__global__ void k_tensor_wrapped(double* out, int comp, int nx, int ny, int nz, int Px, int Py,
                                 int Pz)
{
    const int64_t total = (int64_t)Px * Py * Pz;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int qx = (int)(q % Px);
        const int qy = (int)((q / Px) % Py);
        const int qz = (int)(q / ((int64_t)Px * Py));
        int I, J, K;
        double v = 0.0;
        if (wrap_offset(qx, nx, Px, &I) && wrap_offset(qy, ny, Py, &J) && wrap_offset(qz, nz, Pz, &K))
            v = tensor_component(comp, I, J, K);
        out[q] = v;
    }
}

__global__ void k_tensor_table(double* out, int nx, int ny, int nz)
{
    const int tx = 2 * nx - 1, ty = 2 * ny - 1, tz = 2 * nz - 1;
    const int64_t plane = (int64_t)tx * ty * tz;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < plane;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int I = (int)(q % tx) - (nx - 1);
        const int J = (int)((q / tx) % ty) - (ny - 1);
        const int K = (int)(q / ((int64_t)tx * ty)) - (nz - 1);
        for (int c = 0; c < 6; ++c) out[c * plane + q] = tensor_component(c, I, J, K);
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

static int grid_for(int64_t n, int block)
{
    int64_t g = (n + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_tensor_wrapped(double* out, int comp, int nx, int ny, int nz, int Px, int Py,
                                 int Pz, hipStream_t s)
{
    const int64_t total = (int64_t)Px * Py * Pz;
    hipLaunchKernelGGL(k_tensor_wrapped, dim3(grid_for(total, 256)), dim3(256), 0, s, out, comp, nx,
                       ny, nz, Px, Py, Pz);
    return hipGetLastError();
}

hipError_t launch_tensor_table(double* out, int nx, int ny, int nz, hipStream_t s)
{
    const int64_t total = (int64_t)(2 * nx - 1) * (2 * ny - 1) * (2 * nz - 1);
    hipLaunchKernelGGL(k_tensor_table, dim3(grid_for(total, 256)), dim3(256), 0, s, out, nx, ny, nz);
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

template hipError_t launch_twiddles<float>(void*, int, hipStream_t);
template hipError_t launch_twiddles<double>(void*, int, hipStream_t);
template hipError_t launch_octant<float>(void*, const void*, int, int, int, int64_t, double,
                                         unsigned long long*, hipStream_t);
template hipError_t launch_octant<double>(void*, const void*, int, int, int, int64_t, double,
                                          unsigned long long*, hipStream_t);

}  // namespace mm
