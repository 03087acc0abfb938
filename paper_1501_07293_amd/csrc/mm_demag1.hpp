// mm_demag1.hpp -- arguments and launcher of the one-work-group demag evaluation
// of a small grid (body in mm_generic.hpp, kernel in mm_passes.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mm_common.hpp"

namespace mm {

// One work-group holds the whole padded volume [3][Pz][Py][Px] of a small grid:
// m in, the reduced demag field out, every transform in LDS.
struct Demag1Args {
    const void* m;           // [3][nz][ny][nx]
    void* hd;                // [3][nz][ny][nx]
    int nx, ny, nz, Px, Py, Pz, hx;
    FftPlan plx, ply, plz;
    const void* twx;
    const void* twy;
    const void* twz;
    const void* kern;        // octant [ncomp][Pz/2+1][hx][Py/2+1]
    int ncomp;               // 6, or 4 (xx, xy, yy, zz) when Pz == 1
    int64_t k_cs, k_zs, k_xs;
};

// One work-group of nt threads; hipErrorInvalidValue (nothing launched) when the
// padded volume of the three components exceeds its LDS.
template <typename T>
hipError_t launch_demag_1wg(const Demag1Args& a, int nt, hipStream_t s);

}  // namespace mm
