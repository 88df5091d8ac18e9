// Chebyshev interpolation points of a cluster box (Section 4: tensor
// interpolation on the bounding box of every cluster).  Shared by the build
// kernels and by the apply kernel that regenerates the leaf row bases, so that
// both see the same points.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

namespace h2dlp {

// Point l of one box axis, first kind: c + h cos((2l + 1) pi / (2m)), with c
// the midpoint and h the half extent of [box[axis], box[3 + axis]].
__device__ inline double cheb_point(const double* box, int axis, int m, int l) {
    const double lo = box[axis], hi = box[3 + axis];
    const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
    return c + h * cos((2.0 * l + 1.0) * 3.14159265358979323846 / (2.0 * m));
}

}  // namespace h2dlp
