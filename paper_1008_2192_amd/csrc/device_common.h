// Device helpers shared by the detection kernel (detect.hip) and the other kernels
// of libcrb (kernels.hip).
#pragma once

#include "kernels.h"

namespace crb {

__device__ __forceinline__ float vmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ float vmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return fmax(a, b); }

__device__ __forceinline__ int clampi(int i, int n) { return min(max(i, 0), n - 1); }
__device__ __forceinline__ float med3f(float a, float b, float c) {
    return __builtin_amdgcn_fmed3f(a, b, c);
}
__device__ __forceinline__ float min3f(float a, float b, float c) { return fminf(fminf(a, b), c); }
__device__ __forceinline__ float max3f(float a, float b, float c) { return fmaxf(fmaxf(a, b), c); }

// Iteration k of frame f is skipped when k exceeds its niter, or (early stop) when
// the previous iteration selected no new pixel: that iteration reproduced its input,
// so every later one would too.
__device__ __forceinline__ bool frame_skips(const DevFrame &f, int k) {
    if (k < 1 || k > f.niter)
        return true;
    if (k == 1 || (f.flags & kNoEarlyStop))
        return false;
    return f.nnew[k - 2] == 0ull;
}

}  // namespace crb
