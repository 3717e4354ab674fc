// smooth.hip -- separable Gaussian smoothing of the resampling pre-step
// (gfx950).  One pass per smoothed axis, one thread per output voxel: the
// 2R+1 taps along the axis come from L1/L2 (neighbouring threads share them),
// with edge voxels repeated beyond the volume.  The grid maps (z block, y, x)
// to workgroups, so no thread divides an index.  Accumulation in FP32 with
// FP32 weights normalised on the host in FP64.
#include "device_common.h"
#include "launch.h"

#include <algorithm>
#include <cmath>

namespace ctaug {

template <typename T>
__global__ __launch_bounds__(kThreads) void k_smooth_axis(const T *__restrict__ in,
                                                          float *__restrict__ out, int32_t nx,
                                                          int32_t ny, int32_t nz, int32_t axis,
                                                          GaussTaps K)
{
    const int z = blockIdx.x * kThreads + threadIdx.x;
    const int y = blockIdx.y, x = blockIdx.z;
    if (z >= nz)
        return;
    const int32_t e = (x * ny + y) * nz + z;
    const int i = axis == 0 ? x : axis == 1 ? y : z;
    const int n = axis == 0 ? nx : axis == 1 ? ny : nz;
    const int32_t stride = axis == 0 ? ny * nz : axis == 1 ? nz : 1;
    float acc = K.w[0] * (float)in[e];
    for (int d = 1; d <= K.R; ++d) {
        const int lo = max(i - d, 0) - i, hi = min(i + d, n - 1) - i;
        acc = __builtin_fmaf(K.w[d], (float)in[e + lo * stride] + (float)in[e + hi * stride], acc);
    }
    out[e] = acc;
}

int32_t gauss_radius(float sigma)
{
    return sigma > 0.0f ? (int32_t)std::floor(3.0 * (double)sigma / std::sqrt(2.0) + 0.5) : 0;
}

GaussTaps gauss_taps(float sigma)
{
    GaussTaps K;
    K.R = gauss_radius(sigma);
    double w[kMaxGaussRadius + 1];
    double sum = 0.0;
    for (int d = 0; d <= K.R; ++d) {
        // R = 0 (sigma = 0 included): the single tap 1
        w[d] = K.R == 0 ? 1.0 : std::exp(-(double)d * (double)d / ((double)sigma * (double)sigma));
        sum += d == 0 ? w[d] : 2.0 * w[d];
    }
    for (int d = 0; d <= kMaxGaussRadius; ++d)
        K.w[d] = d <= K.R ? (float)(w[d] / sum) : 0.0f;
    return K;
}

hipError_t launch_smooth_axis(const void *in, bool in_i16, float *out, const int32_t dim[3],
                              int axis, const GaussTaps &K, hipStream_t s)
{
    const dim3 grid((unsigned)((dim[2] + kThreads - 1) / kThreads), (unsigned)dim[1],
                    (unsigned)dim[0]);
    if (in_i16)
        hipLaunchKernelGGL(k_smooth_axis<int16_t>, grid, dim3(kThreads), 0, s,
                           static_cast<const int16_t *>(in), out, dim[0], dim[1], dim[2], axis, K);
    else
        hipLaunchKernelGGL(k_smooth_axis<float>, grid, dim3(kThreads), 0, s,
                           static_cast<const float *>(in), out, dim[0], dim[1], dim[2], axis, K);
    return hipGetLastError();
}

}  // namespace ctaug
