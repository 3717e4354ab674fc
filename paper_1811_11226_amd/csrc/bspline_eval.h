// bspline_eval.h -- evaluation of the uniform cubic B-spline displacement
// field (internal), shared by the upsampling kernel, the fused warp and the
// fused adjoint so that every path computes the same bits.
//
// Control j of an axis with n output voxels and G controls sits at output
// coordinate (j - 1) h with h = (n - 1) / (G - 3); output voxel p lies in cell
// i = min(floor(p / h), G - 4) at fraction t = p / h - i and takes
//   u(p) = sum_{a,b,c} B_a(t_x) B_b(t_y) B_c(t_z) C[i_x + a][i_y + b][i_z + c]
// with the uniform cubic B-spline basis B_0..B_3.  Order of operations (FP32,
// every multiply-add fused and written out): the row profile
//   P(x, y, gz) = sum_a B_a(t_x) (sum_b B_b(t_y) C[i_x + a][i_y + b][gz])
// accumulated b = 0..3 inside a = 0..3, then u = sum_c B_c(t_z) P(x, y, i_z + c)
// accumulated c = 0..3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ctaug {

struct BsplineGeom {
    int32_t ox, oy, oz;                // output (field) dims
    int32_t gx, gy, gz;                // control grid dims, each >= 4
    float inv_hx, inv_hy, inv_hz;      // (G - 3) / (n - 1), or 0 when n == 1
};

// Cell index and fraction of output coordinate p on one axis.
__device__ __forceinline__ void bs_cell(int32_t p, float inv_h, int32_t G, int32_t &i, float &t)
{
    const float s = (float)p * inv_h;
    const float f = fminf(floorf(s), (float)(G - 4));
    i = (int32_t)f;
    t = s - f;
}

__device__ __forceinline__ int32_t bs_index(int32_t p, float inv_h, int32_t G)
{
    return (int32_t)fminf(floorf((float)p * inv_h), (float)(G - 4));
}

__device__ __forceinline__ void bs_basis(float t, float B[4])
{
    const float t2 = t * t, t3 = t2 * t, m = 1.0f - t;
    const float sixth = 1.0f / 6.0f;
    B[0] = m * m * m * sixth;
    B[1] = __builtin_fmaf(3.0f, t3, __builtin_fmaf(-6.0f, t2, 4.0f)) * sixth;
    B[2] = __builtin_fmaf(-3.0f, t3, __builtin_fmaf(3.0f, t2, __builtin_fmaf(3.0f, t, 1.0f))) * sixth;
    B[3] = t3 * sixth;
}

// Row profile P(x, y, gz) of component comp (control layout [3][gx][gy][gz]).
__device__ __forceinline__ float bs_profile(const float *__restrict__ ctrl, const BsplineGeom &G,
                                            int comp, int32_t x, int32_t y, int32_t gz)
{
    int32_t ix, iy;
    float tx, ty, Bx[4], By[4];
    bs_cell(x, G.inv_hx, G.gx, ix, tx);
    bs_basis(tx, Bx);
    bs_cell(y, G.inv_hy, G.gy, iy, ty);
    bs_basis(ty, By);
    const int64_t gstride = (int64_t)G.gx * G.gy * G.gz;
    float s = 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        float sa = 0.0f;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            sa = __builtin_fmaf(By[b],
                                ctrl[comp * gstride + ((int64_t)(ix + a) * G.gy + (iy + b)) * G.gz + gz],
                                sa);
        s = __builtin_fmaf(Bx[a], sa, s);
    }
    return s;
}

// Host: geometry of a control grid G over output dims od.
inline BsplineGeom bspline_geom(const int64_t G[3], const int64_t od[3])
{
    BsplineGeom g;
    g.ox = (int32_t)od[0];
    g.oy = (int32_t)od[1];
    g.oz = (int32_t)od[2];
    g.gx = (int32_t)G[0];
    g.gy = (int32_t)G[1];
    g.gz = (int32_t)G[2];
    g.inv_hx = od[0] > 1 ? (float)((double)(G[0] - 3) / (double)(od[0] - 1)) : 0.0f;
    g.inv_hy = od[1] > 1 ? (float)((double)(G[1] - 3) / (double)(od[1] - 1)) : 0.0f;
    g.inv_hz = od[2] > 1 ? (float)((double)(G[2] - 3) / (double)(od[2] - 1)) : 0.0f;
    return g;
}

}  // namespace ctaug
