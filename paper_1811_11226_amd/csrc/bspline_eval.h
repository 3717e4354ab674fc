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

// Displacement of one thread's run of a tile of 2^lx x 2^ly rows (x, y) by
// 2^lz voxels along z, evaluated from the control grid: the row profiles of
// the tile's rows over its z-control window are computed into s_prof (LDS,
// up to 64 rows; 64 * 3 * kSplineWindow floats, plus the control window and
// the y contraction, 4 * 3 * 64 * kSplineWindow floats in all, when the tile
// touches at most kSplineWindow controls along x and y), then each thread contracts z for its
// own voxels z + k * zstep, k < nvalid, of row rr (x = x0 + (rr >> ly), y =
// y0 + (rr & (2^ly - 1))).  A window of more than kSplineWindow controls (controls
// closer than about 4 voxels along z) evaluates the profiles per voxel when
// PER_VOXEL is set; without it the caller guarantees that every window fits.
// Contains a workgroup barrier: every thread of the workgroup calls it.
constexpr int kSplineWindow = 8;
constexpr int kSplineTileLdsFloats = 3 * 64 * kSplineWindow + 3 * kSplineWindow * kSplineWindow *
                                     kSplineWindow + kSplineWindow * 8 * 3 * kSplineWindow;

template <int NT, bool PER_VOXEL = true>
__device__ __forceinline__ void spline_tile_u(const float *__restrict__ ctrl, const BsplineGeom &B,
                                              int lx, int ly, int x0, int y0, int z0, int x1,
                                              int y1, int z1, int rr, int x, int y, int z,
                                              int zstep, int nvalid, bool mine, float *s_prof,
                                              float (&u)[3][4])
{
    const int izl = bs_index(z0, B.inv_hz, B.gz);
    const int ncz = bs_index(z1, B.inv_hz, B.gz) - izl + 4;
    if (!PER_VOXEL || ncz <= kSplineWindow) {
        const int per_row = 3 * ncz;
        const int nent = per_row << (lx + ly);
        const int ixl = bs_index(x0, B.inv_hx, B.gx), iyl = bs_index(y0, B.inv_hy, B.gy);
        const int ncx = bs_index(x1, B.inv_hx, B.gx) - ixl + 4;
        const int ncy = bs_index(y1, B.inv_hy, B.gy) - iyl + 4;
        if (ncx <= kSplineWindow && ncy <= kSplineWindow) {
            // separable, from the tile's control window staged in LDS: the same
            // fmaf chains as bs_profile, sharing the y contraction of a control
            // column among the rows of one y
            float *Wc = s_prof + kSplineWindow * 3 * 64;                   // [3][ncx][ncy][ncz]
            float *S = Wc + 3 * kSplineWindow * kSplineWindow * kSplineWindow;  // [ncx][ny][3][ncz]
            const int ny = 1 << ly;
            const int64_t gstride = (int64_t)B.gx * B.gy * B.gz;
            const int nw = 3 * ncx * ncy * ncz;
            for (int e = threadIdx.x; e < nw; e += NT) {
                const int c = e % ncz, r1 = e / ncz;
                const int b = r1 % ncy, r2 = r1 / ncy;
                const int a = r2 % ncx, comp = r2 / ncx;
                Wc[e] = ctrl[comp * gstride + ((int64_t)(ixl + a) * B.gy + (iyl + b)) * B.gz +
                             izl + c];
            }
            __syncthreads();
            const int ns = ncx * ny * per_row;
            for (int e = threadIdx.x; e < ns; e += NT) {
                const int cc = e % per_row, r1 = e / per_row;
                const int yr = r1 % ny, a = r1 / ny;
                const int comp = cc / ncz, c = cc - comp * ncz;
                int32_t iy;
                float ty, By[4];
                bs_cell(min(y0 + yr, y1), B.inv_hy, B.gy, iy, ty);
                bs_basis(ty, By);
                const float *w = Wc + ((comp * ncx + a) * ncy + (iy - iyl)) * ncz + c;
                float sa = 0.0f;
#pragma unroll
                for (int bb = 0; bb < 4; ++bb)
                    sa = __builtin_fmaf(By[bb], w[bb * ncz], sa);
                S[e] = sa;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < nent; e += NT) {
                const int row = e / per_row;
                const int cc = e - row * per_row;
                const int yr = row & (ny - 1);
                int32_t ix;
                float tx, Bx[4];
                bs_cell(min(x0 + (row >> ly), x1), B.inv_hx, B.gx, ix, tx);
                bs_basis(tx, Bx);
                const float *sp = S + ((ix - ixl) * ny + yr) * per_row + cc;
                float sv = 0.0f;
#pragma unroll
                for (int a = 0; a < 4; ++a)
                    sv = __builtin_fmaf(Bx[a], sp[a * ny * per_row], sv);
                s_prof[e] = sv;
            }
        } else {
            for (int e = threadIdx.x; e < nent; e += NT) {
                const int row = e / per_row;
                const int rem = e - row * per_row;
                const int comp = rem / ncz, c = rem - comp * ncz;
                const int px = min(x0 + (row >> ly), x1);
                const int py = min(y0 + (row & ((1 << ly) - 1)), y1);
                s_prof[e] = bs_profile(ctrl, B, comp, px, py, izl + c);
            }
        }
        __syncthreads();
        if (!mine)
            return;
        const float *P = s_prof + rr * per_row - izl;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k >= nvalid)
                break;
            int32_t iz;
            float tz, Bz[4];
            bs_cell(z + k * zstep, B.inv_hz, B.gz, iz, tz);
            bs_basis(tz, Bz);
#pragma unroll
            for (int comp = 0; comp < 3; ++comp) {
                float s = 0.0f;
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    s = __builtin_fmaf(Bz[c], P[comp * ncz + iz + c], s);
                u[comp][k] = s;
            }
        }
    } else if (PER_VOXEL && mine) {
        for (int k = 0; k < nvalid; ++k) {
            int32_t iz;
            float tz, Bz[4];
            bs_cell(z + k * zstep, B.inv_hz, B.gz, iz, tz);
            bs_basis(tz, Bz);
#pragma unroll
            for (int comp = 0; comp < 3; ++comp) {
                float s = 0.0f;
#pragma unroll 1
                for (int c = 0; c < 4; ++c) {
                    const float bz = c == 0 ? Bz[0] : c == 1 ? Bz[1] : c == 2 ? Bz[2] : Bz[3];
                    s = __builtin_fmaf(bz, bs_profile(ctrl, B, comp, x, y, iz + c), s);
                }
                u[comp][k] = s;
            }
        }
    }
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
