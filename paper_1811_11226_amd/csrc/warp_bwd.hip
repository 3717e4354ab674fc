// warp_bwd.hip -- adjoint kernels of the warp (gfx950).
//
// For every output voxel the forward coordinate and cell are recomputed; the
// eight corner values (fill substituted outside the volume) give the
// derivative of the trilinear interpolant on that cell, dV/dq.  Then
//   grad_img[c] += w_c * g          affine warps: FP32 atomics into LDS
//                                   accumulators over the tile's input
//                                   footprint, then one global FP32 atomic
//                                   per touched cell (8x fewer than per corner);
//                                   displacement warps (no footprint bound):
//                                   global FP32 atomics per corner
//   grad_disp[i](p) = g * dV/dq_i   coalesced SoA stores
//   per-tile partial of grad_M[i][j] = sum g dV/dq_i [x,y,z,1]_j, reduced in
//   FP64 inside the workgroup in a fixed order and written to workspace slot
//   (tile); a second kernel sums the slots in a fixed order.  grad_M is
//   therefore deterministic; grad_img is not (atomic order).
#include "device_common.h"
#include "launch.h"
#include "tile_geom.h"

#include <algorithm>
#include <climits>

namespace ctaug {

// Launch shape of the backward pass: 8 x 8 x 16 voxel tiles (one run of 4 z
// voxels per thread), persistent workgroups striding over their XCD's tile
// range, and at most kBwdLdsCells FP32 cells of input footprint per
// workgroup (48 KB of LDS), used first for the staged image, then as the
// adjoint accumulators of the same cells.
constexpr Tiling kBwdTiling = {3, 3, 4};
constexpr int32_t kBwdLdsCells = 12288;
constexpr int64_t kBwdMaxGrid = 2048;

static int64_t bwd_tiles(int64_t ox, int64_t oy, int64_t oz)
{
    return ((ox + 7) >> 3) * ((oy + 7) >> 3) * ((oz + 15) >> 4);
}

static int64_t bwd_grid(int64_t ntiles)
{
    return std::min(((ntiles + 7) >> 3) << 3, kBwdMaxGrid);
}

int64_t bwd_partial_rows(int64_t ox, int64_t oy, int64_t oz)
{
    return bwd_grid(bwd_tiles(ox, oy, oz));
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

extern __shared__ __attribute__((aligned(16))) float s_cells[];

// Derivative of the trilinear interpolant on the cell with corners K[a][b][c]
// (a: x, b: y, c: z) at fractions tt.
__device__ __forceinline__ void cell_gradient(const float K[8], const float tt[3], float dV[3])
{
    const float e00 = lerp(K[0], K[1], tt[2]), e01 = lerp(K[2], K[3], tt[2]);
    const float e10 = lerp(K[4], K[5], tt[2]), e11 = lerp(K[6], K[7], tt[2]);
    dV[0] = lerp(e10, e11, tt[1]) - lerp(e00, e01, tt[1]);
    dV[1] = lerp(e01 - e00, e11 - e10, tt[0]);
    dV[2] = lerp(lerp(K[1] - K[0], K[3] - K[2], tt[1]), lerp(K[5] - K[4], K[7] - K[6], tt[1]),
                 tt[0]);
}

template <typename T, bool DISP>
__global__ __launch_bounds__(kThreads) void k_warp_bwd(FwdJob J, const float *__restrict__ g,
                                                       float *__restrict__ g_img,
                                                       float *__restrict__ g_disp,
                                                       double *__restrict__ partials,
                                                       int32_t ntiles, int32_t lds_cells)
{
    const Tiling TL = kBwdTiling;
    const int b = blockIdx.x;
    const int per_xcd_wg = gridDim.x >> 3;
    const int per = (ntiles + 7) >> 3;
    const int start = (b & 7) * per;
    const int end = min(start + per, ntiles);
    const Src src = make_src<T>(J.img, nullptr, J.nx, J.ny, J.nz);
    gconst<float> *disp = gc<float>(J.disp);
    const int32_t nvox = J.ox * J.oy * J.oz;
    const bool empty_in = J.nx == 0 || J.ny == 0 || J.nz == 0;   // every sample is fill

    double acc[12];
#pragma unroll
    for (int i = 0; i < 12; ++i)
        acc[i] = 0.0;

    __shared__ int s_red[kThreads / 64][6];

    // this thread's run inside every tile
    const int zr = threadIdx.x & 3;
    const int yr = (threadIdx.x >> 2) & 7;
    const int xr = threadIdx.x >> 5;

    for (int t = start + (b >> 3); t < end; t += per_xcd_wg) {
        const int tz = t % J.tiles_z, rest = t / J.tiles_z;
        const int ty = rest % J.tiles_y, tx = rest / J.tiles_y;
        const int x0 = tx << TL.lx, y0 = ty << TL.ly, z0 = tz << TL.lz;
        const int x1 = min(x0 + (1 << TL.lx), J.ox) - 1, y1 = min(y0 + (1 << TL.ly), J.oy) - 1,
                  z1 = min(z0 + (1 << TL.lz), J.oz) - 1;
        const int x = x0 + xr, y = y0 + yr, z = z0 + 4 * zr;
        const bool run_ok = x <= x1 && y <= y1 && z <= z1;
        const int nvalid = run_ok ? min(4, J.oz - z) : 0;
        const int32_t v0 = run_ok ? (x * J.oy + y) * J.oz + z : 0;
        // coordinates, guard and upstream gradient of the run's voxels
        float qv[4][3], gpk[4];
        bool gd[4];
        {
            float rb[3];
            row_base(J.M, (float)x, (float)y, rb);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                gd[k] = false;
                gpk[k] = 0.0f;
                qv[k][0] = qv[k][1] = qv[k][2] = 0.0f;
                if (k >= nvalid)
                    continue;
                const int32_t v = v0 + k;
                const float zf = (float)(z + k);
                float qx = coord(J.M, 0, rb, zf), qy = coord(J.M, 1, rb, zf),
                      qz = coord(J.M, 2, rb, zf);
                if (DISP) {
                    qx = qx + disp[v];
                    qy = qy + disp[nvox + v];
                    qz = qz + disp[2 * nvox + v];
                }
                qv[k][0] = qx;
                qv[k][1] = qy;
                qv[k][2] = qz;
                gd[k] = !empty_in && in_guard(qx, qy, qz, J.nx, J.ny, J.nz);
                gpk[k] = g[v];
            }
        }
        TileGeom G;
        if (DISP) {
            // no a-priori bound with a displacement field: the footprint is the
            // range of floor(q) over the tile's guarded samples (block reduction)
            int fmn[3] = {INT_MAX, INT_MAX, INT_MAX}, fmx[3] = {INT_MIN, INT_MIN, INT_MIN};
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (gd[k])
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const int f = (int)floorf(qv[k][i]);
                        fmn[i] = min(fmn[i], f);
                        fmx[i] = max(fmx[i], f);
                    }
            block_minmax3(fmn, fmx, s_red);
            G = geom_from_cells(J, x0, y0, z0, x1, y1, z1, fmn, fmx, lds_cells);
        } else {
            G = box_geom(J, x0, y0, z0, x1, y1, z1, lds_cells);
        }
        const bool lds = G.lds;
        const int ey = G.e[1], pitch = G.pitch, sxy = G.e[1] * G.pitch;
        if (lds) {
            stage_footprint<T, float>(J, src, G, s_cells, nullptr);
            __syncthreads();
        }
        // per voxel of the run: LDS cell of corner (0,0,0), fractions, upstream gradient
        int base[4];
        float tw[4][3], gk[4];
        bool live[4] = {false, false, false, false};
        float S[3] = {0.0f, 0.0f, 0.0f}, Sz[3] = {0.0f, 0.0f, 0.0f};
        if (run_ok) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k >= nvalid)
                    continue;
                const int32_t v = v0 + k;
                const float zf = (float)(z + k);
                const float qx = qv[k][0], qy = qv[k][1], qz = qv[k][2];
                const float gp = gpk[k];
                float dV[3] = {0.0f, 0.0f, 0.0f};
                if (gd[k]) {
                    float K[8], tt[3];
                    if (lds) {
                        const float fx = floorf(qx), fy = floorf(qy), fz = floorf(qz);
                        const int bs = (int)mul24(mul24((uint32_t)((int)fx - G.lo[0]),
                                                        (uint32_t)ey) +
                                                      (uint32_t)((int)fy - G.lo[1]),
                                                  (uint32_t)pitch) +
                                       ((int)fz - G.lo[2]);
                        K[0] = s_cells[bs];
                        K[1] = s_cells[bs + 1];
                        K[2] = s_cells[bs + pitch];
                        K[3] = s_cells[bs + pitch + 1];
                        K[4] = s_cells[bs + sxy];
                        K[5] = s_cells[bs + sxy + 1];
                        K[6] = s_cells[bs + sxy + pitch];
                        K[7] = s_cells[bs + sxy + pitch + 1];
                        tt[0] = qx - fx;
                        tt[1] = qy - fy;
                        tt[2] = qz - fz;
                        cell_gradient(K, tt, dV);
                        if (g_img) {
                            live[k] = true;
                            base[k] = bs;
                            tw[k][0] = tt[0];
                            tw[k][1] = tt[1];
                            tw[k][2] = tt[2];
                            gk[k] = gp;
                        }
                    } else {
                        int32_t i0[3];
                        corners_checked<T>(src, qx, qy, qz, J.fill, K, tt, i0);
                        cell_gradient(K, tt, dV);
                        if (g_img && gp != 0.0f) {
                            const float wx[2] = {1.0f - tt[0], tt[0]};
                            const float wy[2] = {1.0f - tt[1], tt[1]};
                            const float wz[2] = {1.0f - tt[2], tt[2]};
#pragma unroll
                            for (int a = 0; a < 2; ++a)
#pragma unroll
                                for (int bb = 0; bb < 2; ++bb)
#pragma unroll
                                    for (int c = 0; c < 2; ++c) {
                                        const int32_t cx = i0[0] + a, cy = i0[1] + bb,
                                                      cz = i0[2] + c;
                                        const float w = wx[a] * wy[bb] * wz[c];
                                        const bool ok = cx >= 0 && cx < J.nx && cy >= 0 &&
                                                        cy < J.ny && cz >= 0 && cz < J.nz &&
                                                        w != 0.0f;
                                        if (ok)
                                            unsafeAtomicAdd(g_img + (cx * J.ny + cy) * J.nz + cz,
                                                            w * gp);
                                    }
                        }
                    }
                }
                if (DISP && g_disp) {
                    g_disp[v] = gp * dV[0];
                    g_disp[nvox + v] = gp * dV[1];
                    g_disp[2 * nvox + v] = gp * dV[2];
                }
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const float c = gp * dV[i];
                    S[i] += c;
                    Sz[i] = __builtin_fmaf(c, zf, Sz[i]);
                }
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                acc[4 * i + 0] += (double)x * (double)S[i];
                acc[4 * i + 1] += (double)y * (double)S[i];
                acc[4 * i + 2] += (double)Sz[i];
                acc[4 * i + 3] += (double)S[i];
            }
        }
        if (!lds)
            continue;                      // uniform: no barrier is skipped by part of the group
        __syncthreads();                   // every corner read of the staged image is done
        if (g_img) {
            // the footprint cells become FP32 accumulators of w_c * g
            const int cells = G.e[0] * sxy;
            for (int c = 4 * threadIdx.x; c < cells; c += 4 * kThreads)
                *reinterpret_cast<f32x4 *>(s_cells + c) = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!live[k])
                    continue;
                const float wx[2] = {1.0f - tw[k][0], tw[k][0]};
                const float wy[2] = {1.0f - tw[k][1], tw[k][1]};
                const float gz0 = (1.0f - tw[k][2]) * gk[k], gz1 = tw[k][2] * gk[k];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int bb = 0; bb < 2; ++bb) {
                        const float wxy = wx[a] * wy[bb];
                        float *row = s_cells + base[k] + a * sxy + bb * pitch;
                        atomicAdd(row, wxy * gz0);
                        atomicAdd(row + 1, wxy * gz1);
                    }
            }
            __syncthreads();
            // flush: one global atomic per touched in-volume footprint cell
            const float rcp_pitch = 1.0f / (float)pitch, rcp_ey = 1.0f / (float)ey;
            for (int c = threadIdx.x; c < cells; c += kThreads) {
                const float v = s_cells[c];
                if (v == 0.0f)
                    continue;
                const int row = div_small(c, pitch, rcp_pitch);
                const int cz = c - row * pitch;
                const int cx = div_small(row, ey, rcp_ey);
                const int cy = row - cx * ey;
                const int gx = G.lo[0] + cx, gy = G.lo[1] + cy, gz = G.lo[2] + cz;
                if (cz < G.e[2] && (unsigned)gx < (unsigned)J.nx &&
                    (unsigned)gy < (unsigned)J.ny && (unsigned)gz < (unsigned)J.nz)
                    unsafeAtomicAdd(g_img + (gx * J.ny + gy) * J.nz + gz, v);
            }
            __syncthreads();               // LDS is restaged by the next tile
        }
    }

    if (!partials)
        return;
    __shared__ double red[kThreads / 64][12];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        const double sum = wave_sum(acc[i]);
        if (lane == 0)
            red[wave][i] = sum;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
        double sum = 0.0;
        for (int w = 0; w < kThreads / 64; ++w)
            sum += red[w][threadIdx.x];
        partials[(int64_t)blockIdx.x * 12 + threadIdx.x] = sum;
    }
}

// Sum n rows of 12 doubles in a fixed order into out[12].
__global__ __launch_bounds__(kThreads) void k_reduce12(const double *__restrict__ partials,
                                                       int32_t n, double *__restrict__ out)
{
    double acc[12];
#pragma unroll
    for (int i = 0; i < 12; ++i)
        acc[i] = 0.0;
    for (int r = threadIdx.x; r < n; r += kThreads)
#pragma unroll
        for (int i = 0; i < 12; ++i)
            acc[i] += partials[(int64_t)r * 12 + i];
    __shared__ double red[kThreads / 64][12];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        const double s = wave_sum(acc[i]);
        if (lane == 0)
            red[wave][i] = s;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
        double s = 0.0;
        for (int w = 0; w < kThreads / 64; ++w)
            s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

hipError_t launch_warp_bwd(const FwdJob &J0, const float *g, float *g_img, float *g_disp,
                           double *g_M, double *partials, hipStream_t s)
{
    FwdJob J = J0;
    J.tiles_x = (J.ox + 7) >> 3;
    J.tiles_y = (J.oy + 7) >> 3;
    J.tiles_z = (J.oz + 15) >> 4;
    const int64_t ntiles = (int64_t)J.tiles_x * J.tiles_y * J.tiles_z;
    if (ntiles == 0) {
        if (g_M) {
            hipLaunchKernelGGL(k_reduce12, dim3(1), dim3(kThreads), 0, s, partials, 0, g_M);
            return hipGetLastError();
        }
        return hipSuccess;
    }
    const int grid = (int)bwd_grid(ntiles);
    // LDS cells sized for the largest footprint of any tile (a displacement field
    // has no a-priori bound: the full reservation, used when a tile fits it)
    const int32_t cells =
        J.disp ? kBwdLdsCells : std::min(footprint_cells_bound(J, kBwdTiling), kBwdLdsCells);
    const size_t lds = (size_t)cells * sizeof(float);
    double *part = g_M ? partials : nullptr;
    const bool disp = J.disp != nullptr;
    const int nt = (int)ntiles;
    if (J.dtype == kI16) {
        if (disp)
            hipLaunchKernelGGL((k_warp_bwd<int16_t, true>), dim3(grid), dim3(kThreads), lds, s, J,
                               g, g_img, g_disp, part, nt, cells);
        else
            hipLaunchKernelGGL((k_warp_bwd<int16_t, false>), dim3(grid), dim3(kThreads), lds, s,
                               J, g, g_img, g_disp, part, nt, cells);
    } else {
        if (disp)
            hipLaunchKernelGGL((k_warp_bwd<float, true>), dim3(grid), dim3(kThreads), lds, s, J,
                               g, g_img, g_disp, part, nt, cells);
        else
            hipLaunchKernelGGL((k_warp_bwd<float, false>), dim3(grid), dim3(kThreads), lds, s, J,
                               g, g_img, g_disp, part, nt, cells);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !g_M)
        return e;
    hipLaunchKernelGGL(k_reduce12, dim3(1), dim3(kThreads), 0, s, partials, grid, g_M);
    return hipGetLastError();
}

}  // namespace ctaug
