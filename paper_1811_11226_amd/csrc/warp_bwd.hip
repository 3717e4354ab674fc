// warp_bwd.hip -- adjoint kernels of the warp (gfx950).
//
// For every output voxel the forward coordinate and cell are recomputed; the
// eight corner values (fill substituted outside the volume) give the
// derivative of the trilinear interpolant on that cell, dV/dq.  Then
//   grad_img[c] += w_c * g          hardware FP32 atomics at L2 (no-return)
//   grad_disp[i](p) = g * dV/dq_i   coalesced SoA stores
//   per-tile partial of grad_M[i][j] = sum g dV/dq_i [x,y,z,1]_j, reduced in
//   FP64 inside the workgroup in a fixed order and written to workspace slot
//   (tile); a second kernel sums the slots in a fixed order.  grad_M is
//   therefore deterministic; grad_img is not (atomic order).
#include "device_common.h"
#include "launch.h"

namespace ctaug {

// Fixed launch shape of the backward pass: 4 x 8 x 32 voxel tiles.
constexpr Tiling kBwdTiling = {2, 3, 5};

int64_t bwd_num_tiles(int64_t ox, int64_t oy, int64_t oz)
{
    return ((ox + 3) >> 2) * ((oy + 7) >> 3) * ((oz + 31) >> 5);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T, bool DISP>
__global__ __launch_bounds__(kThreads) void k_warp_bwd(FwdJob J, const float *__restrict__ g,
                                                       float *__restrict__ g_img,
                                                       float *__restrict__ g_disp,
                                                       double *__restrict__ partials,
                                                       int32_t ntiles)
{
    const Tiling TL = kBwdTiling;
    const int b = blockIdx.x;
    const int per = (ntiles + 7) >> 3;
    const int t = (b & 7) * per + (b >> 3);
    if (t >= ntiles)
        return;   // uniform per workgroup: no barrier below is skipped by part of it
    const int tz = t % J.tiles_z, rest = t / J.tiles_z;
    const int ty = rest % J.tiles_y, tx = rest / J.tiles_y;
    const int x0 = tx << TL.lx, y0 = ty << TL.ly, z0 = tz << TL.lz;
    const Src src = make_src<T>(J.img, nullptr, J.nx, J.ny, J.nz);
    gconst<float> *disp = gc<float>(J.disp);
    const int32_t nvox = J.ox * J.oy * J.oz;
    const bool empty_in = J.nx == 0 || J.ny == 0 || J.nz == 0;   // every sample is fill

    double acc[12];
#pragma unroll
    for (int i = 0; i < 12; ++i)
        acc[i] = 0.0;

    const int runs_z_log = TL.lz - 2;
    const int nruns = 1 << (TL.lx + TL.ly + runs_z_log);
    for (int r = threadIdx.x; r < nruns; r += kThreads) {
        const int zr = r & ((1 << runs_z_log) - 1);
        const int rr = r >> runs_z_log;
        const int y = y0 + (rr & ((1 << TL.ly) - 1));
        const int x = x0 + (rr >> TL.ly);
        const int z = z0 + 4 * zr;
        if (x >= J.ox || y >= J.oy || z >= J.oz)
            continue;
        const int nvalid = min(4, J.oz - z);
        const int32_t v0 = (x * J.oy + y) * J.oz + z;
        float rb[3];
        row_base(J.M, (float)x, (float)y, rb);
        float S[3] = {0.0f, 0.0f, 0.0f}, Sz[3] = {0.0f, 0.0f, 0.0f};
        for (int k = 0; k < nvalid; ++k) {
            const int32_t v = v0 + k;
            const float zf = (float)(z + k);
            float qx = coord(J.M, 0, rb, zf), qy = coord(J.M, 1, rb, zf),
                  qz = coord(J.M, 2, rb, zf);
            if (DISP) {
                qx = qx + disp[v];
                qy = qy + disp[nvox + v];
                qz = qz + disp[2 * nvox + v];
            }
            const float gp = g[v];
            float dV[3] = {0.0f, 0.0f, 0.0f};
            if (!empty_in && in_guard(qx, qy, qz, J.nx, J.ny, J.nz)) {
                float K[8], tt[3];
                int32_t i0[3];
                corners_checked<T>(src, qx, qy, qz, J.fill, K, tt, i0);
                const float e00 = lerp(K[0], K[1], tt[2]), e01 = lerp(K[2], K[3], tt[2]);
                const float e10 = lerp(K[4], K[5], tt[2]), e11 = lerp(K[6], K[7], tt[2]);
                dV[0] = lerp(e10, e11, tt[1]) - lerp(e00, e01, tt[1]);
                dV[1] = lerp(e01 - e00, e11 - e10, tt[0]);
                dV[2] = lerp(lerp(K[1] - K[0], K[3] - K[2], tt[1]),
                             lerp(K[5] - K[4], K[7] - K[6], tt[1]), tt[0]);
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
                                const int32_t cx = i0[0] + a, cy = i0[1] + bb, cz = i0[2] + c;
                                const float w = wx[a] * wy[bb] * wz[c];
                                const bool ok = cx >= 0 && cx < J.nx && cy >= 0 && cy < J.ny &&
                                                cz >= 0 && cz < J.nz && w != 0.0f;
                                if (ok)
                                    unsafeAtomicAdd(g_img + (cx * J.ny + cy) * J.nz + cz, w * gp);
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

    if (!partials)
        return;
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
        partials[(int64_t)t * 12 + threadIdx.x] = s;
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
    J.tiles_x = (J.ox + 3) >> 2;
    J.tiles_y = (J.oy + 7) >> 3;
    J.tiles_z = (J.oz + 31) >> 5;
    const int ntiles = J.tiles_x * J.tiles_y * J.tiles_z;
    if (ntiles == 0) {
        if (g_M) {
            hipLaunchKernelGGL(k_reduce12, dim3(1), dim3(kThreads), 0, s, partials, 0, g_M);
            return hipGetLastError();
        }
        return hipSuccess;
    }
    const int grid = ((ntiles + 7) >> 3) << 3;
    double *part = g_M ? partials : nullptr;
    const bool disp = J.disp != nullptr;
    if (J.dtype == kI16) {
        if (disp)
            hipLaunchKernelGGL((k_warp_bwd<int16_t, true>), dim3(grid), dim3(kThreads), 0, s, J, g,
                               g_img, g_disp, part, ntiles);
        else
            hipLaunchKernelGGL((k_warp_bwd<int16_t, false>), dim3(grid), dim3(kThreads), 0, s, J, g,
                               g_img, g_disp, part, ntiles);
    } else {
        if (disp)
            hipLaunchKernelGGL((k_warp_bwd<float, true>), dim3(grid), dim3(kThreads), 0, s, J, g,
                               g_img, g_disp, part, ntiles);
        else
            hipLaunchKernelGGL((k_warp_bwd<float, false>), dim3(grid), dim3(kThreads), 0, s, J, g,
                               g_img, g_disp, part, ntiles);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !g_M)
        return e;
    hipLaunchKernelGGL(k_reduce12, dim3(1), dim3(kThreads), 0, s, partials, ntiles, g_M);
    return hipGetLastError();
}

}  // namespace ctaug
