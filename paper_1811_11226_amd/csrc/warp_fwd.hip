// warp_fwd.hip -- fused forward augmentation kernels for gfx950.
//
// One workgroup (256 threads, 4 wave64) per output tile; each thread owns
// runs of 4 consecutive output voxels along z, so that output stores are one
// 16-byte store of intensities plus one 4-byte store of labels, and the four
// Gaussians of a run come from one Philox call.  Per voxel: the pinned FP32
// coordinate, a trilinear gather of the image and a nearest-neighbour gather
// of the labels, then gain/offset, noise, window and gamma in registers.
//
// Each tile is classified once (uniformly for the workgroup) from the
// coordinates of its eight corners, widened by a bound on FP32 rounding:
//   outside  -- every sample fails the (-1, n) guard: fill / label_fill only;
//   interior -- every cell floor(q)..floor(q)+1 is inside the volume: no
//               per-corner bounds checks;
//   boundary -- per-sample guard and per-corner fill substitution.
// The three paths compute identical values where they overlap.
//
// Workgroup-to-tile mapping is XCD-aware: consecutive workgroup ids are
// dispatched round-robin over the 8 XCDs, so workgroup b takes tile
// (b % 8) * ceil(T/8) + b / 8, giving each XCD (and its L2) a contiguous,
// spatially coherent range of tiles.
#include "device_common.h"
#include "launch.h"

#include <algorithm>

namespace ctaug {

enum : int { kOutside = 0, kInterior = 1, kBoundary = 2 };

__device__ __forceinline__ int classify_tile(const FwdJob &J, int x0, int y0, int z0, int x1,
                                             int y1, int z1)
{
    if (J.nx == 0 || J.ny == 0 || J.nz == 0)
        return kOutside;               // empty input: every sample is fill
    if (J.disp)
        return kBoundary;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        float r[3];
        row_base(J.M, (float)((c & 4) ? x1 : x0), (float)((c & 2) ? y1 : y0), r);
        float zf = (float)((c & 1) ? z1 : z0);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            float q = coord(J.M, i, r, zf);
            lo[i] = fminf(lo[i], q);
            hi[i] = fmaxf(hi[i], q);
        }
    }
    const float n[3] = {(float)J.nx, (float)J.ny, (float)J.nz};
    bool outside = false, interior = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        float l = lo[i] - J.delta[i], h = hi[i] + J.delta[i];
        outside = outside || (h <= -1.0f) || (l >= n[i]);
        interior = interior && (l >= 0.0f) && (h < n[i] - 1.0f);
    }
    return outside ? kOutside : (interior ? kInterior : kBoundary);
}

// Tile t of job J -> origin and last in-range voxel.
struct TileBox {
    int x0, y0, z0, x1, y1, z1;
};

__device__ __forceinline__ TileBox tile_box(const FwdJob &J, int t, const Tiling &TL)
{
    int tz = t % J.tiles_z;
    int rest = t / J.tiles_z;
    int ty = rest % J.tiles_y;
    int tx = rest / J.tiles_y;
    TileBox b;
    b.x0 = tx << TL.lx;
    b.y0 = ty << TL.ly;
    b.z0 = tz << TL.lz;
    b.x1 = min(b.x0 + (1 << TL.lx), J.ox) - 1;
    b.y1 = min(b.y0 + (1 << TL.ly), J.oy) - 1;
    b.z1 = min(b.z0 + (1 << TL.lz), J.oz) - 1;
    return b;
}

template <typename T, bool VEC>
__device__ __forceinline__ void fwd_tile(const FwdJob &J, int t, const Tiling &TL)
{
    const TileBox B = tile_box(J, t, TL);
    const int cls = classify_tile(J, B.x0, B.y0, B.z0, B.x1, B.y1, B.z1);
    const T *img = static_cast<const T *>(J.img);
    const bool labels = (J.flags & kFlagLabels) != 0;
    const Photo P = photo_of(J);
    const int32_t nvox = J.ox * J.oy * J.oz;
    const int runs_z_log = TL.lz - 2;
    const int nruns = 1 << (TL.lx + TL.ly + runs_z_log);

    for (int r = threadIdx.x; r < nruns; r += kThreads) {
        const int zr = r & ((1 << runs_z_log) - 1);
        const int rr = r >> runs_z_log;
        const int y = B.y0 + (rr & ((1 << TL.ly) - 1));
        const int x = B.x0 + (rr >> TL.ly);
        const int z = B.z0 + 4 * zr;
        if (x > B.x1 || y > B.y1 || z > B.z1)
            continue;
        const int nvalid = VEC ? 4 : min(4, J.oz - z);
        const int32_t v0 = (x * J.oy + y) * J.oz + z;
        float rb[3];
        row_base(J.M, (float)x, (float)y, rb);

        float V[4];
        int8_t L[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            V[k] = J.fill;
            L[k] = (int8_t)J.label_fill;
            if (!VEC && k >= nvalid)
                continue;
            const float zf = (float)(z + k);
            float qx = coord(J.M, 0, rb, zf), qy = coord(J.M, 1, rb, zf),
                  qz = coord(J.M, 2, rb, zf);
            if (J.disp) {
                qx = qx + J.disp[v0 + k];
                qy = qy + J.disp[nvox + v0 + k];
                qz = qz + J.disp[2 * nvox + v0 + k];
            }
            if (cls == kInterior) {
                V[k] = sample_interior(img, J.ny, J.nz, qx, qy, qz);
                if (labels)
                    L[k] = label_interior(J.lbl, J.ny, J.nz, qx, qy, qz);
            } else if (cls == kBoundary) {
                V[k] = sample_checked(img, J.nx, J.ny, J.nz, qx, qy, qz, J.fill);
                if (labels)
                    L[k] = label_checked(J.lbl, J.nx, J.ny, J.nz, qx, qy, qz,
                                         (int8_t)J.label_fill);
            }
        }

        if (P.flags & kFlagPhoto) {
            float n[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (P.flags & kFlagNoise)
                gauss_run((uint64_t)v0, J.vol_id, J.key0, J.key1, n);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                V[k] = photometric(P, V[k], n[k]);
        }

        if (VEC) {
            *reinterpret_cast<float4 *>(J.out + v0) = make_float4(V[0], V[1], V[2], V[3]);
            if (labels) {
                uint32_t packed = (uint32_t)(uint8_t)L[0] | ((uint32_t)(uint8_t)L[1] << 8) |
                                  ((uint32_t)(uint8_t)L[2] << 16) | ((uint32_t)(uint8_t)L[3] << 24);
                *reinterpret_cast<uint32_t *>(J.lout + v0) = packed;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k < nvalid) {
                    J.out[v0 + k] = V[k];
                    if (labels)
                        J.lout[v0 + k] = L[k];
                }
        }
    }
}

template <typename T>
__device__ __forceinline__ void fwd_tile_dispatch(const FwdJob &J, int t, const Tiling &TL)
{
    if (J.flags & kFlagVec)
        fwd_tile<T, true>(J, t, TL);
    else
        fwd_tile<T, false>(J, t, TL);
}

// Single job, job in kernel arguments, one workgroup per tile.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_warp_single(FwdJob J, Tiling TL, int32_t ntiles)
{
    const int b = blockIdx.x;
    const int per = (ntiles + 7) >> 3;
    const int t = (b & 7) * per + (b >> 3);
    if (t >= ntiles)
        return;
    fwd_tile_dispatch<T>(J, t, TL);
}

// Batch of jobs from a device table.  prefix[j] = first global tile of job j,
// prefix[njobs] = total.  Workgroups stride over the tiles of their XCD's
// contiguous range (persistent when gridDim.x is a few per CU).
__global__ __launch_bounds__(kThreads) void k_warp_batch(const FwdJob *__restrict__ jobs,
                                                         const int32_t *__restrict__ prefix,
                                                         int32_t njobs, Tiling TL)
{
    const int total = prefix[njobs];
    const int b = blockIdx.x;
    const int per_xcd_wg = gridDim.x >> 3;
    const int xcd = b & 7;
    const int per = (total + 7) >> 3;
    const int start = xcd * per;
    const int end = min(start + per, total);
    int j = 0;
    for (int t = start + (b >> 3); t < end; t += per_xcd_wg) {
        while (j + 1 < njobs && prefix[j + 1] <= t)
            ++j;
        const FwdJob J = jobs[j];
        const int lt = t - prefix[j];
        if (J.dtype == kI16)
            fwd_tile_dispatch<int16_t>(J, lt, TL);
        else
            fwd_tile_dispatch<float>(J, lt, TL);
    }
}

hipError_t launch_warp_single(const FwdJob &J, const Tiling &TL, hipStream_t s)
{
    const int ntiles = J.tiles_x * J.tiles_y * J.tiles_z;
    if (ntiles == 0)
        return hipSuccess;
    const int grid = ((ntiles + 7) >> 3) << 3;
    if (J.dtype == kI16)
        hipLaunchKernelGGL(k_warp_single<int16_t>, dim3(grid), dim3(kThreads), 0, s, J, TL, ntiles);
    else
        hipLaunchKernelGGL(k_warp_single<float>, dim3(grid), dim3(kThreads), 0, s, J, TL, ntiles);
    return hipGetLastError();
}

hipError_t launch_warp_batch(const FwdJob *jobs_dev, const int32_t *prefix_dev, int32_t njobs,
                             int32_t total_tiles, int32_t grid, const Tiling &TL, hipStream_t s)
{
    if (total_tiles == 0 || njobs == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_warp_batch, dim3(grid), dim3(kThreads), 0, s, jobs_dev, prefix_dev, njobs,
                       TL);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Standalone photometric pass (in place) and raw noise generator.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_photometric(float *data, int64_t n, Photo P,
                                                          uint32_t vol, uint32_t k0, uint32_t k1,
                                                          int vec)
{
    const int64_t ngroups = (n + 3) >> 2;
    for (int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x; g < ngroups;
         g += (int64_t)gridDim.x * kThreads) {
        const int64_t v0 = g << 2;
        float nz[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (P.flags & kFlagNoise)
            gauss_group((uint64_t)g, vol, k0, k1, nz);
        if (vec) {
            float4 x = *reinterpret_cast<float4 *>(data + v0);
            x.x = photometric(P, x.x, nz[0]);
            x.y = photometric(P, x.y, nz[1]);
            x.z = photometric(P, x.z, nz[2]);
            x.w = photometric(P, x.w, nz[3]);
            *reinterpret_cast<float4 *>(data + v0) = x;
        } else {
            for (int k = 0; k < 4; ++k)
                if (v0 + k < n)
                    data[v0 + k] = photometric(P, data[v0 + k], nz[k]);
        }
    }
}

hipError_t launch_photometric(float *data, int64_t n, const Photo &P, uint32_t vol, uint32_t k0,
                              uint32_t k1, bool vec, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const int64_t ngroups = (n + 3) >> 2;
    const int64_t blocks = std::min<int64_t>((ngroups + kThreads - 1) / kThreads, 256 * 64);
    hipLaunchKernelGGL(k_photometric, dim3((unsigned)blocks), dim3(kThreads), 0, s, data, n, P, vol,
                       k0, k1, vec ? 1 : 0);
    return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_noise(uint64_t v0, int64_t n, uint32_t vol,
                                                    uint32_t k0, uint32_t k1, float *gauss,
                                                    uint32_t *words)
{
    const uint64_t g0 = v0 >> 2;
    const uint64_t g1 = (v0 + (uint64_t)n - 1) >> 2;
    const int64_t ng = (int64_t)(g1 - g0) + 1;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < ng;
         i += (int64_t)gridDim.x * kThreads) {
        const uint64_t g = g0 + (uint64_t)i;
        uint32_t c[4] = {(uint32_t)g, (uint32_t)(g >> 32), vol, 0u};
        philox4x32_10(c, k0, k1);
        if (words) {
            words[4 * i + 0] = c[0];
            words[4 * i + 1] = c[1];
            words[4 * i + 2] = c[2];
            words[4 * i + 3] = c[3];
        }
        if (gauss) {
            float z[4];
            box_muller(c[0], c[1], z[0], z[1]);
            box_muller(c[2], c[3], z[2], z[3]);
            for (int k = 0; k < 4; ++k) {
                const uint64_t v = 4 * g + k;
                if (v >= v0 && v < v0 + (uint64_t)n)
                    gauss[v - v0] = z[k];
            }
        }
    }
}

hipError_t launch_noise(uint64_t v0, int64_t n, uint32_t vol, uint32_t k0, uint32_t k1,
                        float *gauss, uint32_t *words, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const int64_t ng = (int64_t)(((v0 + (uint64_t)n - 1) >> 2) - (v0 >> 2)) + 1;
    const int64_t blocks = std::min<int64_t>((ng + kThreads - 1) / kThreads, 256 * 64);
    hipLaunchKernelGGL(k_noise, dim3((unsigned)blocks), dim3(kThreads), 0, s, v0, n, vol, k0, k1,
                       gauss, words);
    return hipGetLastError();
}

}  // namespace ctaug
