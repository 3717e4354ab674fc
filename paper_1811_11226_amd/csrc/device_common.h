// device_common.h -- device-side building blocks shared by the gfx950 kernels:
// job descriptors, the pinned coordinate map, trilinear / nearest sampling,
// the Philox4x32-10 + Box-Muller noise generator and the photometric chain.
//
// Everything here is compiled with -ffp-contract=off: every fused multiply-add
// is written out explicitly, so the same inputs give the same bits in every
// kernel that uses these functions (fused and unfused photometrics agree).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ctaug {

constexpr int kThreads = 256;          // workgroup size of every warp kernel
constexpr int kRun = 4;                // output voxels per thread along z

enum : uint32_t {
    kFlagWindow = 1u,                  // window + gamma
    kFlagPhoto = 2u,                   // photometric chain enabled
    kFlagLabels = 4u,                  // warp a label volume
    kFlagNoise = 8u,                   // sigma > 0
    kFlagGamma = 16u,                  // gamma != 1
    kFlagVec = 32u,                    // 16-byte aligned outputs, Zo % 4 == 0
};

enum : int32_t { kF32 = 0, kI16 = 1, kI8 = 2 };

// One forward warp job as the kernels see it.  Built on the host from the
// public arguments; lives in kernel arguments (single calls) or in a device
// table (batched calls).
struct FwdJob {
    const void *img;                   // F32 or I16 [nx][ny][nz]
    const int8_t *lbl;                 // I8 [nx][ny][nz] or null
    float *out;                        // F32 [ox][oy][oz]
    int8_t *lout;                      // I8 [ox][oy][oz] or null
    const float *disp;                 // F32 SoA [3][ox][oy][oz] or null
    int32_t dtype;
    int32_t nx, ny, nz;
    int32_t ox, oy, oz;
    uint32_t flags;
    float M[12];                       // [A|b] row-major
    float delta[3];                    // bound on FP32 rounding of q per axis
    float fill;
    int32_t label_fill;
    float gain, offset, sigma, win_lo, inv_range, gamma;
    uint32_t vol_id, key0, key1;
    int32_t tiles_x, tiles_y, tiles_z; // tile grid of this job's output
};

// Launch shape: tile extents as log2 (voxels), z extent >= 4.
struct Tiling {
    int32_t lx, ly, lz;
};

// ---------------------------------------------------------------------------
// Coordinate map: q_i = fmaf(A_i2, z, fmaf(A_i1, y, fmaf(A_i0, x, b_i))).
// The row part r_i = fmaf(A_i1, y, fmaf(A_i0, x, b_i)) is shared by a z-run.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void row_base(const float *M, float xf, float yf, float r[3])
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
        r[i] = __builtin_fmaf(M[4 * i + 1], yf, __builtin_fmaf(M[4 * i + 0], xf, M[4 * i + 3]));
}

__device__ __forceinline__ float coord(const float *M, int i, const float r[3], float zf)
{
    return __builtin_fmaf(M[4 * i + 2], zf, r[i]);
}

// ---------------------------------------------------------------------------
// Input element loads
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ float ld(const T *p, int32_t i);
template <> __device__ __forceinline__ float ld<float>(const float *p, int32_t i) { return p[i]; }
template <> __device__ __forceinline__ float ld<int16_t>(const int16_t *p, int32_t i)
{
    return (float)p[i];
}

__device__ __forceinline__ float lerp(float a, float b, float t)
{
    return __builtin_fmaf(t, b - a, a);
}

// Trilinear value from the eight corners k[a][b][c] (a: x, b: y, c: z).
__device__ __forceinline__ float tri(const float k[8], float tx, float ty, float tz)
{
    float e00 = lerp(k[0], k[1], tz), e01 = lerp(k[2], k[3], tz);
    float e10 = lerp(k[4], k[5], tz), e11 = lerp(k[6], k[7], tz);
    return lerp(lerp(e00, e01, ty), lerp(e10, e11, ty), tx);
}

// Sample whose cell [i0, i0+1]^3 is known to lie inside the volume.
template <typename T>
__device__ __forceinline__ float sample_interior(const T *img, int32_t ny, int32_t nz, float qx,
                                                 float qy, float qz)
{
    float fx = floorf(qx), fy = floorf(qy), fz = floorf(qz);
    float tx = qx - fx, ty = qy - fy, tz = qz - fz;
    int32_t base = ((int32_t)fx * ny + (int32_t)fy) * nz + (int32_t)fz;
    int32_t sy = nz, sx = ny * nz;
    float k[8];
    k[0] = ld(img, base);
    k[1] = ld(img, base + 1);
    k[2] = ld(img, base + sy);
    k[3] = ld(img, base + sy + 1);
    k[4] = ld(img, base + sx);
    k[5] = ld(img, base + sx + 1);
    k[6] = ld(img, base + sx + sy);
    k[7] = ld(img, base + sx + sy + 1);
    return tri(k, tx, ty, tz);
}

__device__ __forceinline__ bool in_guard(float qx, float qy, float qz, int32_t nx, int32_t ny,
                                         int32_t nz)
{
    return qx > -1.0f && qx < (float)nx && qy > -1.0f && qy < (float)ny && qz > -1.0f &&
           qz < (float)nz;
}

// Corners of the cell floor(q) with `fill` for every corner outside the
// volume.  Requires in_guard(q).  Addresses are clamped so every load is in
// bounds; the clamped value is then replaced by fill.
template <typename T>
__device__ __forceinline__ void corners_checked(const T *img, int32_t nx, int32_t ny, int32_t nz,
                                                float qx, float qy, float qz, float fill,
                                                float k[8], float t[3], int32_t i0[3])
{
    float fx = floorf(qx), fy = floorf(qy), fz = floorf(qz);
    t[0] = qx - fx;
    t[1] = qy - fy;
    t[2] = qz - fz;
    int32_t ix = (int32_t)fx, iy = (int32_t)fy, iz = (int32_t)fz;
    i0[0] = ix;
    i0[1] = iy;
    i0[2] = iz;
    bool vx[2] = {ix >= 0, ix + 1 < nx};
    bool vy[2] = {iy >= 0, iy + 1 < ny};
    bool vz[2] = {iz >= 0, iz + 1 < nz};
    int32_t cx[2] = {max(ix, 0), min(ix + 1, nx - 1)};
    int32_t cy[2] = {max(iy, 0), min(iy + 1, ny - 1)};
    int32_t cz[2] = {max(iz, 0), min(iz + 1, nz - 1)};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                float v = ld(img, (cx[a] * ny + cy[b]) * nz + cz[c]);
                k[4 * a + 2 * b + c] = (vx[a] && vy[b] && vz[c]) ? v : fill;
            }
}

template <typename T>
__device__ __forceinline__ float sample_checked(const T *img, int32_t nx, int32_t ny, int32_t nz,
                                                float qx, float qy, float qz, float fill)
{
    if (!in_guard(qx, qy, qz, nx, ny, nz))
        return fill;
    float k[8], t[3];
    int32_t i0[3];
    corners_checked(img, nx, ny, nz, qx, qy, qz, fill, k, t, i0);
    return tri(k, t[0], t[1], t[2]);
}

// Nearest label: j = floorf(q + 0.5f) per axis (FP32, ties up).
__device__ __forceinline__ int32_t nn_index(float q) { return (int32_t)floorf(q + 0.5f); }

__device__ __forceinline__ int8_t label_checked(const int8_t *lbl, int32_t nx, int32_t ny,
                                                int32_t nz, float qx, float qy, float qz,
                                                int8_t label_fill)
{
    if (!in_guard(qx, qy, qz, nx, ny, nz))
        return label_fill;
    int32_t jx = nn_index(qx), jy = nn_index(qy), jz = nn_index(qz);
    bool ok = jx >= 0 && jx < nx && jy >= 0 && jy < ny && jz >= 0 && jz < nz;
    int32_t idx = (min(max(jx, 0), nx - 1) * ny + min(max(jy, 0), ny - 1)) * nz +
                  min(max(jz, 0), nz - 1);
    int8_t l = lbl[idx];
    return ok ? l : label_fill;
}

__device__ __forceinline__ int8_t label_interior(const int8_t *lbl, int32_t ny, int32_t nz,
                                                 float qx, float qy, float qz)
{
    return lbl[(nn_index(qx) * ny + nn_index(qy)) * nz + nn_index(qz)];
}

// ---------------------------------------------------------------------------
// Noise: Philox4x32-10 (Salmon et al., SC'11) at counter (lo, hi, vol, 0)
// with key (k0, k1); uniforms ((w >> 9) + 0.5) 2^-23; Box-Muller pairs
// (w0, w1) and (w2, w3).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ float uniform01(uint32_t w)
{
    return ((float)(w >> 9) + 0.5f) * 0x1p-23f;
}

// (r cos theta, r sin theta) with r = sqrt(-2 ln U(wr)), theta = 2 pi U(wt).
// sincospi takes 2U exactly, so the angle carries no rounding of 2 pi.
__device__ __forceinline__ void box_muller(uint32_t wr, uint32_t wt, float &c, float &s)
{
    float r = sqrtf(-2.0f * logf(uniform01(wr)));
    float sn, cs;
    sincospif(2.0f * uniform01(wt), &sn, &cs);
    c = r * cs;
    s = r * sn;
}

// Standard normals of the four voxels of noise group g.
__device__ __forceinline__ void gauss_group(uint64_t g, uint32_t vol, uint32_t k0, uint32_t k1,
                                            float n[4])
{
    uint32_t c[4] = {(uint32_t)g, (uint32_t)(g >> 32), vol, 0u};
    philox4x32_10(c, k0, k1);
    box_muller(c[0], c[1], n[0], n[1]);
    box_muller(c[2], c[3], n[2], n[3]);
}

// Standard normals of voxels v0 .. v0+3 (any alignment).
__device__ __forceinline__ void gauss_run(uint64_t v0, uint32_t vol, uint32_t k0, uint32_t k1,
                                          float n[4])
{
    if ((v0 & 3u) == 0) {
        gauss_group(v0 >> 2, vol, k0, k1, n);
        return;
    }
    float a[4], b[4];
    gauss_group(v0 >> 2, vol, k0, k1, a);
    gauss_group((v0 >> 2) + 1, vol, k0, k1, b);
    uint32_t s = (uint32_t)(v0 & 3u);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t j = s + k;            // position within the two groups
        float va = j == 0 ? a[0] : j == 1 ? a[1] : j == 2 ? a[2] : a[3];
        float vb = j == 4 ? b[0] : j == 5 ? b[1] : j == 6 ? b[2] : b[3];
        n[k] = j < 4 ? va : vb;
    }
}

// ---------------------------------------------------------------------------
// Photometric chain on one value (noise n already drawn).
// ---------------------------------------------------------------------------
struct Photo {
    uint32_t flags;
    float gain, offset, sigma, win_lo, inv_range, gamma;
};

__device__ __forceinline__ float photometric(const Photo &P, float V, float n)
{
    float v = __builtin_fmaf(P.gain, V, P.offset);
    if (P.flags & kFlagNoise)
        v = __builtin_fmaf(P.sigma, n, v);
    if (P.flags & kFlagWindow) {
        float t = (v - P.win_lo) * P.inv_range;
        t = fminf(fmaxf(t, 0.0f), 1.0f);
        if (P.flags & kFlagGamma)
            t = t > 0.0f ? __builtin_amdgcn_exp2f(P.gamma * __builtin_amdgcn_logf(t)) : 0.0f;
        v = t;
    }
    return v;
}

__device__ __forceinline__ Photo photo_of(const FwdJob &J)
{
    Photo P;
    P.flags = J.flags;
    P.gain = J.gain;
    P.offset = J.offset;
    P.sigma = J.sigma;
    P.win_lo = J.win_lo;
    P.inv_range = J.inv_range;
    P.gamma = J.gamma;
    return P;
}

}  // namespace ctaug
