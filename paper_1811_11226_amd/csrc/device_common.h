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

#include "bspline_eval.h"

namespace ctaug {

constexpr int kThreads = 256;          // workgroup size of every warp kernel
constexpr int kRun = 4;                // output voxels per thread along z
constexpr int kMaxLdsBytes = 61440;    // LDS footprint reservation per workgroup (60 KB)

// XCD-aware tile order.  Consecutive workgroup ids are dispatched round-robin
// over the 8 XCDs, so workgroup b runs on XCD b % 8.  Tiles are dealt to the
// XCDs in chunks of 2^kXcdChunkLog consecutive tiles, round-robin, and the
// workgroups of an XCD take its tiles in increasing order: each XCD (and its
// L2) gets spatially coherent runs of tiles from every part of the grid, so
// that jobs of uneven cost spread over all XCDs.  Slot i of XCD x holds tile
// xcd_tile(x, i); tiles increase with i, and xcd_slots(n) slots per XCD cover
// n tiles.
constexpr int kXcdChunkLog = 6;
__host__ __device__ __forceinline__ int xcd_tile(int xcd, int i)
{
    return ((((i >> kXcdChunkLog) << 3) + xcd) << kXcdChunkLog) + (i & ((1 << kXcdChunkLog) - 1));
}
__host__ __device__ __forceinline__ int xcd_slots(int n)
{
    return ((n + (8 << kXcdChunkLog) - 1) >> (kXcdChunkLog + 3)) << kXcdChunkLog;
}

// Slots of one persistent workgroup w of an XCD with W workgroups: in round k
// it takes slot k W + ((w + 77 k) mod W).  Each round is a permutation of its
// W slots and a workgroup's slots increase, as with slots w, w + W, ...; the
// shift keeps a workgroup from meeting the same place of every chunk (the
// same y-z position of every x slab), whose tiles cost alike.
struct XcdSlots {
    int W, skew, pos, base;
    __device__ __forceinline__ XcdSlots(int w, int nw) : W(nw), skew(77 % nw), pos(w), base(0) {}
    __device__ __forceinline__ int slot() const { return base + pos; }
    __device__ __forceinline__ void next()
    {
        base += W;
        pos += skew;
        if (pos >= W)
            pos -= W;
    }
};

enum : uint32_t {
    kFlagWindow = 1u,                  // window + gamma
    kFlagPhoto = 2u,                   // photometric chain enabled
    kFlagLabels = 4u,                  // warp a label volume
    kFlagNoise = 8u,                   // sigma > 0
    kFlagGamma = 16u,                  // gamma != 1
    kFlagVec = 32u,                    // 16-byte aligned outputs, Zo % 4 == 0
    kFlagFillInT = 64u,                // fill is exactly representable as an int16
    kFlagLds16 = 128u,                 // int16 input staged as int16 LDS cells
    kFlagOcclude = 256u,               // output z-slab [occ_lo, occ_hi] set to 0
};

enum : int32_t { kF32 = 0, kI16 = 1, kI8 = 2 };

// Source of the per-voxel displacement of a warp: none (affine), a dense
// field, or the cubic B-spline of a control grid evaluated in the kernel.
enum : int { kDispNone = 0, kDispField = 1, kDispSpline = 2 };

// One forward warp job as the kernels see it.  Built on the host from the
// public arguments; lives in kernel arguments (single calls) or in a device
// table (batched calls).
struct FwdJob {
    const void *img;                   // F32 or I16 [nx][ny][nz]
    const int8_t *lbl;                 // I8 [nx][ny][nz] or null
    float *out;                        // F32 [ox][oy][oz]
    int8_t *lout;                      // I8 [ox][oy][oz] or null
    const float *disp;                 // F32 SoA [3][ox][oy][oz] or null
    const float *ctrl;                 // F32 control grid [3][gx][gy][gz] or null; the
                                       // displacement is evaluated from it in the kernel
    BsplineGeom bs;                    // geometry of ctrl over the output
    int32_t dtype;
    int32_t nx, ny, nz;
    int32_t in_ry, in_sy;              // input layout: rows per x plane, elements per y row
    int32_t in_extent;                 // elements from the first to past the last input voxel
    int32_t ox, oy, oz;
    uint32_t flags;
    float M[12];                       // [A|b] row-major
    float delta[3];                    // bound on FP32 rounding of q per axis
    float fill;
    int32_t label_fill;
    float gain, offset, sigma, win_lo, inv_range, gamma;
    float occ_lo, occ_hi;              // occluded output slab occ_lo <= z <= occ_hi
    uint32_t vol_id, key0, key1;
    int32_t tiles_x, tiles_y, tiles_z; // tile grid of this job's output
    int32_t sub[3];                    // log2 extents of the sub-tiles a tile is staged in
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
// Global-memory pointer types.  Pointers read from a job table are generic to
// the compiler; casting them to the global address space gives global_load /
// global_store with an SGPR base and a 32-bit VGPR offset instead of flat
// accesses.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <typename T> using gconst = __attribute__((address_space(1))) const T;
template <typename T> using gmut = __attribute__((address_space(1))) T;

template <typename T> __device__ __forceinline__ gconst<T> *gc(const void *p)
{
    return (gconst<T> *)p;
}
template <typename T> __device__ __forceinline__ gmut<T> *gm(void *p) { return (gmut<T> *)p; }

// ---------------------------------------------------------------------------
// Buffer resources.  Input gathers use raw buffer loads: an SGPR descriptor
// with the base and byte size, a 32-bit VGPR byte offset, an optional SGPR
// offset and a 12-bit immediate.  Every load is kept inside the volume (the
// compiler may merge loads at adjacent offsets into one wider load, whose
// range check would then also cover the in-range neighbour), so corners that
// will be replaced by the fill value are loaded from clamped indices.
// ---------------------------------------------------------------------------
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kRawBufferFlags = 0x00020000;   // raw (unformatted) dword buffer, gfx9 encoding

__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             kRawBufferFlags);
}

template <typename T> struct Elem;
template <> struct Elem<float> {
    static __device__ __forceinline__ float raw(rsrc_t r, uint32_t off, int32_t soff)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
    }
    static __device__ __forceinline__ float load(rsrc_t r, uint32_t off, int32_t soff)
    {
        return raw(r, off, soff);
    }
};
template <> struct Elem<int16_t> {
    static __device__ __forceinline__ int16_t raw(rsrc_t r, uint32_t off, int32_t soff)
    {
        return (int16_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0);
    }
    static __device__ __forceinline__ float load(rsrc_t r, uint32_t off, int32_t soff)
    {
        return (float)raw(r, off, soff);
    }
};

__device__ __forceinline__ int8_t load_i8(rsrc_t r, uint32_t off)
{
    return (int8_t)__builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0);
}

// 24-bit multiply (full rate); operands and product must stay below 2^24 / 2^32.
__device__ __forceinline__ uint32_t mul24(uint32_t a, uint32_t b) { return __umul24(a, b); }

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

// Input volume geometry for gathers: dims, layout (ry rows per x plane, sy
// elements per y row, z contiguous), byte strides between x / y neighbours,
// and the buffer resources of image and labels (which share the layout).
struct Src {
    rsrc_t img, lbl;
    int32_t nx, ny, nz;
    int32_t ry, rsy;                   // rows per x plane, elements per y row
    int32_t sy, sx, sxy;               // byte offsets of the +y, +x, +x+y corner rows
};

template <typename T> __device__ __forceinline__ Src make_src(const FwdJob &J)
{
    Src S;
    const uint32_t n = (uint32_t)J.in_extent;
    S.img = make_rsrc(J.img, n * (uint32_t)sizeof(T));
    S.lbl = make_rsrc(J.lbl, J.lbl ? n : 0u);
    S.nx = J.nx;
    S.ny = J.ny;
    S.nz = J.nz;
    S.ry = J.in_ry;
    S.rsy = J.in_sy;
    S.sy = J.in_sy * (int32_t)sizeof(T);
    S.sx = J.in_ry * J.in_sy * (int32_t)sizeof(T);
    S.sxy = S.sx + S.sy;
    return S;
}

// Element offset of input voxel (ix, iy, iz) inside the volume: (ix ry + iy)
// sy + iz with 24-bit multiplies (the host admits only layouts whose row
// count and row pitch stay below 2^24).
__device__ __forceinline__ uint32_t elem_index(const Src &S, int32_t ix, int32_t iy, int32_t iz)
{
    return mul24(mul24((uint32_t)ix, (uint32_t)S.ry) + (uint32_t)iy, (uint32_t)S.rsy) + (uint32_t)iz;
}

// Sample whose cell [i0, i0+1]^3 is known to lie inside the volume: one VGPR
// offset, the other corner rows through SGPR offsets and the immediate.
template <typename T>
__device__ __forceinline__ float sample_interior(const Src &S, float qx, float qy, float qz)
{
    const float fx = floorf(qx), fy = floorf(qy), fz = floorf(qz);
    const uint32_t off = elem_index(S, (int32_t)fx, (int32_t)fy, (int32_t)fz) * (uint32_t)sizeof(T);
    constexpr uint32_t e = sizeof(T);
    float k[8];
    k[0] = Elem<T>::load(S.img, off, 0);
    k[1] = Elem<T>::load(S.img, off + e, 0);
    k[2] = Elem<T>::load(S.img, off, S.sy);
    k[3] = Elem<T>::load(S.img, off + e, S.sy);
    k[4] = Elem<T>::load(S.img, off, S.sx);
    k[5] = Elem<T>::load(S.img, off + e, S.sx);
    k[6] = Elem<T>::load(S.img, off, S.sxy);
    k[7] = Elem<T>::load(S.img, off + e, S.sxy);
    return tri(k, qx - fx, qy - fy, qz - fz);
}

__device__ __forceinline__ bool in_guard(float qx, float qy, float qz, int32_t nx, int32_t ny,
                                         int32_t nz)
{
    return qx > -1.0f && qx < (float)nx && qy > -1.0f && qy < (float)ny && qz > -1.0f &&
           qz < (float)nz;
}

// Corners of the cell floor(q) with `fill` for every corner outside the
// volume.  Requires in_guard(q).  Out-of-volume corners are loaded from the
// clamped index and then replaced by fill.
template <typename T>
__device__ __forceinline__ void corners_checked(const Src &S, float qx, float qy, float qz,
                                                float fill, float k[8], float t[3],
                                                int32_t i0[3])
{
    const float fx = floorf(qx), fy = floorf(qy), fz = floorf(qz);
    t[0] = qx - fx;
    t[1] = qy - fy;
    t[2] = qz - fz;
    const int32_t ix = (int32_t)fx, iy = (int32_t)fy, iz = (int32_t)fz;
    i0[0] = ix;
    i0[1] = iy;
    i0[2] = iz;
    const bool vx[2] = {ix >= 0, ix + 1 < S.nx};
    const bool vy[2] = {iy >= 0, iy + 1 < S.ny};
    const bool vz[2] = {iz >= 0, iz + 1 < S.nz};
    const int32_t cx[2] = {max(ix, 0), min(ix + 1, S.nx - 1)};
    const int32_t cy[2] = {max(iy, 0), min(iy + 1, S.ny - 1)};
    const int32_t cz[2] = {max(iz, 0), min(iz + 1, S.nz - 1)};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const uint32_t off = elem_index(S, cx[a], cy[b], cz[c]) * (uint32_t)sizeof(T);
                const float v = Elem<T>::load(S.img, off, 0);
                k[4 * a + 2 * b + c] = (vx[a] && vy[b] && vz[c]) ? v : fill;
            }
}

template <typename T>
__device__ __forceinline__ float sample_checked(const Src &S, float qx, float qy, float qz,
                                                float fill)
{
    if (!in_guard(qx, qy, qz, S.nx, S.ny, S.nz))
        return fill;
    float k[8], t[3];
    int32_t i0[3];
    corners_checked<T>(S, qx, qy, qz, fill, k, t, i0);
    return tri(k, t[0], t[1], t[2]);
}

// Nearest label: j = floorf(q + 0.5f) per axis (FP32, ties up).
__device__ __forceinline__ int32_t nn_index(float q) { return (int32_t)floorf(q + 0.5f); }

__device__ __forceinline__ int8_t label_checked(const Src &S, float qx, float qy, float qz,
                                                int8_t label_fill)
{
    if (!in_guard(qx, qy, qz, S.nx, S.ny, S.nz))
        return label_fill;
    const int32_t jx = nn_index(qx), jy = nn_index(qy), jz = nn_index(qz);
    const bool ok = jx >= 0 && jx < S.nx && jy >= 0 && jy < S.ny && jz >= 0 && jz < S.nz;
    const int8_t l = load_i8(S.lbl, elem_index(S, min(max(jx, 0), S.nx - 1),
                                               min(max(jy, 0), S.ny - 1),
                                               min(max(jz, 0), S.nz - 1)));
    return ok ? l : label_fill;
}

__device__ __forceinline__ int8_t label_interior(const Src &S, float qx, float qy, float qz)
{
    return load_i8(S.lbl, elem_index(S, nn_index(qx), nn_index(qy), nn_index(qz)));
}

// ---------------------------------------------------------------------------
// Noise: Philox4x32-10 (Salmon et al., SC'11) at counter (lo, hi, vol, 0)
// with key (k0, k1); uniforms ((w >> 9) + 0.5) 2^-23; Box-Muller pairs
// (w0, w1) and (w2, w3).
// ---------------------------------------------------------------------------
// a ^ b ^ c in one VALU instruction (the compiler emits two when one operand
// is uniform).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t n0 = xor3((uint32_t)(p1 >> 32), c[1], k0);
        uint32_t n2 = xor3((uint32_t)(p0 >> 32), c[3], k1);
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        // bump the key in SALU each round rather than keeping all ten round
        // keys live in scalar registers across the caller's loops
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
        asm volatile("" : "+s"(k0), "+s"(k1));
    }
}

__device__ __forceinline__ float uniform01(uint32_t w)
{
    return ((float)(w >> 9) + 0.5f) * 0x1p-23f;
}

// (r cos theta, r sin theta) with r = sqrt(-2 ln U(wr)), theta = 2 pi U(wt),
// on the hardware transcendental units: v_log_f32 (log2), v_sqrt_f32, and
// v_sin_f32 / v_cos_f32, which take their argument in revolutions, so the
// angle is U itself with no rounding of 2 pi.  Measured over all 2^23
// uniforms on gfx950: |dr|/r <= 1.35e-7 and |d sin|, |d cos| <= 1.25e-7, which
// bounds the error of each normal by 1.35e-7 |n| + 5.77 * 1.25e-7 + rounding
// < 1e-6 max(1, |n|).
__device__ __forceinline__ void box_muller(uint32_t wr, uint32_t wt, float &c, float &s)
{
    const float r2 = -1.38629436111989061883f * __builtin_amdgcn_logf(uniform01(wr));  // -2 ln U
    const float r = __builtin_amdgcn_sqrtf(r2);
    const float t = uniform01(wt);
    c = r * __builtin_amdgcn_cosf(t);
    s = r * __builtin_amdgcn_sinf(t);
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

// Standard normals of voxels v0 .. v0+3 when v0 is not a multiple of 4 (the
// run straddles two noise groups): only volumes whose z extent is not a
// multiple of 4.
__device__ __forceinline__ void gauss_run_split(uint64_t v0, uint32_t vol, uint32_t k0,
                                                uint32_t k1, float n[4])
{
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

// Standard normals of voxels v0 .. v0+3 (any alignment).
__device__ __forceinline__ void gauss_run(uint64_t v0, uint32_t vol, uint32_t k0, uint32_t k1,
                                          float n[4])
{
    if ((v0 & 3u) == 0)
        gauss_group(v0 >> 2, vol, k0, k1, n);
    else
        gauss_run_split(v0, vol, k0, k1, n);
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
