// tile_geom.h -- geometry of an output box's input footprint and its staging
// into LDS (internal; shared by the forward and adjoint kernels).
//
// The coordinate is affine in the output voxel, so over a box its extremes
// per axis are the value at the box origin plus the negative / positive parts
// of A_ij * span_j, widened by a bound on FP32 rounding.  From them: whether
// every sample of the box fails the guard (outside), whether every trilinear
// cell lies inside the volume (interior), and the AABB of input cells
// floor(q) .. floor(q) + 1 of every guarded sample, clamped to [-1, n].
#pragma once

#include "device_common.h"

namespace ctaug {

enum : int { kOutside = 0, kInterior = 1, kBoundary = 2 };

// LDS row pitch for rows of e cells: whole quads of 4 cells, and an odd
// number of quads so that neighbouring rows start in different LDS banks
// (rows a multiple of 8 cells apart would all fall on the same banks).
__device__ __host__ __forceinline__ int lds_pitch(int e)
{
    const int p = (e + 3) & ~3;
    return (p & 4) ? p : p + 4;
}

// Geometry of one output tile, uniform over the workgroup.
struct TileGeom {
    int x0, y0, z0, x1, y1, z1;        // output voxels covered (inclusive)
    int cls;                           // kOutside / kInterior / kBoundary
    int lo[3], e[3];                   // input cells [lo, lo + e) the tile can touch
    int quads;                         // 4-cell quads staged per row: ceil(e[2] / 4)
    int pitch;                         // LDS row pitch: 4 * quads, padded to 4 mod 8 cells
    bool lds;                          // footprint staged in LDS
};

// Geometry of the output box [x0, x1] x [y0, y1] x [z0, z1] (inclusive).
__device__ __forceinline__ TileGeom box_geom(const FwdJob &J, int x0, int y0, int z0, int x1,
                                             int y1, int z1, int32_t lds_cells)
{
    TileGeom G;
    G.x0 = x0;
    G.y0 = y0;
    G.z0 = z0;
    G.x1 = x1;
    G.y1 = y1;
    G.z1 = z1;
    G.lds = false;
    G.quads = 0;
    G.pitch = 0;
    if (J.nx == 0 || J.ny == 0 || J.nz == 0) {
        G.cls = kOutside;              // empty input: every sample is fill
        return G;
    }
    if (J.disp) {
        G.cls = kBoundary;             // displacement: per-sample checks, direct gathers
        return G;
    }
    // The coordinate is affine in p: its extremes over the box are the value at
    // the origin plus the negative / positive parts of A_ij * span_j.  The
    // margin delta covers FP32 rounding of both this bound and of q itself.
    const float span[3] = {(float)(G.x1 - G.x0), (float)(G.y1 - G.y0), (float)(G.z1 - G.z0)};
    float rb[3];
    row_base(J.M, (float)G.x0, (float)G.y0, rb);
    const int n[3] = {J.nx, J.ny, J.nz};
    bool outside = false, interior = true;
    int cells = 1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float q0 = coord(J.M, i, rb, (float)G.z0);
        float dn = 0.0f, up = 0.0f;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const float d = J.M[4 * i + j] * span[j];
            dn += fminf(d, 0.0f);
            up += fmaxf(d, 0.0f);
        }
        const float l = q0 + dn - J.delta[i], h = q0 + up + J.delta[i];
        outside = outside || (h <= -1.0f) || (l >= (float)n[i]);
        interior = interior && (l >= 0.0f) && (h < (float)(n[i] - 1));
        // cells floor(q) .. floor(q) + 1 of every guarded sample, clamped to [-1, n]
        const int a = (int)fmaxf(floorf(l), -1.0f);
        const int b = min((int)fminf(floorf(h), (float)n[i]) + 1, n[i]);
        G.lo[i] = a;
        G.e[i] = max(b - a + 1, 1);
    }
    G.quads = (G.e[2] + 3) >> 2;
    G.pitch = lds_pitch(G.e[2]);
    cells = G.e[0] * G.e[1] * G.pitch;
    G.cls = outside ? kOutside : (interior ? kInterior : kBoundary);
    // an int16 footprint must hold fill exactly
    G.lds = !outside && cells <= lds_cells && (!(J.flags & kFlagLds16) || (J.flags & kFlagFillInT));
    return G;
}

// Footprint rows are quads of 4 cells.  When one x-slab of the footprint
// (ey rows of quads_per_row quads) fits the workgroup, each lane keeps one
// fixed (y row, quad) for the whole tile and walks the x-slabs: the row
// bookkeeping is two additions per quad.  Larger slabs use a generic loop.
__device__ __forceinline__ void store4(float *dst, const float v[4])
{
    *reinterpret_cast<f32x4 *>(dst) = f32x4{v[0], v[1], v[2], v[3]};
}

__device__ __forceinline__ void store4(int16_t *dst, const int16_t v[4])
{
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    *reinterpret_cast<u32x2 *>(dst) =
        u32x2{(uint32_t)(uint16_t)v[0] | ((uint32_t)(uint16_t)v[1] << 16),
              (uint32_t)(uint16_t)v[2] | ((uint32_t)(uint16_t)v[3] << 16)};
}

// Four consecutive input cells at byte offset `off` copied into LDS cells of
// type LT with one buffer load (16 bytes of FP32 or 8 bytes of int16; the
// offset need only be element-aligned).
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void copy_quad(rsrc_t r, uint32_t off, float *dst, float)
{
    *reinterpret_cast<u32x4 *>(dst) = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
}

__device__ __forceinline__ void copy_quad(rsrc_t r, uint32_t off, int16_t *dst, int16_t)
{
    *reinterpret_cast<u32x2 *>(dst) = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
}

__device__ __forceinline__ void copy_quad(rsrc_t r, uint32_t off, float *dst, int16_t)
{
    const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    *reinterpret_cast<f32x4 *>(dst) =
        f32x4{(float)(int16_t)(w.x & 0xffffu), (float)((int32_t)w.x >> 16),
              (float)(int16_t)(w.y & 0xffffu), (float)((int32_t)w.y >> 16)};
}

template <typename T, typename LT, bool INSIDE, bool LBL>
__device__ __forceinline__ void stage_quad(const FwdJob &J, const Src &S, const TileGeom &G,
                                           int gx, int gy, int cz0, uint32_t grow_inside,
                                           LT *dst, int8_t *ldst)
{
    constexpr uint32_t es = sizeof(T);
    if (INSIDE) {
        // every cell of the quad lies in the volume: one load per array
        const uint32_t e = grow_inside + (uint32_t)cz0;
        copy_quad(S.img, e * es, dst + cz0, T());
        if (LBL)
            *reinterpret_cast<uint32_t *>(ldst + cz0) =
                __builtin_amdgcn_raw_buffer_load_b32(S.lbl, e, 0, 0);
        return;
    }
    const int8_t lfill = (int8_t)J.label_fill;
    const bool row_in = (unsigned)gx < (unsigned)J.nx && (unsigned)gy < (unsigned)J.ny;
    const uint32_t grow = elem_index(S, min(max(gx, 0), J.nx - 1), min(max(gy, 0), J.ny - 1), 0);
    const LT tfill = (LT)J.fill;
    LT v[4];
    uint32_t lp = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        // indices clamped into the volume: every load stays in range
        const int gz = G.lo[2] + cz0 + u;
        const uint32_t e = grow + (uint32_t)min(max(gz, 0), J.nz - 1);
        const T raw = Elem<T>::raw(S.img, e * es, 0);
        const int8_t lab = LBL ? load_i8(S.lbl, e) : lfill;
        const bool in = row_in && (unsigned)gz < (unsigned)J.nz;
        v[u] = in ? (LT)raw : tfill;
        if (LBL)
            lp |= (uint32_t)(uint8_t)(in ? lab : lfill) << (8 * u);
    }
    store4(dst + cz0, v);
    if (LBL)
        *reinterpret_cast<uint32_t *>(ldst + cz0) = lp;
}

template <typename T, typename LT, bool INSIDE, bool LBL>
__device__ __forceinline__ void stage_rows(const FwdJob &J, const Src &S, const TileGeom &G,
                                           LT *s_img, int8_t *s_lbl)
{
    const int ex = G.e[0], ey = G.e[1], P = G.pitch;
    const int qpr = G.quads;
    const int slab = ey * qpr;
    if (slab <= kThreads) {
        const int ng = kThreads / slab;                    // x-slabs per pass
        const int g = threadIdx.x / slab;
        const int s = threadIdx.x - g * slab;
        if (g >= ng)
            return;
        const int cy = s / qpr;
        const int cz0 = 4 * (s - cy * qpr);
        const int gy = G.lo[1] + cy;
        // element index of (lo_x + cx, gy, lo_z): advanced by ng x-planes per pass
        const uint32_t plane = mul24((uint32_t)S.ny, (uint32_t)S.nz);
        uint32_t grow = INSIDE ? elem_index(S, G.lo[0] + g, gy, G.lo[2]) : 0u;
        const uint32_t gstep = mul24((uint32_t)ng, plane);
        const int lstep = ng * ey * P;
        int loff = (g * ey + cy) * P;
#pragma unroll 4
        for (int cx = g; cx < ex; cx += ng) {
            stage_quad<T, LT, INSIDE, LBL>(J, S, G, G.lo[0] + cx, gy, cz0, grow, s_img + loff,
                                       s_lbl + loff);
            grow += gstep;
            loff += lstep;
        }
        return;
    }
    // generic: lanes x rows
    const int quads = qpr;
    const int lr_log = quads <= 4 ? 2 : quads <= 8 ? 3 : quads <= 16 ? 4 : quads <= 32 ? 5 : 6;
    const int LR = 1 << lr_log;
    const int rpi = kThreads >> lr_log;
    const int lane_q = threadIdx.x & (LR - 1);
    const int rows = ex * ey;
    for (int r = threadIdx.x >> lr_log; r < rows; r += rpi) {
        const int cx = r / ey;
        const int cy = r - cx * ey;
        const int gx = G.lo[0] + cx, gy = G.lo[1] + cy;
        const uint32_t grow = INSIDE ? elem_index(S, gx, gy, G.lo[2]) : 0u;
        for (int q = lane_q; q < quads; q += LR)
            stage_quad<T, LT, INSIDE, LBL>(J, S, G, gx, gy, 4 * q, grow, s_img + r * P,
                                       s_lbl + r * P);
    }
}

// Copy the tile's input footprint into LDS in the input type (labels as int8), with
// fill / label_fill in cells outside the volume.  Each lane moves 4
// consecutive cells of one row: buffer loads from one VGPR offset (the cell
// steps are immediates), one 16-byte and one 4-byte LDS store.  When the whole
// footprint lies inside the volume no per-cell test is compiled in.
template <typename T, typename LT>
__device__ __forceinline__ void stage_footprint(const FwdJob &J, const Src &S, const TileGeom &G,
                                                LT *s_img, int8_t *s_lbl)
{
    const bool labels = (J.flags & kFlagLabels) != 0;
    const bool inside = G.lo[0] >= 0 && G.lo[1] >= 0 && G.lo[2] >= 0 &&
                        G.lo[0] + G.e[0] <= J.nx && G.lo[1] + G.e[1] <= J.ny &&
                        G.lo[2] + 4 * G.quads <= J.nz;
    if (inside) {
        if (labels)
            stage_rows<T, LT, true, true>(J, S, G, s_img, s_lbl);
        else
            stage_rows<T, LT, true, false>(J, S, G, s_img, s_lbl);
    } else {
        if (labels)
            stage_rows<T, LT, false, true>(J, S, G, s_img, s_lbl);
        else
            stage_rows<T, LT, false, false>(J, S, G, s_img, s_lbl);
    }
}

}  // namespace ctaug
