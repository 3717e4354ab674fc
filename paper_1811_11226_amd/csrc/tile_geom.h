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

#include <climits>

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
    // an interior footprint whose last quad would reach past z = nz - 1 starts
    // its z window earlier (the extra cells are in the volume), so that every
    // staged quad of an interior tile lies inside the volume
    if (G.cls == kInterior && 4 * G.quads <= J.nz && G.lo[2] + 4 * G.quads > J.nz) {
        const int shift = G.lo[2] + 4 * G.quads - J.nz;
        G.lo[2] -= shift;
        G.e[2] += shift;
    }
    // an int16 footprint must hold fill exactly
    G.lds = !outside && cells <= lds_cells && (!(J.flags & kFlagLds16) || (J.flags & kFlagFillInT));
    return G;
}

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

// The raw bytes of four consecutive input cells of type T at element offset e
// (one wide load), and their store as LDS cells of type LT.
template <typename T> struct QuadRaw;
template <> struct QuadRaw<float> {
    typedef u32x4 type;
    static __device__ __forceinline__ type load(rsrc_t r, uint32_t e)
    {
        return __builtin_amdgcn_raw_buffer_load_b128(r, e * 4u, 0, 0);
    }
    static __device__ __forceinline__ void store(type w, float *dst)
    {
        *reinterpret_cast<u32x4 *>(dst) = w;
    }
};
template <> struct QuadRaw<int16_t> {
    typedef u32x2 type;
    static __device__ __forceinline__ type load(rsrc_t r, uint32_t e)
    {
        return __builtin_amdgcn_raw_buffer_load_b64(r, e * 2u, 0, 0);
    }
    static __device__ __forceinline__ void store(type w, int16_t *dst)
    {
        *reinterpret_cast<u32x2 *>(dst) = w;
    }
    static __device__ __forceinline__ void store(type w, float *dst)
    {
        *reinterpret_cast<f32x4 *>(dst) =
            f32x4{(float)(int16_t)(w.x & 0xffffu), (float)((int32_t)w.x >> 16),
                  (float)(int16_t)(w.y & 0xffffu), (float)((int32_t)w.y >> 16)};
    }
};

// floor(a / b) for 0 <= a < 2^24, 0 < b < 2^16: FP32 reciprocal estimate and
// one integer correction step.
__device__ __forceinline__ int div_small(int a, int b, float rcp_b)
{
    int q = (int)((float)a * rcp_b);
    const int r = a - q * b;
    q += (r >= b) - (r < 0);
    return q;
}

// A quad of four input cells (gx, gy, gz0 .. gz0 + 3) wholly inside the volume,
// at element offset e: one wide load.
template <typename T, typename LT>
__device__ __forceinline__ void quad_inside(const Src &S, uint32_t e, LT *dst)
{
    copy_quad(S.img, e * (uint32_t)sizeof(T), dst, T());
}

// A quad of an in-volume row (element offset e_row0 of its z = 0 cell) whose
// z range leaves the volume: each cell is loaded from its z clamped into the
// volume (every load stays in range) and replaced by fill outside.
template <typename T, typename LT>
__device__ __forceinline__ void quad_partial(const FwdJob &J, const Src &S, int e_row0, int gz0,
                                             LT *dst)
{
    constexpr uint32_t es = sizeof(T);
    const LT tfill = (LT)J.fill;
    LT v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int gz = gz0 + u;
        const uint32_t e = (uint32_t)(e_row0 + min(max(gz, 0), J.nz - 1));
        const T raw = Elem<T>::raw(S.img, e * es, 0);
        v[u] = (unsigned)gz < (unsigned)J.nz ? (LT)raw : tfill;
    }
    store4(dst, v);
}

// A quad of a row outside the volume: fill, nothing loaded.
template <typename LT>
__device__ __forceinline__ void quad_fill(const FwdJob &J, LT *dst)
{
    const LT tfill = (LT)J.fill;
    const LT v[4] = {tfill, tfill, tfill, tfill};
    store4(dst, v);
}

// Row walk of the footprint staging: the lane takes rows row, row + rpp, ...
// (rpp = rows per pass), tracking the row's input cell (cx, cy), its element
// offset and its LDS offset by additions of per-tile constants.
struct RowWalk {
    int row, cx, cy, e_row, l_row;     // e_row: element offset of cell (lo0 + cx, lo1 + cy, 0)
    int rpp, step_x, step_y, ey, de, de_wrap, dl;

    __device__ __forceinline__ void init(const Src &S, const TileGeom &G, int first_row,
                                         int rows_per_pass, int lane_cell)
    {
        ey = G.e[1];
        rpp = rows_per_pass;
        const float rcp_y = 1.0f / (float)ey;
        step_x = div_small(rpp, ey, rcp_y);            // rpp = step_x * ey + step_y
        step_y = rpp - step_x * ey;
        row = first_row;
        cx = div_small(row, ey, rcp_y);
        cy = row - cx * ey;
        const int plane = S.ry * S.rsy;                 // elements per x plane
        e_row = (G.lo[0] + cx) * plane + (G.lo[1] + cy) * S.rsy;
        de = step_x * plane + step_y * S.rsy;
        de_wrap = plane - ey * S.rsy;
        l_row = row * G.pitch + lane_cell;
        dl = rpp * G.pitch;
    }
    __device__ __forceinline__ void next()
    {
        row += rpp;
        cx += step_x;
        cy += step_y;
        e_row += de;
        l_row += dl;
        if (cy >= ey) {
            cy -= ey;
            cx += 1;
            e_row += de_wrap;
        }
    }
};

// Copy the tile's input image footprint into LDS in the LDS cell type, with
// fill in cells outside the volume (labels are gathered from global memory
// while sampling, so that the LDS holds image cells only).  The footprint is
// e[0] x e[1] rows of `quads` quads of 4 cells (row pitch G.pitch cells).
// A row of at most 16 quads is taken by `quads` consecutive lanes, one quad
// each, so a workgroup covers floor(256 / quads) rows per pass with every lane
// but the last 256 mod quads busy; a longer row is taken by 16 lanes (a lane
// takes quads q, q + 16, ...).  Rows advance by additions (RowWalk), with no
// per-quad division or multiplication.  An interior footprint (every quad
// inside the volume, see box_geom) of at most 16 quads per row is copied
// without any test: each lane issues the loads of four rows before it
// converts and writes them.  Other footprints test each row and quad: rows
// outside the volume are filled without loads, quads crossing its z ends
// load per cell from clamped indices.
template <typename T, typename LT>
__device__ __forceinline__ void stage_footprint(const FwdJob &J, const Src &S, const TileGeom &G,
                                                LT *s_img)
{
    const int qpr = G.quads, rows = G.e[0] * G.e[1];
    int lpr, ql, row0, rpp;
    if (qpr <= 16) {
        // qpr lanes per row, floor(256 / qpr) rows per pass; lanes past the
        // last whole row stay idle (ql = qpr)
        lpr = qpr;
        row0 = div_small(threadIdx.x, qpr, 1.0f / (float)qpr);
        rpp = kThreads / qpr;
        ql = row0 < rpp ? threadIdx.x - row0 * qpr : qpr;
    } else {
        lpr = 16;
        row0 = threadIdx.x >> 4;
        rpp = kThreads >> 4;
        ql = threadIdx.x & 15;
    }
    RowWalk W;
    W.init(S, G, row0, rpp, 4 * min(ql, qpr - 1));
    const bool fast = G.cls == kInterior && G.lo[2] >= 0 && G.lo[2] + 4 * qpr <= J.nz &&
                      qpr <= 16;
    if (fast) {
        if (ql >= qpr)
            return;                    // lanes past the last whole row stay idle
        const int gz0 = G.lo[2] + 4 * ql;
        constexpr int B = 4;           // rows whose loads are in flight together
        for (; W.row < rows;) {
            uint32_t e[B];
            int l[B];
            bool ok[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                ok[u] = W.row < rows;
                e[u] = (uint32_t)(W.e_row + gz0);
                l[u] = W.l_row;
                W.next();
            }
            typename QuadRaw<T>::type w[B];
#pragma unroll
            for (int u = 0; u < B; ++u)
                w[u] = QuadRaw<T>::load(S.img, ok[u] ? e[u] : e[0]);   // in the volume either way
#pragma unroll
            for (int u = 0; u < B; ++u) {
                if (!ok[u])
                    break;
                QuadRaw<T>::store(w[u], s_img + l[u]);
            }
        }
        return;
    }
    for (; W.row < rows; W.next()) {
        const int gx = G.lo[0] + W.cx, gy = G.lo[1] + W.cy;
        const bool row_in = (unsigned)gx < (unsigned)J.nx && (unsigned)gy < (unsigned)J.ny;
        for (int q = ql; q < qpr; q += lpr) {
            const int gz0 = G.lo[2] + 4 * q;
            LT *dst = s_img + W.l_row + 4 * (q - ql);
            if (!row_in)
                quad_fill<LT>(J, dst);
            else if (gz0 >= 0 && gz0 + 3 < J.nz)
                quad_inside<T, LT>(S, (uint32_t)(W.e_row + gz0), dst);
            else
                quad_partial<T, LT>(J, S, W.e_row, gz0, dst);
        }
    }
}

// Workgroup-wide min of mn[] and max of mx[] (3 ints each); every thread gets
// the result.  s_red: 4 x 6 ints of LDS.  Ends with a barrier.
__device__ __forceinline__ void block_minmax3(int mn[3], int mx[3], int (*s_red)[6])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            mn[i] = min(mn[i], __shfl_xor(mn[i], off, 64));
            mx[i] = max(mx[i], __shfl_xor(mx[i], off, 64));
        }
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            s_red[wave][i] = mn[i];
            s_red[wave][3 + i] = mx[i];
        }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        mn[i] = s_red[0][i];
        mx[i] = s_red[0][3 + i];
#pragma unroll
        for (int w = 1; w < kThreads / 64; ++w) {
            mn[i] = min(mn[i], s_red[w][i]);
            mx[i] = max(mx[i], s_red[w][3 + i]);
        }
    }
    __syncthreads();
}

// Footprint of an output box from the range [fmn, fmx] of floor(q) over its
// guarded samples (fmn > fmx: no guarded sample): cells floor(q) .. floor(q) + 1,
// clamped to [-1, n].
__device__ __forceinline__ TileGeom geom_from_cells(const FwdJob &J, int x0, int y0, int z0,
                                                    int x1, int y1, int z1, const int fmn[3],
                                                    const int fmx[3], int32_t lds_cells)
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
    if (fmn[0] > fmx[0]) {
        G.cls = kOutside;
        return G;
    }
    const int n[3] = {J.nx, J.ny, J.nz};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int a = max(fmn[i], -1), b = min(fmx[i] + 1, n[i]);
        G.lo[i] = a;
        G.e[i] = b - a + 1;
    }
    G.quads = (G.e[2] + 3) >> 2;
    G.pitch = lds_pitch(G.e[2]);
    // samples outside the guard may remain: always the per-sample checked path
    G.cls = kBoundary;
    G.lds = (int64_t)G.e[0] * G.e[1] * G.pitch <= lds_cells;
    return G;
}

}  // namespace ctaug
