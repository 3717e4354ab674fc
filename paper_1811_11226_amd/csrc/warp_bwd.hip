// warp_bwd.hip -- adjoint kernels of the warp (gfx950).
//
// Persistent workgroups over 8 x 8 x 16 output tiles.  For every output voxel
// the upstream gradient is taken through the adjoint of the photometric chain
// (gain, zero on the occluded slab), the forward coordinate and cell are
// recomputed; the eight corner values
// (staged in LDS, fill substituted outside the volume) give the derivative of
// the trilinear interpolant on that cell, dV/dq.  Then
//   grad_img[c] += w_c * g          summed per tile in fixed point in LDS
//                                   (integer atomics, order-independent; 32
//                                   bits in one pass where the host bounds a
//                                   cell's samples, else 64 bits in x-plane
//                                   passes), then one global FP32 atomic per touched
//                                   cell; tiles whose footprint exceeds the
//                                   reservation, or with non-finite g, add
//                                   per corner with global FP32 atomics
//   grad_disp[i](p) = g * dV/dq_i   coalesced SoA stores
//   grad_ctrl                        B-spline warps evaluated from a control
//                                   grid: the tile's g dV/dq is contracted
//                                   with the spline weights along z, y and x
//                                   in LDS and added to the workgroup's LDS
//                                   accumulators of the control entries; one
//                                   row per workgroup, summed in a fixed order
//   grad_M[i][j] = sum g dV/dq_i [x,y,z,1]_j, FP64 per thread, reduced in the
//   workgroup and then across workgroups in a fixed order.
// grad_M and grad_ctrl are deterministic for a given device; grad_img is
// deterministic within a tile, and tiles meet in FP32 atomics.
#include "device_common.h"
#include "launch.h"
#include "tile_geom.h"

#include <algorithm>
#include <climits>
#include <cstring>
#include <cmath>
#include <mutex>
#include <vector>

namespace ctaug {

// Launch shape of the backward pass: 8 x 8 x 16 voxel tiles (one run of 4 z
// voxels per thread), persistent workgroups striding over their XCD's tiles
// (xcd_tile), and at most kBwdLdsCells FP32 cells of input footprint per
// workgroup (48 KB of LDS), used first for the staged image, then as the
// adjoint accumulators of the same cells.
constexpr Tiling kBwdTiling = {3, 3, 4};
constexpr int32_t kBwdLdsCells = 12288;
constexpr int64_t kBwdMaxGrid = kBwdMaxRows;

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

// Largest control grid (3 Gx Gy Gz entries) whose gradient is fused into the
// adjoint kernel: FP32 accumulators in LDS beside a footprint reservation
// shrunk by as much, so that the workgroup's LDS stays at 48 KB; one FP64 row
// per workgroup in the workspace; rows summed in kCtrlRowGroups groups, then
// the groups (both in a fixed order).
constexpr int32_t kCtrlMaxEntries = 2048;
constexpr int32_t kSplineBwdCells = kBwdLdsCells - kCtrlMaxEntries;
constexpr int32_t kCtrlRowGroups = 64;
static_assert(kSplineTileLdsFloats <= kSplineBwdCells, "the B-spline scratch fits the reservation");

// v + (v of the lane at quad position q ^ 1), then ^ 2: sum over the 4 lanes
// of a quad, in the same order on every lane (DPP quad permutes, no LDS).
__device__ __forceinline__ float quad_sum(float v)
{
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
    return v;
}

// Fixed-point image adjoint.  A tile's contributions w_c * g are added into
// 64-bit integer LDS accumulators (integer LDS atomics run at full rate where
// FP32 ones do not, and integer sums do not depend on the order of the
// additions): with gmax the tile's largest |g| and gmax < 2^e, each FP32
// contribution v is scaled by S = 2^(50 - e) (exact) and rounded to the
// nearest integer (ties to even), so |v S| < 2^50 and, as the weights of a
// sample sum to 1, every cell's sum over the tile's 1024 samples stays below
// 2^60.  The rounding adds 1.5 * 2^52 in FP64, which leaves the integer in
// the low mantissa bits: two integer operations recover it.
__device__ __forceinline__ long long to_fixed(float v, double S)
{
    constexpr double kMagic = 0x1.8p52;
    const double d = __builtin_fma((double)v, S, kMagic);
    return __double_as_longlong(d) - __double_as_longlong(kMagic);
}

// The 32-bit variant for affine jobs, one pass over the whole footprint (the
// accumulators take the cells the staged image took).  The host bounds how
// many of a tile's samples can have one input cell among their corners: at
// most 2^b (fixed32_bits).  Each contribution is scaled by 2^sc, sc = 30 - b
// - e (exact: the voxel's gradient is multiplied by the power of two before
// the weights, which rounds as the unscaled product would), and rounded to
// the nearest integer: |v 2^sc| < 2^(30 - b), so a cell's sum of at most 2^b
// of them stays within 2^30.  The unit 2^-sc is at most 2^(b - 29) gmax, so
// for b <= kFixed32MaxBits the rounding stays within 2^-23 gmax, the order
// of the FP32 product's own.
constexpr int kFixed32MaxBits = 7;

// Spline weight matrix of one tile axis: Wt[p][c] = B_{c - (i(p) - i(p0))}(t(p))
// for the 2^lp voxels p0 + p <= p1 of the axis and the window of kSplineWindow
// controls starting at i(p0); 0 elsewhere.  One entry per calling thread.
__device__ __forceinline__ void spline_weight_entry(int e, int p0, int p1, float inv_h, int32_t G,
                                                    float *Wt)
{
    const int p = p0 + (e / kSplineWindow), c = e % kSplineWindow;
    float w = 0.0f;
    if (p <= p1) {
        int32_t i;
        float t, Bw[4];
        bs_cell(p, inv_h, G, i, t);
        bs_basis(t, Bw);
        const int j = c - (i - bs_index(p0, inv_h, G));
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
            if (j == jj)
                w = Bw[jj];
    }
    Wt[e] = w;
}

// Control-grid adjoint of one 8 x 8 x 16 displacement tile.  gu[k][i] is
// g dV/dq_i of voxel k of the thread's run (0 outside the tile or the guard).
// Contractions in LDS, each in a fixed order (FP32 inside the tile):
//   W[row][i][c]   = sum_z  Zw[z][c] gu_i(row, z)        (4 lanes of a row, butterfly)
//   H[x][i][b][c]  = sum_y  Yw[y][b] W[(x, y)][i][c]
//   R[i][a][b][c]  = sum_x  Xw[x][a] H[x][i][b][c]
// then R is added to the workgroup's FP32 accumulators acc (LDS, one per
// control entry; each entry is updated by one thread per tile and tiles come
// in a fixed order, so the sums are deterministic).  Every axis window must
// hold at most kSplineWindow controls (checked on the host).  The caller
// guarantees that no thread reads the scratch LDS on entry; ends with a
// barrier.
__device__ __forceinline__ void ctrl_adjoint_tile(const BsplineGeom &B, int x0, int y0, int z0,
                                                  int x1, int y1, int z1, int rr, int zr,
                                                  const float (&gu)[4][3], float *lds, float *acc)
{
    constexpr int NW = kSplineWindow;
    static_assert(NW == 8, "window entries are indexed with 3-bit fields");
    float *Zw = lds;                           // [16][NW]
    float *Yw = Zw + 16 * NW;                  // [8][NW]
    float *Xw = Yw + 8 * NW;                   // [8][NW]
    float *W = Xw + 8 * NW;                    // [64][3][NW]
    float *H = W + 64 * 3 * NW;                // [8][3][NW][NW]
    float *R = H + 8 * 3 * NW * NW;            // [3][NW][NW][NW]
    static_assert(16 * NW + 16 * NW + 64 * 3 * NW + 8 * 3 * NW * NW + 3 * NW * NW * NW <=
                      kSplineBwdCells,
                  "the tile's contraction scratch fits the footprint reservation");
    const int t = threadIdx.x;
    // controls of the tile's window per axis (at most NW): contractions stop
    // there, as every weight beyond is zero and no later stage reads beyond
    const int ixl = bs_index(x0, B.inv_hx, B.gx), iyl = bs_index(y0, B.inv_hy, B.gy),
              izl = bs_index(z0, B.inv_hz, B.gz);
    const int ncx = bs_index(x1, B.inv_hx, B.gx) - ixl + 4,
              ncy = bs_index(y1, B.inv_hy, B.gy) - iyl + 4,
              ncz = bs_index(z1, B.inv_hz, B.gz) - izl + 4;
    if (t < 16 * NW)
        spline_weight_entry(t, z0, z1, B.inv_hz, B.gz, Zw);
    else if (t < 24 * NW)
        spline_weight_entry(t - 16 * NW, y0, y1, B.inv_hy, B.gy, Yw);
    else if (t < 32 * NW)
        spline_weight_entry(t - 24 * NW, x0, x1, B.inv_hx, B.gx, Xw);
    __syncthreads();
    // z: the 4 lanes of a row hold its 16 voxels; butterfly sum over them
#pragma unroll 1
    for (int c = 0; c < ncz; ++c) {
        const float *zc = Zw + zr * NW + c;    // voxel k of the run sits at z offset zr + 4k
        const float w0 = zc[0], w1 = zc[4 * NW], w2 = zc[8 * NW], w3 = zc[12 * NW];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            float v = w0 * gu[0][i];
            v = __builtin_fmaf(w1, gu[1][i], v);
            v = __builtin_fmaf(w2, gu[2][i], v);
            v = __builtin_fmaf(w3, gu[3][i], v);
            v = quad_sum(v);
            if (zr == 0)
                W[(rr * 3 + i) * NW + c] = v;
        }
    }
    __syncthreads();
    if (t < 8 * 3 * NW && (t & (NW - 1)) < ncz) {   // (x, i, c) -> H[x][i][b][c], b < ncy
        const int xr = t / (3 * NW), ic = t - xr * 3 * NW;
        const int i = ic / NW, c = ic - i * NW;
        float wv[8];
#pragma unroll
        for (int yr = 0; yr < 8; ++yr)
            wv[yr] = W[((xr * 8 + yr) * 3 + i) * NW + c];
#pragma unroll 1
        for (int b = 0; b < ncy; ++b) {
            float h = 0.0f;
#pragma unroll
            for (int yr = 0; yr < 8; ++yr)
                h = __builtin_fmaf(Yw[yr * NW + b], wv[yr], h);
            H[((xr * 3 + i) * NW + b) * NW + c] = h;
        }
    }
    __syncthreads();
    if (t < 3 * NW * NW && (t & (NW - 1)) < ncz && ((t >> 3) & (NW - 1)) < ncy) {
        // (i, b, c) -> R[i][a][b][c], a < ncx
        const int i = t / (NW * NW), bc = t - i * NW * NW;
        float hv[8];
#pragma unroll
        for (int xr = 0; xr < 8; ++xr)
            hv[xr] = H[(xr * 3 + i) * NW * NW + bc];
#pragma unroll 1
        for (int a = 0; a < ncx; ++a) {
            float r = 0.0f;
#pragma unroll
            for (int xr = 0; xr < 8; ++xr)
                r = __builtin_fmaf(Xw[xr * NW + a], hv[xr], r);
            R[(i * NW + a) * NW * NW + bc] = r;
        }
    }
    __syncthreads();
    for (int e = t; e < 3 * NW * NW * NW; e += kThreads) {
        const int c = e & (NW - 1), b = (e >> 3) & (NW - 1), a = (e >> 6) & (NW - 1), i = e >> 9;
        if (a < ncx && b < ncy && c < ncz)
            acc[((i * B.gx + ixl + a) * B.gy + iyl + b) * B.gz + izl + c] += R[e];
    }
    __syncthreads();
}

// The workgroup's sum of acc[12] (fixed order: wave butterflies, then the
// four waves in order) written to row[0..11].  Every thread must call it;
// ends after a barrier.
__device__ __forceinline__ void write_partial_row(const double (&acc)[12],
                                                  double (*red)[12], double *row)
{
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
        row[threadIdx.x] = sum;
    }
    __syncthreads();                   // red is reused by the next row
}

// The upstream gradient of the calling thread's run in tile t of job J
// (voxels z0 + zr + 4k of row (x0 + xr, y0 + yr)); 0 past the output.
__device__ __forceinline__ void load_run_g(const FwdJob &J, const float *__restrict__ g, int t,
                                           int zr, int yr, int xr, float (&gv)[4])
{
    const Tiling TL = kBwdTiling;
    const int tz = t % J.tiles_z, rest = t / J.tiles_z;
    const int ty = rest % J.tiles_y, tx = rest / J.tiles_y;
    const int x = (tx << TL.lx) + xr, y = (ty << TL.ly) + yr, z = (tz << TL.lz) + zr;
    const bool row_ok = x < J.ox && y < J.oy;
    const int32_t v0 = row_ok ? (x * J.oy + y) * J.oz + z : 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        gv[k] = row_ok && z + 4 * k < J.oz ? g[v0 + 4 * k] : 0.0f;
}

// The adjoint of one 8 x 8 x 16 output tile t of job J, for the calling
// thread's run (voxels z0 + zr + 4k of row (xr, yr)): coordinates, the
// staged footprint, dV/dq and its FP64 parameter sums (into acc), the image
// adjoint (fixed-point tile sums, flushed with FP32 atomics), the
// displacement gradient and the control-grid contraction.  gin holds the
// run's upstream gradient (load_run_g); the next tile's (tn of job Jn, when
// has_next) is loaded into gnext once the image scatter is done, so that its
// latency hides behind the flush.  Uniform over the workgroup; ends with
// every LDS read and write of the tile done.
template <typename T, int DISP, bool NARROW>
__device__ __forceinline__ void bwd_tile(const FwdJob &J, int t, const Src &src,
                                         gconst<float> *disp, int32_t nvox, bool empty_in,
                                         bool want_ctrl, bool need_dv, const float (&gin)[4],
                                         bool has_next, const FwdJob &Jn,
                                         const float *__restrict__ gn, int tn, float (&gnext)[4],
                                         float *__restrict__ g_img, float *__restrict__ g_disp,
                                         float *s_ctrl, int32_t lds_cells, int fix_bits, int zr,
                                         int yr, int xr, double (&acc)[12], int (*s_red)[6],
                                         float *s_gmax)
{
    const Tiling TL = kBwdTiling;
    const int tz = t % J.tiles_z, rest = t / J.tiles_z;
    const int ty = rest % J.tiles_y, tx = rest / J.tiles_y;
    const int x0 = tx << TL.lx, y0 = ty << TL.ly, z0 = tz << TL.lz;
    const int x1 = min(x0 + (1 << TL.lx), J.ox) - 1, y1 = min(y0 + (1 << TL.ly), J.oy) - 1,
              z1 = min(z0 + (1 << TL.lz), J.oz) - 1;
    const int x = x0 + xr, y = y0 + yr, z = z0 + zr;
    const bool run_ok = x <= x1 && y <= y1 && z <= z1;
    bool fetched = false;              // gnext loaded (uniform)
    const int nvalid = run_ok ? min(4, (z1 - z) / 4 + 1) : 0;
    const int32_t v0 = run_ok ? (x * J.oy + y) * J.oz + z : 0;
    // coordinates, guard and upstream gradient of the run's voxels
    float qv[4][3], gpk[4];
    bool gd[4];
    float u[3][4];
    if (DISP == kDispSpline)
        spline_tile_u<kThreads, false>(J.ctrl, J.bs, TL.lx, TL.ly, x0, y0, z0, x1, y1, z1,
                                       threadIdx.x >> 2, x, y, z, 4, nvalid, run_ok,
                                       s_cells, u);
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
            const int32_t v = v0 + 4 * k;
            const float zf = (float)(z + 4 * k);
            float qx = coord(J.M, 0, rb, zf), qy = coord(J.M, 1, rb, zf),
                  qz = coord(J.M, 2, rb, zf);
            if (DISP == kDispField) {
                qx = qx + disp[v];
                qy = qy + disp[nvox + v];
                qz = qz + disp[2 * nvox + v];
            } else if (DISP == kDispSpline) {
                qx = qx + u[0][k];
                qy = qy + u[1][k];
                qz = qz + u[2][k];
            }
            qv[k][0] = qx;
            qv[k][1] = qy;
            qv[k][2] = qz;
            gd[k] = !empty_in && in_guard(qx, qy, qz, J.nx, J.ny, J.nz);
            // adjoint of the photometric chain without window: the output
            // is gain * V + offset + sigma * n off the occluded slab and
            // does not depend on V on it
            float gv = gin[k];
            if (J.flags & kFlagPhoto) {
                gv = J.gain * gv;
                if ((J.flags & kFlagOcclude) && zf >= J.occ_lo && zf <= J.occ_hi)
                    gv = 0.0f;
            }
            gpk[k] = gv;
        }
    }
    TileGeom G;
    if (DISP != kDispNone) {
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
    if (lds && g_img) {
        // the tile's largest |g| over its guarded samples: reduced in each
        // wave here, across the waves after the barrier that ends the corner
        // reads; +inf when any g is not finite (NaN included, which fmaxf
        // alone would drop), which sends the tile to the per-corner FP32 path
        float gw = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (gd[k]) {
                const float a = fabsf(gpk[k]);
                gw = a <= 3.40282347e38f ? fmaxf(gw, a) : __builtin_inff();
            }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            gw = fmaxf(gw, __shfl_xor(gw, off, 64));
        if ((threadIdx.x & 63) == 0)
            s_gmax[threadIdx.x >> 6] = gw;
    }
    if (lds && need_dv) {              // the image adjoint alone needs no corner values
        stage_footprint<T, float>(J, src, G, s_cells);
        __syncthreads();
    }
    // per voxel of the run: LDS cell of corner (0,0,0), fractions, upstream gradient
    int base[4], cx0[4];
    float tw[4][3], gk[4];
    bool live[4] = {false, false, false, false};
    float S[3] = {0.0f, 0.0f, 0.0f}, Sz[3] = {0.0f, 0.0f, 0.0f};
    float gu[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        gu[k][0] = gu[k][1] = gu[k][2] = 0.0f;
    if (run_ok) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k >= nvalid)
                continue;
            const int32_t v = v0 + 4 * k;
            const float zf = (float)(z + 4 * k);
            const float qx = qv[k][0], qy = qv[k][1], qz = qv[k][2];
            const float gp = gpk[k];
            float dV[3] = {0.0f, 0.0f, 0.0f};
            if (gd[k]) {
                float K[8], tt[3];
                if (lds) {
                    const float fx = floorf(qx), fy = floorf(qy), fz = floorf(qz);
                    // LDS cell (i - lo) . (sxy, pitch, 1) in exact FP32 (integers < 2^24)
                    const int bs = (int)__builtin_fmaf(
                        fx - (float)G.lo[0], (float)sxy,
                        __builtin_fmaf(fy - (float)G.lo[1], (float)pitch, fz - (float)G.lo[2]));
                    tt[0] = qx - fx;
                    tt[1] = qy - fy;
                    tt[2] = qz - fz;
                    if (need_dv) {
                        K[0] = s_cells[bs];
                        K[1] = s_cells[bs + 1];
                        K[2] = s_cells[bs + pitch];
                        K[3] = s_cells[bs + pitch + 1];
                        K[4] = s_cells[bs + sxy];
                        K[5] = s_cells[bs + sxy + 1];
                        K[6] = s_cells[bs + sxy + pitch];
                        K[7] = s_cells[bs + sxy + pitch + 1];
                        cell_gradient(K, tt, dV);
                    }
                    if (g_img) {
                        live[k] = true;
                        base[k] = bs;
                        cx0[k] = (int)fx - G.lo[0];
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
                                    // zero contributions are skipped; a non-finite
                                    // g reaches every in-volume corner (0 * inf and
                                    // 0 * NaN are NaN), as in the per-corner path
                                    const float cw = wx[a] * wy[bb] * wz[c] * gp;
                                    const bool ok = cx >= 0 && cx < J.nx && cy >= 0 &&
                                                    cy < J.ny && cz >= 0 && cz < J.nz &&
                                                    cw != 0.0f;
                                    if (ok)
                                        unsafeAtomicAdd(g_img + (cx * J.ny + cy) * J.nz + cz,
                                                        cw);
                                }
                    }
                }
            }
            if (DISP != kDispNone && g_disp) {
                g_disp[v] = gp * dV[0];
                g_disp[nvox + v] = gp * dV[1];
                g_disp[2 * nvox + v] = gp * dV[2];
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const float c = gp * dV[i];
                gu[k][i] = c;
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
    if (lds)                           // uniform: no barrier is skipped by part of the group
        __syncthreads();               // every corner read of the staged image is done
    if (want_ctrl)                     // before the image scatter: gu dies here
        ctrl_adjoint_tile(J.bs, x0, y0, z0, x1, y1, z1, threadIdx.x >> 2, zr, gu, s_cells,
                          s_ctrl);
    if (lds) {
        if (g_img) {
            // the tile's largest |g| (the waves' maxima, written before the
            // barrier that ended the corner reads); every wave reads it before
            // any wave goes on to the next tile, which writes s_gmax again:
            // each branch below passes a barrier before the tile ends
            float gm = s_gmax[0];
#pragma unroll
            for (int w = 1; w < kThreads / 64; ++w)
                gm = fmaxf(gm, s_gmax[w]);
            // x-planes of 64-bit accumulators that fit the footprint reservation
            const int planes = (lds_cells >> 1) / sxy;
            const float rcp_pitch = 1.0f / (float)pitch, rcp_ey = 1.0f / (float)ey;
            if (NARROW && gm >= 0x1p-96f && gm <= 3.40282347e38f) {
                // one pass, 32-bit accumulators (gmax >= 2^-96 keeps every
                // scaled value and every flushed sum in the normal range)
                const int sc = 30 - fix_bits - (ilogbf(gm) + 1);
                const float S32 = __builtin_ldexpf(1.0f, sc);    // normal: sc in [-105, 125]
                int *s_acc = reinterpret_cast<int *>(s_cells);
                const int n = G.e[0] * sxy;                      // a multiple of 4
                for (int c = 4 * threadIdx.x; c < n; c += 4 * kThreads)
                    *reinterpret_cast<f32x4 *>(s_acc + c) = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                __syncthreads();
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (!live[k])
                        continue;
                    const float wx[2] = {1.0f - tw[k][0], tw[k][0]};
                    const float wy[2] = {1.0f - tw[k][1], tw[k][1]};
                    const float gks = gk[k] * S32;
                    const float gz0 = (1.0f - tw[k][2]) * gks, gz1 = tw[k][2] * gks;
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int bb = 0; bb < 2; ++bb) {
                            const float wxy = wx[a] * wy[bb];
                            int *row = s_acc + base[k] + a * sxy + bb * pitch;
                            atomicAdd(row, (int)__builtin_rintf(wxy * gz0));
                            atomicAdd(row + 1, (int)__builtin_rintf(wxy * gz1));
                        }
                    __builtin_amdgcn_sched_barrier(0);       // one voxel at a time
                }
                __syncthreads();
                if (has_next && !fetched) {
                    load_run_g(Jn, gn, tn, zr, yr, xr, gnext);
                    fetched = true;
                }
                // flush: one global atomic per touched in-volume footprint cell
                for (int c = threadIdx.x; c < n; c += kThreads) {
                    const int v = s_acc[c];
                    if (v == 0)
                        continue;
                    const int row = div_small(c, pitch, rcp_pitch);
                    const int cz = c - row * pitch;
                    const int cx = div_small(row, ey, rcp_ey);
                    const int cy = row - cx * ey;
                    const int gx = G.lo[0] + cx, gy = G.lo[1] + cy, gz = G.lo[2] + cz;
                    if (cz < G.e[2] && (unsigned)gx < (unsigned)J.nx &&
                        (unsigned)gy < (unsigned)J.ny && (unsigned)gz < (unsigned)J.nz)
                        unsafeAtomicAdd(g_img + (gx * J.ny + gy) * J.nz + gz,
                                        __builtin_ldexpf((float)v, -sc));
                }
                __syncthreads();       // LDS is reused next
            } else if (!NARROW && gm > 0.0f && gm <= 3.40282347e38f && planes > 0) {
                const int e = ilogbf(gm) + 1;          // gm < 2^e
                const double S = ldexp(1.0, 50 - e);
                const double rS = ldexp(1.0, e - 50);
                long long *s_acc = reinterpret_cast<long long *>(s_cells);
                for (int sx0 = 0; sx0 < G.e[0]; sx0 += planes) {   // uniform
                    const int np = min(planes, G.e[0] - sx0);
                    const int n = np * sxy;                        // a multiple of 4
                    for (int c = 2 * threadIdx.x; c < n; c += 2 * kThreads)
                        *reinterpret_cast<f32x4 *>(s_acc + c) = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if (!live[k])
                            continue;
                        const float wx[2] = {1.0f - tw[k][0], tw[k][0]};
                        const float wy[2] = {1.0f - tw[k][1], tw[k][1]};
                        const float gz0 = (1.0f - tw[k][2]) * gk[k], gz1 = tw[k][2] * gk[k];
#pragma unroll
                        for (int a = 0; a < 2; ++a) {
                            const int px = cx0[k] + a - sx0;
                            if ((unsigned)px >= (unsigned)np)
                                continue;
#pragma unroll
                            for (int bb = 0; bb < 2; ++bb) {
                                const float wxy = wx[a] * wy[bb];
                                unsigned long long *row = reinterpret_cast<unsigned long long *>(
                                    s_acc + base[k] - cx0[k] * sxy + px * sxy + bb * pitch);
                                atomicAdd(row, (unsigned long long)to_fixed(wxy * gz0, S));
                                atomicAdd(row + 1, (unsigned long long)to_fixed(wxy * gz1, S));
                            }
                        }
                        // one voxel's conversions at a time (register pressure)
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    __syncthreads();
                    // flush: one global atomic per touched in-volume footprint cell
                    for (int c = threadIdx.x; c < n; c += kThreads) {
                        const long long v = s_acc[c];
                        if (v == 0)
                            continue;
                        const int row = div_small(c, pitch, rcp_pitch);
                        const int cz = c - row * pitch;
                        const int cx = div_small(row, ey, rcp_ey);
                        const int cy = row - cx * ey;
                        const int gx = G.lo[0] + sx0 + cx, gy = G.lo[1] + cy,
                                  gz = G.lo[2] + cz;
                        if (cz < G.e[2] && (unsigned)gx < (unsigned)J.nx &&
                            (unsigned)gy < (unsigned)J.ny && (unsigned)gz < (unsigned)J.nz)
                            unsafeAtomicAdd(g_img + (gx * J.ny + gy) * J.nz + gz,
                                            (float)((double)v * rS));
                    }
                    __syncthreads();   // LDS is reused next
                }
            } else {
                __syncthreads();       // every wave has read s_gmax
                // non-finite gradients, a footprint too large for one x-plane
                // of 64-bit accumulators, or a 32-bit tile with gmax < 2^-96:
                // FP32 global atomics per corner (none when gmax = 0)
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (!live[k] || gm == 0.0f)
                        continue;
                    const int rel = base[k] - cx0[k] * sxy;
                    const int cy0 = rel / pitch, cz0 = rel - cy0 * pitch;
                    const float wx[2] = {1.0f - tw[k][0], tw[k][0]};
                    const float wy[2] = {1.0f - tw[k][1], tw[k][1]};
                    const float gz[2] = {(1.0f - tw[k][2]) * gk[k], tw[k][2] * gk[k]};
                    for (int a = 0; a < 2; ++a)
                        for (int bb = 0; bb < 2; ++bb)
                            for (int c = 0; c < 2; ++c) {
                                const int gx = G.lo[0] + cx0[k] + a, gy = G.lo[1] + cy0 + bb,
                                          gz2 = G.lo[2] + cz0 + c;
                                if ((unsigned)gx < (unsigned)J.nx &&
                                    (unsigned)gy < (unsigned)J.ny &&
                                    (unsigned)gz2 < (unsigned)J.nz)
                                    unsafeAtomicAdd(g_img + (gx * J.ny + gy) * J.nz + gz2,
                                                    wx[a] * wy[bb] * gz[c]);
                            }
                }
            }
        }
    }
    if (!fetched) {
        if (has_next)
            load_run_g(Jn, gn, tn, zr, yr, xr, gnext);
        else
#pragma unroll
            for (int k = 0; k < 4; ++k)
                gnext[k] = 0.0f;
    }
}

// Register budgets follow the LDS: a displacement takes the whole 48 KB
// reservation (3 workgroups per CU), so at most 168 VGPRs (3 waves per SIMD);
// an affine job's footprint bound usually keeps a workgroup within 40 KB
// (4 per CU), so at most 128 VGPRs, a few of them spilled.  NARROW (affine
// jobs with a bound fix_bits >= 0) takes the 32-bit image adjoint: a kernel
// of its own, as register allocation over both fixed-point paths spills.
template <typename T, int DISP, bool NARROW>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(
    DISP == kDispNone ? 4 : 3))) void k_warp_bwd(FwdJob J, const float *__restrict__ g,
                                                       float *__restrict__ g_img,
                                                       float *__restrict__ g_disp,
                                                       double *__restrict__ partials,
                                                       double *__restrict__ ctrl_part,
                                                       int32_t ntiles, int32_t lds_cells,
                                                       int32_t fix_bits)
{
    const int b = blockIdx.x;
    const int per_xcd_wg = gridDim.x >> 3;
    const Src src = make_src<T>(J);
    gconst<float> *disp = gc<float>(J.disp);
    const int32_t nvox = J.ox * J.oy * J.oz;
    const bool empty_in = J.nx == 0 || J.ny == 0 || J.nz == 0;   // every sample is fill

    double acc[12];
#pragma unroll
    for (int i = 0; i < 12; ++i)
        acc[i] = 0.0;

    // B-spline warps: this workgroup's control-grid gradient accumulators, in
    // LDS after the footprint reservation
    const bool want_ctrl = DISP == kDispSpline && ctrl_part != nullptr;
    const int32_t nctrl = 3 * J.bs.gx * J.bs.gy * J.bs.gz;
    // dV/dq (and so the staged corner values) is needed by every output but grad_img
    const bool need_dv = partials != nullptr || g_disp != nullptr || want_ctrl;
    float *s_ctrl = s_cells + lds_cells;
    if (want_ctrl) {
        for (int e = threadIdx.x; e < nctrl; e += kThreads)
            s_ctrl[e] = 0.0f;
        __syncthreads();
    }

    __shared__ int s_red[kThreads / 64][6];
    __shared__ float s_gmax[kThreads / 64];

    // this thread's run inside every tile: voxels z0 + zr + 4k, k = 0..3, of row
    // (xr, yr).  Lanes next to each other take neighbouring z, so that the LDS
    // accumulator updates of one instruction fall in different banks.
    const int zr = threadIdx.x & 3;
    const int yr = (threadIdx.x >> 2) & 7;
    const int xr = threadIdx.x >> 5;

    XcdSlots slots(b >> 3, per_xcd_wg);
    int t = xcd_tile(b & 7, slots.slot());
    float gcur[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (t < ntiles)
        load_run_g(J, g, t, zr, yr, xr, gcur);
    while (t < ntiles) {
        slots.next();
        const int tn = xcd_tile(b & 7, slots.slot());
        float gnext[4];
        // affine: the next tile's gradient is loaded during this tile's flush;
        // a displacement's tiles load their own at the start
        bwd_tile<T, DISP, NARROW>(J, t, src, disp, nvox, empty_in, want_ctrl, need_dv, gcur,
                                  DISP == kDispNone && tn < ntiles, J, g, tn, gnext, g_img, g_disp,
                                  s_ctrl, lds_cells, fix_bits, zr, yr, xr, acc, s_red, s_gmax);
        if (DISP != kDispNone && tn < ntiles)
            load_run_g(J, g, tn, zr, yr, xr, gnext);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            gcur[k] = gnext[k];
        t = tn;
    }

    if (want_ctrl)                         // the last tile ended with a barrier
        for (int e = threadIdx.x; e < nctrl; e += kThreads)
            ctrl_part[(int64_t)blockIdx.x * nctrl + e] = (double)s_ctrl[e];

    if (!partials)
        return;
    __shared__ double red[kThreads / 64][12];
    write_partial_row(acc, red, partials + (int64_t)blockIdx.x * 12);
}

// Batched adjoint: the tiles of up to kBwdBatchMax jobs in one persistent
// launch, the job table passed by value in the kernel arguments (no upload,
// nothing to allocate).  prefix[j] = first global tile of job j,
// prefix[njobs] = total; workgroups stride over their XCD's tiles in
// increasing order (xcd_tile), so the jobs a workgroup meets come in
// increasing order.  The
// workgroup's FP64 parameter sums of job j go to partials row
// j * gridDim.x + b; it writes zeros to the rows of the jobs it never meets
// (no zeroing launch before).
template <typename T, bool NARROW>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_warp_bwd_batch(const BwdBatch B,
                                                             double *__restrict__ partials,
                                                             int32_t lds_cells)
{
    const int total = B.prefix[B.njobs];
    const int b = blockIdx.x;
    const int per_xcd_wg = gridDim.x >> 3;
    __shared__ int s_red[kThreads / 64][6];
    __shared__ float s_gmax[kThreads / 64];
    __shared__ double red[kThreads / 64][12];
    const int zr = threadIdx.x & 3;
    const int yr = (threadIdx.x >> 2) & 7;
    const int xr = threadIdx.x >> 5;
    double acc[12];
#pragma unroll
    for (int i = 0; i < 12; ++i)
        acc[i] = 0.0;
    // rows of jobs jlo .. jhi - 1, which this workgroup does not meet: zeros
    // (only jobs with grad_M have rows: without any, partials may be null)
    auto zero_rows = [&](int jlo, int jhi) {
        for (int e = threadIdx.x; e < (jhi - jlo) * 12; e += kThreads) {
            const int jj = jlo + e / 12;
            if (B.jobs[jj].g_M)
                partials[((int64_t)jj * gridDim.x + b) * 12 + e % 12] = 0.0;
        }
    };
    auto job_of = [&](int t) {         // the job holding tile t (uniform)
        int j = 0;
        for (int i = 1; i < B.njobs; ++i)
            j += B.prefix[i] <= t;
        return j;
    };
    int jcur = -1;
    XcdSlots slots(b >> 3, per_xcd_wg);
    int t = xcd_tile(b & 7, slots.slot());
    int j = t < total ? job_of(t) : 0;
    float gcur[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (t < total)
        load_run_g(B.jobs[j].J, B.jobs[j].g, t - B.prefix[j], zr, yr, xr, gcur);
    while (t < total) {
        if (j != jcur) {               // the whole workgroup switches jobs (j > jcur)
            if (jcur >= 0 && B.jobs[jcur].g_M) {
                write_partial_row(acc, red, partials + ((int64_t)jcur * gridDim.x + b) * 12);
#pragma unroll
                for (int i = 0; i < 12; ++i)
                    acc[i] = 0.0;
            }
            zero_rows(jcur + 1, j);
            jcur = j;
        }
        slots.next();
        const int tn = xcd_tile(b & 7, slots.slot());
        const int jn = tn < total ? job_of(tn) : j;
        const BwdJob &BJ = B.jobs[j];
        const BwdJob &BN = B.jobs[jn];
        const Src src = make_src<T>(BJ.J);
        const bool empty_in = BJ.J.nx == 0 || BJ.J.ny == 0 || BJ.J.nz == 0;
        float gnext[4];
        bwd_tile<T, kDispNone, NARROW>(BJ.J, t - B.prefix[j], src, nullptr,
                                       BJ.J.ox * BJ.J.oy * BJ.J.oz, empty_in, false,
                                       BJ.g_M != nullptr, gcur, tn < total, BN.J, BN.g,
                                       tn - B.prefix[jn], gnext, BJ.g_img, nullptr, nullptr,
                                       lds_cells, B.fix_bits[j], zr, yr, xr, acc, s_red, s_gmax);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            gcur[k] = gnext[k];
        t = tn;
        j = jn;
    }
    if (jcur >= 0 && B.jobs[jcur].g_M)
        write_partial_row(acc, red, partials + ((int64_t)jcur * gridDim.x + b) * 12);
    zero_rows(jcur + 1, B.njobs);
}

// grad_M of job blockIdx.x: its rows j * nrows .. (j + 1) * nrows - 1 summed
// in a fixed order (jobs without grad_M are skipped).
__global__ __launch_bounds__(kThreads) void k_reduce12_batch(const BwdBatch B,
                                                             const double *__restrict__ partials,
                                                             int32_t nrows)
{
    double *out = B.jobs[blockIdx.x].g_M;
    if (!out)
        return;
    const double *rows = partials + (int64_t)blockIdx.x * nrows * 12;
    double acc[12];
#pragma unroll
    for (int i = 0; i < 12; ++i)
        acc[i] = 0.0;
#pragma unroll 4
    for (int r = threadIdx.x; r < nrows; r += kThreads)   // loads issue ahead; sums keep their order
#pragma unroll
        for (int i = 0; i < 12; ++i)
            acc[i] += rows[(int64_t)r * 12 + i];
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
        out[threadIdx.x] = sum;
    }
}

// Zero n doubles (rows of partials that a batched adjoint may leave unwritten).
__global__ __launch_bounds__(kThreads) void k_zero_f64(double *__restrict__ p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n)
        p[i] = 0.0;
}

// Sum n rows of 12 doubles in a fixed order into out[12].
__global__ __launch_bounds__(kThreads) void k_reduce12(const double *__restrict__ partials,
                                                       int32_t n, double *__restrict__ out)
{
    double acc[12];
#pragma unroll
    for (int i = 0; i < 12; ++i)
        acc[i] = 0.0;

#pragma unroll 4
    for (int r = threadIdx.x; r < n; r += kThreads)   // loads issue ahead; sums keep their order
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

// Control-grid rows, stage 1: group g (blockIdx.y) sums rows g*chunk ..
// (g+1)*chunk - 1 in order for 64 consecutive entries (one wave, coalesced).
__global__ __launch_bounds__(64) void k_reduce_ctrl_rows(const double *__restrict__ part,
                                                        int32_t rows, int32_t chunk, int32_t n,
                                                        double *__restrict__ groups)
{
    const int32_t e = blockIdx.x * 64 + threadIdx.x;
    if (e >= n)
        return;
    const int32_t r0 = blockIdx.y * chunk, r1 = min(r0 + chunk, rows);
    double s = 0.0;
#pragma unroll 8
    for (int32_t r = r0; r < r1; ++r)          // loads issue ahead; the sum keeps its order
        s += part[(int64_t)r * n + e];
    groups[(int64_t)blockIdx.y * n + e] = s;
}

// Stage 2: out[e] = sum over the groups in order (0 when there are none).
__global__ __launch_bounds__(kThreads) void k_reduce_ctrl_groups(const double *__restrict__ groups,
                                                                 int32_t ngroups, int32_t n,
                                                                 float *__restrict__ out)
{
    const int32_t e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= n)
        return;
    double s = 0.0;
#pragma unroll 8
    for (int32_t g = 0; g < ngroups; ++g)      // loads issue ahead; the sum keeps its order
        s += groups[(int64_t)g * n + e];
    out[e] = (float)s;
}

int64_t ctrl_reduce_doubles(int64_t rows, int64_t nctrl)
{
    return (rows + std::min<int64_t>(rows, kCtrlRowGroups)) * nctrl;
}

static hipError_t reduce_ctrl(const double *part, int32_t rows, int32_t n, float *out,
                              hipStream_t s)
{
    const int32_t ngroups = std::min(rows, kCtrlRowGroups);
    const double *groups = part + (int64_t)rows * n;
    if (ngroups > 0) {
        const int32_t chunk = (rows + ngroups - 1) / ngroups;
        hipLaunchKernelGGL(k_reduce_ctrl_rows, dim3((n + 63) / 64, ngroups), dim3(64), 0, s, part,
                           rows, chunk, n, const_cast<double *>(groups));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_reduce_ctrl_groups, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0,
                       s, groups, ngroups, n, out);
    return hipGetLastError();
}

// Host replica of bs_index (the same single FP32 multiply and floor).
static int32_t host_bs_index(int64_t p, float inv_h, int32_t G)
{
    const float s = (float)p * inv_h;
    return (int32_t)std::fmin(std::floor(s), (float)(G - 4));
}

// Largest number of controls any tile of extent 2^l touches along one axis.
static int32_t max_window(int64_t n, int l, float inv_h, int32_t G)
{
    int32_t w = 0;
    for (int64_t p0 = 0; p0 < n; p0 += (int64_t)1 << l) {
        const int64_t p1 = std::min(p0 + ((int64_t)1 << l), n) - 1;
        w = std::max(w, host_bs_index(p1, inv_h, G) - host_bs_index(p0, inv_h, G) + 4);
    }
    return w;
}

bool bwd_spline_eval_ok(const BsplineGeom &B)
{
    return max_window(B.oz, kBwdTiling.lz, B.inv_hz, B.gz) <= kSplineWindow;
}

bool bwd_ctrl_fused(const BsplineGeom &B)
{
    if (3 * (int64_t)B.gx * B.gy * B.gz > kCtrlMaxEntries)
        return false;
    return bwd_spline_eval_ok(B) &&
           max_window(B.ox, kBwdTiling.lx, B.inv_hx, B.gx) <= kSplineWindow &&
           max_window(B.oy, kBwdTiling.ly, B.inv_hy, B.gy) <= kSplineWindow;
}

// Exponent b of the 32-bit fixed-point image adjoint of an affine job (see
// kFixed32MaxBits), or -1 for the 64-bit one.  Sample p reaches input cell c when
// q(p) = A p + t lies in [c - 1, c + 1) per axis, widened by the bound delta
// on q's FP32 rounding; those p lie in A^-1 of that cube, whose extent along
// output axis i is w_i = (2 + 2 delta) sum_j |A^-1_ij|, which holds at most
// floor(w_i) + 1 integer values of p_i, and the tile at most its extent.  A strongly shrinking or
// near-singular map exceeds kFixed32MaxBits and keeps 64-bit sums.
static int32_t fixed32_bits(const FwdJob &J)
{
    double a[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            a[i][j] = (double)J.M[4 * i + j];
    double c[3][3];                    // cofactors
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            c[i][j] = a[i1][j1] * a[i2][j2] - a[i1][j2] * a[i2][j1];
        }
    const double det = a[0][0] * c[0][0] + a[0][1] * c[0][1] + a[0][2] * c[0][2];
    if (!std::isfinite(det) || det == 0.0)
        return -1;
    const double slack = std::max({(double)J.delta[0], (double)J.delta[1], (double)J.delta[2]});
    const int ext[3] = {1 << kBwdTiling.lx, 1 << kBwdTiling.ly, 1 << kBwdTiling.lz};
    int64_t K = 1;
    for (int i = 0; i < 3; ++i) {      // row i of A^-1 = column i of the cofactors / det
        const double w =
            (2.0 + 2.0 * slack) *
            (std::fabs(c[0][i]) + std::fabs(c[1][i]) + std::fabs(c[2][i])) / std::fabs(det);
        K *= (std::isfinite(w) && w < (double)ext[i])
                 ? std::min<int64_t>(ext[i], (int64_t)std::floor(w) + 1)
                 : ext[i];
    }
    int b = 0;
    while (((int64_t)1 << b) < K)
        ++b;
    return b <= kFixed32MaxBits ? b : -1;
}

// Workgroups the device keeps resident for kernel fn with lds bytes of dynamic
// LDS (occupancy x compute units), cached per device, kernel and LDS size.
static int resident_groups(const void *fn, size_t lds)
{
    // a fixed table (no heap allocation on the call path); when it is full
    // the occupancy is queried again on every call
    struct Entry {
        int dev;
        const void *fn;
        size_t lds;
        int groups;
    };
    constexpr int kEntries = 256;
    static std::mutex mu;
    static Entry cache[kEntries];
    static int used = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 0;
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < used; ++i)
        if (cache[i].dev == dev && cache[i].fn == fn && cache[i].lds == lds)
            return cache[i].groups;
    int cus = 0, occ = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, kThreads, lds) != hipSuccess)
        return 0;
    if (used < kEntries)
        cache[used++] = {dev, fn, lds, cus * occ};
    return cus * occ;
}

// Persistent grid: at most one wave of resident workgroups (a multiple of 8,
// as the XCD tile order assumes), at most the workspace's rows.
static int bwd_launch_grid(const void *fn, size_t lds, int64_t ntiles)
{
    const int64_t rows = bwd_grid(ntiles);
    const int resident = resident_groups(fn, lds) & ~7;
    return (int)(resident >= 8 ? std::min<int64_t>(rows, resident) : rows);
}

template <int DISP>
static int launch_bwd_t(const FwdJob &J, int64_t ntiles, size_t lds, hipStream_t s,
                        const float *g, float *g_img, float *g_disp, double *part,
                        double *ctrl_part, int32_t cells)
{
    const int32_t fix_bits = DISP == kDispNone ? fixed32_bits(J) : -1;
    const int nt = (int)ntiles;
    int grid = 0;
    auto launch = [&](auto kern) {
        grid = bwd_launch_grid(reinterpret_cast<const void *>(kern), lds, ntiles);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, s, J, g, g_img, g_disp, part,
                           ctrl_part, nt, cells, fix_bits);
    };
    if constexpr (DISP == kDispNone) {
        if (fix_bits >= 0) {
            if (J.dtype == kI16)
                launch(&k_warp_bwd<int16_t, DISP, true>);
            else
                launch(&k_warp_bwd<float, DISP, true>);
            return grid;
        }
    }
    if (J.dtype == kI16)
        launch(&k_warp_bwd<int16_t, DISP, false>);
    else
        launch(&k_warp_bwd<float, DISP, false>);
    return grid;
}

hipError_t launch_warp_bwd(const FwdJob &J0, const float *g, float *g_img, float *g_disp,
                           double *g_M, double *partials, double *ctrl_part, float *g_ctrl,
                           hipStream_t s)
{
    FwdJob J = J0;
    J.tiles_x = (J.ox + 7) >> 3;
    J.tiles_y = (J.oy + 7) >> 3;
    J.tiles_z = (J.oz + 15) >> 4;
    const int64_t ntiles = (int64_t)J.tiles_x * J.tiles_y * J.tiles_z;
    const int32_t nctrl = 3 * J.bs.gx * J.bs.gy * J.bs.gz;
    if (ntiles == 0) {
        if (g_ctrl && nctrl > 0) {     // no tiles, no rows: zeros
            hipError_t e = reduce_ctrl(ctrl_part, 0, nctrl, g_ctrl, s);
            if (e != hipSuccess)
                return e;
        }
        if (g_M) {
            hipLaunchKernelGGL(k_reduce12, dim3(1), dim3(kThreads), 0, s, partials, 0, g_M);
            return hipGetLastError();
        }
        return hipSuccess;
    }
    // LDS cells sized for the largest footprint of any tile (a displacement has
    // no a-priori bound: the full reservation, used when a tile fits it)
    const bool displaced = J.disp || J.ctrl;
    const int32_t cells =
        J.ctrl ? kSplineBwdCells
               : displaced ? kBwdLdsCells
                           : std::min(footprint_cells_bound(J, kBwdTiling), kBwdLdsCells);
    const size_t lds = (size_t)(J.ctrl ? kBwdLdsCells : cells) * sizeof(float);
    double *part = g_M ? partials : nullptr;
    double *cpart = g_ctrl ? ctrl_part : nullptr;
    int grid;
    if (J.ctrl)
        grid = launch_bwd_t<kDispSpline>(J, ntiles, lds, s, g, g_img, g_disp, part, cpart, cells);
    else if (J.disp)
        grid = launch_bwd_t<kDispField>(J, ntiles, lds, s, g, g_img, g_disp, part, nullptr, cells);
    else
        grid = launch_bwd_t<kDispNone>(J, ntiles, lds, s, g, g_img, nullptr, part, nullptr, cells);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (cpart) {
        e = reduce_ctrl(cpart, grid, nctrl, g_ctrl, s);
        if (e != hipSuccess)
            return e;
    }
    if (!g_M)
        return hipSuccess;
    hipLaunchKernelGGL(k_reduce12, dim3(1), dim3(kThreads), 0, s, partials, grid, g_M);
    return hipGetLastError();
}

// Batched affine adjoint: chunks of up to kBwdBatchMax jobs, each one
// persistent launch (its job table in the kernel arguments; every workgroup
// writes its partial row of every job, zeros where it met none of the job's
// tiles) and one reduction launch; a chunk with no tiles zeroes its rows in
// a launch of its own.  partials: kBwdMaxRows * 12 doubles per job.
hipError_t launch_warp_bwd_batch(const BwdJob *jobs, int32_t n, double *partials, hipStream_t s)
{
    for (int32_t c0 = 0; c0 < n; c0 += kBwdBatchMax) {
        BwdBatch B;
        std::memset(&B, 0, sizeof B);
        B.njobs = std::min<int32_t>(kBwdBatchMax, n - c0);
        int64_t total = 0;
        int32_t cells = 64;
        bool any_M = false;
        for (int i = 0; i < B.njobs; ++i) {
            B.jobs[i] = jobs[c0 + i];
            FwdJob &J = B.jobs[i].J;
            J.tiles_x = (J.ox + 7) >> 3;
            J.tiles_y = (J.oy + 7) >> 3;
            J.tiles_z = (J.oz + 15) >> 4;
            B.prefix[i] = (int32_t)total;
            B.fix_bits[i] = fixed32_bits(J);
            total += (int64_t)J.tiles_x * J.tiles_y * J.tiles_z;
            if (J.nx > 0 && J.ny > 0 && J.nz > 0 && J.ox > 0 && J.oy > 0 && J.oz > 0)
                cells = std::max(cells, std::min(footprint_cells_bound(J, kBwdTiling), kBwdLdsCells));
            any_M = any_M || B.jobs[i].g_M;
        }
        B.prefix[B.njobs] = (int32_t)total;
        double *part = partials ? partials + (int64_t)c0 * kBwdMaxRows * 12 : nullptr;
        const bool i16 = B.jobs[0].J.dtype == kI16;
        const size_t lds = (size_t)cells * sizeof(float);
        bool narrow = true;            // the 32-bit image adjoint when every job has a bound
        for (int i = 0; i < B.njobs; ++i)
            narrow = narrow && B.fix_bits[i] >= 0;
        using BatchKernel = void (*)(const BwdBatch, double *, int32_t);
        const BatchKernel kern =
            i16 ? (narrow ? &k_warp_bwd_batch<int16_t, true> : &k_warp_bwd_batch<int16_t, false>)
                : (narrow ? &k_warp_bwd_batch<float, true> : &k_warp_bwd_batch<float, false>);
        const int grid =
            total > 0 ? bwd_launch_grid(reinterpret_cast<const void *>(kern), lds, total) : 8;
        if (any_M && total == 0) {     // else the kernel writes every row
            const int64_t nz = (int64_t)B.njobs * grid * 12;
            hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((nz + kThreads - 1) / kThreads)),
                               dim3(kThreads), 0, s, part, nz);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return e;
        }
        if (total > 0) {
            hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, s, B, part, cells);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return e;
        }
        if (any_M) {
            hipLaunchKernelGGL(k_reduce12_batch, dim3(B.njobs), dim3(kThreads), 0, s, B, part,
                               grid);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return e;
        }
    }
    return hipSuccess;
}

}  // namespace ctaug
