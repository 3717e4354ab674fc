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
// Workgroup-to-tile mapping is XCD-aware (xcd_tile): consecutive workgroup
// ids are dispatched round-robin over the 8 XCDs, and tiles are dealt to the
// XCDs in chunks of consecutive tiles, so that each XCD's L2 sees spatially
// coherent runs and every XCD gets a share of every job.
#include "device_common.h"
#include "launch.h"
#include "tile_geom.h"

#include <algorithm>
#include <cmath>

namespace ctaug {

enum : int { kPathOutside, kPathLdsInterior, kPathLdsBoundary, kPathDirectInterior,
             kPathDirectBoundary };

// Sample coordinates of one thread's run, computed once by a displacement
// tile (which needs them to bound its footprint) and reused for sampling.
struct RunQ {
    float q[3][4];
};

// All runs of one tile along one sampling path.  Each thread owns runs of 4
// consecutive output voxels along z.  With a displacement (DISP) the tile has
// exactly one run per thread and its coordinates come precomputed in Q.
template <typename T, typename LT, int PATH, bool ALIGNED, bool LBL, int DISP>
__device__ __forceinline__ void run_tile(const FwdJob &J, const TileGeom &G, const Tiling &SL,
                                         const LT *s_img, const RunQ &Q)
{
    const Src S = make_src<T>(J);
    gmut<float> *out = gm<float>(J.out);
    gmut<int8_t> *lout = gm<int8_t>(J.lout);
    Photo P = photo_of(J);
    const int runs_z_log = SL.lz - 2;
    const int nruns = 1 << (SL.lx + SL.ly + runs_z_log);
    const int pitch = G.pitch, sxy = G.e[1] * G.pitch;
    // LDS cell index of input cell i: (i - lo) . (sxy, pitch, 1), evaluated in
    // FP32 (full-rate FMA) on integer values below 2^24, hence exactly
    const float lo_f[3] = {(float)G.lo[0], (float)G.lo[1], (float)G.lo[2]};
    const float sxy_f = (float)sxy, pitch_f = (float)pitch;
    const int8_t lfill = (int8_t)J.label_fill;

    for (int r = threadIdx.x; r < nruns; r += kThreads) {
        if (DISP != kDispNone && r != (int)threadIdx.x)
            break;
        const int zr = r & ((1 << runs_z_log) - 1);
        const int rr = r >> runs_z_log;
        const int y = G.y0 + (rr & ((1 << SL.ly) - 1));
        const int x = G.x0 + (rr >> SL.ly);
        const int z = G.z0 + 4 * zr;
        if (x > G.x1 || y > G.y1 || z > G.z1)
            continue;
        // The flags are re-read each iteration so that the compiler tests their
        // bits in SALU where they are used instead of keeping one 64-bit lane
        // mask per flag live across the loop (scalar register pressure).
        uint32_t fl = J.flags;
        asm volatile("" : "+s"(fl));
        constexpr bool labels = LBL;      // a template parameter: the 4 voxels of a
                                          // run stay one basic block
        const bool vec = (fl & kFlagVec) != 0;
        P.flags = fl;
        const int nvalid = ALIGNED ? 4 : min(4, J.oz - z);
        const uint32_t v0 = (uint32_t)((x * J.oy + y) * J.oz + z);
        float rb[3];
        row_base(J.M, (float)x, (float)y, rb);

        float V[4];
        int8_t L[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            V[k] = J.fill;
            L[k] = lfill;
            if (PATH == kPathOutside || (!ALIGNED && k >= nvalid))
                continue;
            const float zf = (float)(z + k);
            float qx = coord(J.M, 0, rb, zf), qy = coord(J.M, 1, rb, zf),
                  qz = coord(J.M, 2, rb, zf);
            if (DISP != kDispNone) {
                qx = Q.q[0][k];
                qy = Q.q[1][k];
                qz = Q.q[2][k];
            }
            if (PATH == kPathLdsInterior || PATH == kPathLdsBoundary) {
                // A boundary tile samples without branches: a sample outside the
                // guard is moved to the footprint's first cell pair (lo .. lo + 1
                // on each axis, inside every footprint of a box that is not
                // outside, as box_geom and geom_from_cells make e >= 2), and its
                // results are replaced by fill / label_fill below.
                // labels straight from global memory: an interior tile's
                // nearest voxel is inside the volume
                if (labels)
                    L[k] = PATH == kPathLdsInterior ? label_interior(S, qx, qy, qz)
                                                    : label_checked(S, qx, qy, qz, lfill);
                bool guarded = true;
                if (PATH == kPathLdsBoundary) {
                    guarded = in_guard(qx, qy, qz, J.nx, J.ny, J.nz);
                    qx = guarded ? qx : lo_f[0] + 0.25f;
                    qy = guarded ? qy : lo_f[1] + 0.25f;
                    qz = guarded ? qz : lo_f[2] + 0.25f;
                }
                const float fx = floorf(qx), fy = floorf(qy), fz = floorf(qz);
                const int base = (int)__builtin_fmaf(
                    fx - lo_f[0], sxy_f, __builtin_fmaf(fy - lo_f[1], pitch_f, fz - lo_f[2]));
                float kk[8];
                kk[0] = (float)s_img[base];
                kk[1] = (float)s_img[base + 1];
                kk[2] = (float)s_img[base + pitch];
                kk[3] = (float)s_img[base + pitch + 1];
                kk[4] = (float)s_img[base + sxy];
                kk[5] = (float)s_img[base + sxy + 1];
                kk[6] = (float)s_img[base + sxy + pitch];
                kk[7] = (float)s_img[base + sxy + pitch + 1];
                V[k] = tri(kk, qx - fx, qy - fy, qz - fz);
                if (PATH == kPathLdsBoundary)
                    V[k] = guarded ? V[k] : J.fill;
            } else {
                if (PATH == kPathDirectInterior) {
                    V[k] = sample_interior<T>(S, qx, qy, qz);
                    if (labels)
                        L[k] = label_interior(S, qx, qy, qz);
                } else {
                    V[k] = sample_checked<T>(S, qx, qy, qz, J.fill);
                    if (labels)
                        L[k] = label_checked(S, qx, qy, qz, lfill);
                }
            }
        }

        if (fl & kFlagOcclude) {
            // I_occ: the occluded output slab is 0 in place of the warped image
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float zf = (float)(z + k);
                if (zf >= J.occ_lo && zf <= J.occ_hi)
                    V[k] = 0.0f;
            }
        }

        if (P.flags & kFlagPhoto) {
            float n[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (P.flags & kFlagNoise) {
                if (ALIGNED)
                    gauss_group((uint64_t)(v0 >> 2), J.vol_id, J.key0, J.key1, n);
                else
                    gauss_run((uint64_t)v0, J.vol_id, J.key0, J.key1, n);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                V[k] = photometric(P, V[k], n[k]);
        }

        if (ALIGNED && vec) {
            *reinterpret_cast<gmut<f32x4> *>(out + v0) = f32x4{V[0], V[1], V[2], V[3]};
            if (labels) {
                const uint32_t packed = (uint32_t)(uint8_t)L[0] | ((uint32_t)(uint8_t)L[1] << 8) |
                                        ((uint32_t)(uint8_t)L[2] << 16) |
                                        ((uint32_t)(uint8_t)L[3] << 24);
                *reinterpret_cast<gmut<uint32_t> *>(lout + v0) = packed;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k < nvalid) {
                    out[v0 + k] = V[k];
                    if (labels)
                        lout[v0 + k] = L[k];
                }
        }
    }
}

// ALIGNED: the output z extent is a multiple of 4, so every run is one noise
// group and (with 16-byte aligned outputs) one vector store.  LT: type of the
// LDS footprint cells (FP32, or int16 for int16 inputs: half the LDS, twice
// the LDS reads).
template <typename T, typename LT, bool ALIGNED, bool LBL, int DISP>
__device__ __forceinline__ void fwd_box_l(const FwdJob &J, const TileGeom &G, const Tiling &SL,
                                         uint8_t *s_lds, int32_t lds_cells, const RunQ &Q)
{
    LT *s_img = reinterpret_cast<LT *>(s_lds);
    if (G.cls == kOutside) {
        run_tile<T, LT, kPathOutside, ALIGNED, LBL, DISP>(J, G, SL, s_img, Q);
    } else if (G.lds) {
        stage_footprint<T, LT>(J, make_src<T>(J), G, s_img);
        __syncthreads();
        if (G.cls == kInterior)
            run_tile<T, LT, kPathLdsInterior, ALIGNED, LBL, DISP>(J, G, SL, s_img, Q);
        else
            run_tile<T, LT, kPathLdsBoundary, ALIGNED, LBL, DISP>(J, G, SL, s_img, Q);
        __syncthreads();               // LDS is reused by the next box
    } else if (G.cls == kInterior) {
        run_tile<T, LT, kPathDirectInterior, ALIGNED, LBL, DISP>(J, G, SL, s_img, Q);
    } else {
        run_tile<T, LT, kPathDirectBoundary, ALIGNED, LBL, DISP>(J, G, SL, s_img, Q);
    }
}

template <typename T, typename LT, bool ALIGNED, int DISP>
__device__ __forceinline__ void fwd_box(const FwdJob &J, const TileGeom &G, const Tiling &SL,
                                       uint8_t *s_lds, int32_t lds_cells, const RunQ &Q)
{
    if (J.flags & kFlagLabels)
        fwd_box_l<T, LT, ALIGNED, true, DISP>(J, G, SL, s_lds, lds_cells, Q);
    else
        fwd_box_l<T, LT, ALIGNED, false, DISP>(J, G, SL, s_lds, lds_cells, Q);
}

// One output tile, processed as sub-tiles of the job's sub-tile shape (the
// whole tile unless its input footprint would not fit the LDS reservation).
// ALIGNED: the output z extent is a multiple of 4, so every run is one noise
// group and (with 16-byte aligned outputs) one vector store.  LT: type of the
// LDS footprint cells (FP32, or int16 for int16 inputs: half the LDS, twice
// the LDS reads).
template <typename T, typename LT, bool ALIGNED, int DISP>
__device__ __forceinline__ void fwd_tile_lt(const FwdJob &J, int t, const Tiling &TL,
                                            int32_t lds_cells, uint8_t *s_lds)
{
    const int tz = t % J.tiles_z;
    const int rest = t / J.tiles_z;
    const int ty = rest % J.tiles_y;
    const int tx = rest / J.tiles_y;
    const int x0 = tx << TL.lx, y0 = ty << TL.ly, z0 = tz << TL.lz;
    const int x1 = min(x0 + (1 << TL.lx), J.ox) - 1;
    const int y1 = min(y0 + (1 << TL.ly), J.oy) - 1;
    const int z1 = min(z0 + (1 << TL.lz), J.oz) - 1;
    const Tiling SL = {J.sub[0], J.sub[1], J.sub[2]};
    if (DISP != kDispNone) {
        // A displacement has no a-priori footprint bound: the tile (one run of
        // 4 z voxels per thread) computes its coordinates once, reduces floor(q)
        // over its guarded samples, and stages that footprint when it fits the
        // reservation.
        __shared__ int s_red[kThreads / 64][6];
        const int zr = threadIdx.x & ((1 << (TL.lz - 2)) - 1);
        const int rr = threadIdx.x >> (TL.lz - 2);
        const int x = x0 + (rr >> TL.ly), y = y0 + (rr & ((1 << TL.ly) - 1)), z = z0 + 4 * zr;
        const bool mine = x <= x1 && y <= y1 && z <= z1;
        const int nvalid = min(4, J.oz - z);
        float u[3][4];
        if (DISP == kDispSpline)
            spline_tile_u<kThreads>(J.ctrl, J.bs, TL.lx, TL.ly, x0, y0, z0, x1, y1, z1, rr, x, y,
                                    z, 1, nvalid, mine, reinterpret_cast<float *>(s_lds), u);
        RunQ Q;
        int fmn[3] = {INT_MAX, INT_MAX, INT_MAX}, fmx[3] = {INT_MIN, INT_MIN, INT_MIN};
        if (mine) {
            gconst<float> *disp = gc<float>(J.disp);
            const int32_t nvox = J.ox * J.oy * J.oz;
            const int32_t v0 = (x * J.oy + y) * J.oz + z;
            const bool any_in = J.nx > 0 && J.ny > 0 && J.nz > 0;
            float rb[3];
            row_base(J.M, (float)x, (float)y, rb);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k >= nvalid)
                    break;
                const float zf = (float)(z + k);
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    Q.q[i][k] = coord(J.M, i, rb, zf) +
                                (DISP == kDispField ? disp[i * nvox + v0 + k] : u[i][k]);
                if (!any_in || !in_guard(Q.q[0][k], Q.q[1][k], Q.q[2][k], J.nx, J.ny, J.nz))
                    continue;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const int f = (int)floorf(Q.q[i][k]);
                    fmn[i] = min(fmn[i], f);
                    fmx[i] = max(fmx[i], f);
                }
            }
        }
        block_minmax3(fmn, fmx, s_red);
        TileGeom G = geom_from_cells(J, x0, y0, z0, x1, y1, z1, fmn, fmx, lds_cells);
        if (G.lds && (J.flags & kFlagLds16) && !(J.flags & kFlagFillInT))
            G.lds = false;             // an int16 footprint must hold fill exactly
        fwd_box<T, LT, ALIGNED, DISP>(J, G, TL, s_lds, lds_cells, Q);
        return;
    }
    const RunQ Q0{};
    const int nz = ((z1 - z0) >> SL.lz) + 1, ny = ((y1 - y0) >> SL.ly) + 1,
              nx = ((x1 - x0) >> SL.lx) + 1;
    const int nsub = nx * ny * nz;     // sub-boxes, x-major
    auto geom = [&](int i) {
        const int iz = i % nz, r = i / nz, iy = r % ny, ix = r / ny;
        const int sx = x0 + (ix << SL.lx), sy = y0 + (iy << SL.ly), sz = z0 + (iz << SL.lz);
        return box_geom(J, sx, sy, sz, min(sx + (1 << SL.lx) - 1, x1),
                        min(sy + (1 << SL.ly) - 1, y1), min(sz + (1 << SL.lz) - 1, z1),
                        lds_cells);
    };
    // the geometry of every sub-box at once, sub-box i in lane i of each wave
    // (one dependent chain per tile instead of one per box), read per box;
    // choose_subtile keeps a tile at no more than 16 sub-boxes
    __builtin_assume(nsub <= 64);
    const TileGeom Gl = geom(min((int)(threadIdx.x & 63), nsub - 1));
    for (int i = 0; i < nsub; ++i) {
        TileGeom G;
        G.x0 = __builtin_amdgcn_readlane(Gl.x0, i);
        G.y0 = __builtin_amdgcn_readlane(Gl.y0, i);
        G.z0 = __builtin_amdgcn_readlane(Gl.z0, i);
        G.x1 = __builtin_amdgcn_readlane(Gl.x1, i);
        G.y1 = __builtin_amdgcn_readlane(Gl.y1, i);
        G.z1 = __builtin_amdgcn_readlane(Gl.z1, i);
        G.cls = __builtin_amdgcn_readlane(Gl.cls, i);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            G.lo[a] = __builtin_amdgcn_readlane(Gl.lo[a], i);
            G.e[a] = __builtin_amdgcn_readlane(Gl.e[a], i);
        }
        G.quads = __builtin_amdgcn_readlane(Gl.quads, i);
        G.pitch = __builtin_amdgcn_readlane(Gl.pitch, i);
        G.lds = __builtin_amdgcn_readlane((int)Gl.lds, i) != 0;
        fwd_box<T, LT, ALIGNED, kDispNone>(J, G, SL, s_lds, lds_cells, Q0);
    }
}

template <typename T, bool ALIGNED, int DISP>
__device__ __forceinline__ void fwd_tile(const FwdJob &J, int t, const Tiling &TL,
                                         int32_t lds_cells, uint8_t *s_lds)
{
    if (sizeof(T) == 2 && (J.flags & kFlagLds16))
        fwd_tile_lt<T, T, ALIGNED, DISP>(J, t, TL, lds_cells, s_lds);
    else
        fwd_tile_lt<T, float, ALIGNED, DISP>(J, t, TL, lds_cells, s_lds);
}

// Dynamic LDS: lds_cells input-type cells of image footprint (rounded up to
// 16 bytes); labels are gathered from global memory.
extern __shared__ __attribute__((aligned(16))) uint8_t s_footprint[];

// Single job, job in kernel arguments, one workgroup per tile.
template <typename T, bool ALIGNED, int DISP>
__global__ __launch_bounds__(kThreads) void k_warp_single(FwdJob J, Tiling TL, int32_t ntiles,
                                                          int32_t lds_cells)
{
    const int b = blockIdx.x;
    const int t = xcd_tile(b & 7, b >> 3);
    if (t >= ntiles)
        return;
    fwd_tile<T, ALIGNED, DISP>(J, t, TL, lds_cells, s_footprint);
}

// Index of the job holding global tile t: the number of i in [1, njobs) with
// prefix[i] <= t (the prefix is nondecreasing), 64 entries per step with one
// vector load and a ballot, so that a workgroup finds its job in one memory
// round trip (for up to 64 jobs) rather than one per job passed over.  The
// count is the same on every lane; it is returned as a scalar.
__device__ __forceinline__ int job_of(const int32_t *__restrict__ prefix, int njobs, int t)
{
    int j = 0;
    const int lane = threadIdx.x & 63;
    for (int base = 1; base < njobs; base += 64) {
        const int i = base + lane;
        const bool le = i < njobs && prefix[i] <= t;
        j += __popcll(__ballot(le));
    }
    return __builtin_amdgcn_readfirstlane(j);
}

// Batch of jobs from a device table.  prefix[j] = first global tile of job j,
// prefix[njobs] = total.  Workgroups stride over the tiles of their XCD
// (xcd_tile; persistent when gridDim.x is a few per CU).  MODE fixes
// the input and LDS cell types when every job shares them (fewer code paths
// in the kernel, less register pressure); kBatchMixed dispatches per job.
template <bool ALIGNED, int MODE>
__global__ __launch_bounds__(kThreads) void k_warp_batch(const FwdJob *__restrict__ jobs,
                                                         const int32_t *__restrict__ prefix,
                                                         int32_t njobs, Tiling TL,
                                                         int32_t lds_cells)
{
    const int total = prefix[njobs];
    const int b = blockIdx.x;
    const int per_xcd_wg = gridDim.x >> 3;
    const int xcd = b & 7;
    for (int i = b >> 3;; i += per_xcd_wg) {
        const int t = xcd_tile(xcd, i);
        if (t >= total)
            break;
        const int j = job_of(prefix, njobs, t);
        const FwdJob J = jobs[j];
        const int lt = t - prefix[j];
        if constexpr (MODE == kBatchSplineI16) {
            fwd_tile_lt<int16_t, float, ALIGNED, kDispSpline>(J, lt, TL, lds_cells, s_footprint);
        } else if constexpr (MODE == kBatchSplineF32) {
            fwd_tile_lt<float, float, ALIGNED, kDispSpline>(J, lt, TL, lds_cells, s_footprint);
        } else if constexpr (MODE == kBatchSplineMixed) {
            if (J.dtype == kI16)
                fwd_tile_lt<int16_t, float, ALIGNED, kDispSpline>(J, lt, TL, lds_cells, s_footprint);
            else
                fwd_tile_lt<float, float, ALIGNED, kDispSpline>(J, lt, TL, lds_cells, s_footprint);
        } else if constexpr (MODE == kBatchI16F32) {
            fwd_tile_lt<int16_t, float, ALIGNED, kDispNone>(J, lt, TL, lds_cells, s_footprint);
        } else if constexpr (MODE == kBatchI16I16) {
            fwd_tile_lt<int16_t, int16_t, ALIGNED, kDispNone>(J, lt, TL, lds_cells, s_footprint);
        } else if constexpr (MODE == kBatchF32) {
            fwd_tile_lt<float, float, ALIGNED, kDispNone>(J, lt, TL, lds_cells, s_footprint);
        } else {
            if (J.dtype == kI16)
                fwd_tile<int16_t, ALIGNED, kDispNone>(J, lt, TL, lds_cells, s_footprint);
            else
                fwd_tile<float, ALIGNED, kDispNone>(J, lt, TL, lds_cells, s_footprint);
        }
    }
}

// Upper bound on the footprint cells of any tile of job J (see box_geom).
int32_t footprint_cells_bound(const FwdJob &J, const Tiling &TL)
{
    const int t[3] = {1 << TL.lx, 1 << TL.ly, 1 << TL.lz};
    const int n[3] = {J.nx, J.ny, J.nz};
    int64_t cells = 1;
    for (int i = 0; i < 3; ++i) {
        double span = 2.0 * (double)J.delta[i];
        for (int j = 0; j < 3; ++j)
            span += std::fabs((double)J.M[4 * i + j]) * (double)(t[j] - 1);
        int64_t e = std::min<int64_t>((int64_t)std::floor(span) + 3, (int64_t)n[i] + 2);
        e = std::max<int64_t>(e, 1);
        if (i == 2)
            e = lds_pitch((int32_t)e);       // LDS row pitch
        cells *= e;
        if (cells > (int64_t)1 << 30)
            return 1 << 30;
    }
    return (int32_t)cells;
}

// Sub-tile shape of job J for tile TL and an LDS reservation of lds_cells
// cells: the whole tile when its footprint bound fits; otherwise the sub-box
// of the tile with the most voxels (at least 2^10, or the tile's own count if
// smaller; z extent >= 4) whose bound fits, fewest cells per voxel among
// equals; the whole tile (direct gathers) when none fits.  As tiles hold at
// most 2^14 voxels, a tile has at most 16 sub-tiles (the kernels read one
// sub-tile's geometry per lane of a wave).
Tiling choose_subtile(const FwdJob &J, const Tiling &TL, int32_t lds_cells)
{
    if (J.disp || J.ctrl || lds_cells <= 0 || footprint_cells_bound(J, TL) <= lds_cells)
        return TL;
    const int min_log = std::min(10, TL.lx + TL.ly + TL.lz);
    Tiling best = TL;
    int best_log = -1;
    double best_ratio = 0.0;
    for (int a = 0; a <= TL.lx; ++a)
        for (int b = 0; b <= TL.ly; ++b)
            for (int c = 2; c <= TL.lz; ++c) {
                if (a + b + c < min_log)
                    continue;
                const Tiling S = {a, b, c};
                const int32_t cells = footprint_cells_bound(J, S);
                if (cells > lds_cells)
                    continue;
                const double ratio = (double)cells / (double)(1 << (a + b + c));
                if (a + b + c > best_log || (a + b + c == best_log && ratio < best_ratio)) {
                    best = S;
                    best_log = a + b + c;
                    best_ratio = ratio;
                }
            }
    return best;
}

int32_t lds_cells_cap(int32_t elem_bytes)
{
    return (kMaxLdsBytes - 16) / elem_bytes & ~15;
}

int32_t lds_cells_for(int32_t bound, int32_t elem_bytes)
{
    return std::min(bound, lds_cells_cap(elem_bytes));
}

size_t lds_bytes_for(int32_t cells, int32_t elem_bytes)
{
    return ((size_t)cells * (size_t)elem_bytes + 15) & ~(size_t)15;
}

template <int DISP>
static void launch_single_t(const FwdJob &J, const Tiling &TL, int ntiles, int32_t cells, int grid,
                            size_t lds, bool aligned, hipStream_t s)
{
    if (J.dtype == kI16) {
        if (aligned)
            hipLaunchKernelGGL((k_warp_single<int16_t, true, DISP>), dim3(grid), dim3(kThreads), lds,
                               s, J, TL, ntiles, cells);
        else
            hipLaunchKernelGGL((k_warp_single<int16_t, false, DISP>), dim3(grid), dim3(kThreads),
                               lds, s, J, TL, ntiles, cells);
    } else {
        if (aligned)
            hipLaunchKernelGGL((k_warp_single<float, true, DISP>), dim3(grid), dim3(kThreads), lds,
                               s, J, TL, ntiles, cells);
        else
            hipLaunchKernelGGL((k_warp_single<float, false, DISP>), dim3(grid), dim3(kThreads), lds,
                               s, J, TL, ntiles, cells);
    }
}

static_assert(1 << (3 + 3 + 4 - 2) == kThreads, "one run of a displacement tile per thread");
static_assert(2 * kDispLdsCells >= kSplineTileLdsFloats * (int32_t)sizeof(float),
              "the B-spline scratch of a tile fits its smallest footprint reservation");

// Labels alone: one thread per run of 4 output voxels along z (one packed
// 4-byte store with kFlagVec), the coordinate and the nearest-neighbour gather
// of the fused warps (row_base, coord, label_checked), so the labels equal
// theirs bit for bit.  Block row blockIdx.y is the x-slab x = x0 + blockIdx.y;
// within it run r covers z = 4 (r mod runs_z) .. + 3 of y = r / runs_z.
__global__ __launch_bounds__(kThreads) void k_warp_labels(FwdJob J, int32_t runs_z, int32_t x0)
{
    const int r = blockIdx.x * kThreads + threadIdx.x;
    if (r >= J.oy * runs_z)
        return;
    const int x = x0 + (int)blockIdx.y;
    const int y = r / runs_z;
    const int z = 4 * (r - y * runs_z);
    const int32_t row = x * J.oy + y;
    Src S;
    S.lbl = make_rsrc(J.lbl, (uint32_t)J.in_extent);
    S.img = S.lbl;                     // not read
    S.nx = J.nx;
    S.ny = J.ny;
    S.nz = J.nz;
    S.ry = J.in_ry;
    S.rsy = J.in_sy;
    S.sy = S.sx = S.sxy = 0;
    const int8_t lfill = (int8_t)J.label_fill;
    const bool any_in = J.nx > 0 && J.ny > 0 && J.nz > 0;
    float rb[3];
    row_base(J.M, (float)x, (float)y, rb);
    int8_t L[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        L[k] = lfill;
        if (!any_in || z + k >= J.oz)
            continue;
        const float zf = (float)(z + k);
        L[k] = label_checked(S, coord(J.M, 0, rb, zf), coord(J.M, 1, rb, zf),
                             coord(J.M, 2, rb, zf), lfill);
    }
    gmut<int8_t> *lout = gm<int8_t>(J.lout);
    const uint32_t v0 = (uint32_t)row * (uint32_t)J.oz + (uint32_t)z;
    if (J.flags & kFlagVec) {
        *reinterpret_cast<gmut<uint32_t> *>(lout + v0) =
            (uint32_t)(uint8_t)L[0] | ((uint32_t)(uint8_t)L[1] << 8) |
            ((uint32_t)(uint8_t)L[2] << 16) | ((uint32_t)(uint8_t)L[3] << 24);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (z + k < J.oz)
                lout[v0 + k] = L[k];
    }
}

hipError_t launch_warp_labels(const FwdJob &J, hipStream_t s)
{
    const int32_t runs_z = (J.oz + 3) >> 2;
    const int64_t slab = (int64_t)J.oy * runs_z;     // runs per x-slab (< 2^31)
    if (slab == 0 || J.ox == 0)
        return hipSuccess;
    const unsigned bx = (unsigned)((slab + kThreads - 1) / kThreads);
    for (int32_t x0 = 0; x0 < J.ox; x0 += 65535) {   // grid y: at most 65535 slabs a launch
        const unsigned nx = (unsigned)std::min<int32_t>(65535, J.ox - x0);
        hipLaunchKernelGGL(k_warp_labels, dim3(bx, nx), dim3(kThreads), 0, s, J, runs_z, x0);
    }
    return hipGetLastError();
}

hipError_t launch_warp_single(const FwdJob &J0, const Tiling &TL0, hipStream_t s)
{
    FwdJob Js = J0;
    const bool displaced = J0.disp || J0.ctrl;
    const Tiling TL = displaced ? kDispTiling : TL0;
    Js.tiles_x = (Js.ox + (1 << TL.lx) - 1) >> TL.lx;
    Js.tiles_y = (Js.oy + (1 << TL.ly) - 1) >> TL.ly;
    Js.tiles_z = (Js.oz + (1 << TL.lz) - 1) >> TL.lz;
    const FwdJob &J = Js;
    const int ntiles = J.tiles_x * J.tiles_y * J.tiles_z;
    if (ntiles == 0)
        return hipSuccess;
    const int grid = 8 * xcd_slots(ntiles);
    const int32_t esz = (J.flags & kFlagLds16) ? 2 : 4;
    const int32_t cells = displaced ? lds_cells_for(kDispLdsCells, esz)
                                 : lds_cells_for(footprint_cells_bound(J, TL), esz);
    const size_t lds = lds_bytes_for(cells, esz);
    const bool aligned = J.oz % 4 == 0;
    const Tiling SL = choose_subtile(J, TL, cells);
    Js.sub[0] = SL.lx;
    Js.sub[1] = SL.ly;
    Js.sub[2] = SL.lz;
    if (J.ctrl)
        launch_single_t<kDispSpline>(Js, TL, ntiles, cells, grid, lds, aligned, s);
    else if (J.disp)
        launch_single_t<kDispField>(Js, TL, ntiles, cells, grid, lds, aligned, s);
    else
        launch_single_t<kDispNone>(Js, TL, ntiles, cells, grid, lds, aligned, s);
    return hipGetLastError();
}

template <bool ALIGNED>
static void launch_batch_mode(int mode, const FwdJob *jobs_dev, const int32_t *prefix_dev,
                              int32_t njobs, int32_t grid, const Tiling &TL, int32_t lds_cells,
                              size_t lds, hipStream_t s)
{
    switch (mode) {
    case kBatchI16F32:
        hipLaunchKernelGGL((k_warp_batch<ALIGNED, kBatchI16F32>), dim3(grid), dim3(kThreads), lds,
                           s, jobs_dev, prefix_dev, njobs, TL, lds_cells);
        break;
    case kBatchI16I16:
        hipLaunchKernelGGL((k_warp_batch<ALIGNED, kBatchI16I16>), dim3(grid), dim3(kThreads), lds,
                           s, jobs_dev, prefix_dev, njobs, TL, lds_cells);
        break;
    case kBatchF32:
        hipLaunchKernelGGL((k_warp_batch<ALIGNED, kBatchF32>), dim3(grid), dim3(kThreads), lds, s,
                           jobs_dev, prefix_dev, njobs, TL, lds_cells);
        break;
    case kBatchSplineI16:
        hipLaunchKernelGGL((k_warp_batch<ALIGNED, kBatchSplineI16>), dim3(grid), dim3(kThreads),
                           lds, s, jobs_dev, prefix_dev, njobs, TL, lds_cells);
        break;
    case kBatchSplineF32:
        hipLaunchKernelGGL((k_warp_batch<ALIGNED, kBatchSplineF32>), dim3(grid), dim3(kThreads),
                           lds, s, jobs_dev, prefix_dev, njobs, TL, lds_cells);
        break;
    case kBatchSplineMixed:
        hipLaunchKernelGGL((k_warp_batch<ALIGNED, kBatchSplineMixed>), dim3(grid), dim3(kThreads),
                           lds, s, jobs_dev, prefix_dev, njobs, TL, lds_cells);
        break;
    default:
        hipLaunchKernelGGL((k_warp_batch<ALIGNED, kBatchMixed>), dim3(grid), dim3(kThreads), lds,
                           s, jobs_dev, prefix_dev, njobs, TL, lds_cells);
    }
}

hipError_t launch_warp_batch(const FwdJob *jobs_dev, const int32_t *prefix_dev, int32_t njobs,
                             int32_t total_tiles, int32_t grid, const Tiling &TL,
                             int32_t lds_cells, int32_t elem_bytes, int mode, bool aligned,
                             hipStream_t s)
{
    if (total_tiles == 0 || njobs == 0)
        return hipSuccess;
    const size_t lds = lds_bytes_for(lds_cells, elem_bytes);
    if (aligned)
        launch_batch_mode<true>(mode, jobs_dev, prefix_dev, njobs, grid, TL, lds_cells, lds, s);
    else
        launch_batch_mode<false>(mode, jobs_dev, prefix_dev, njobs, grid, TL, lds_cells, lds, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Standalone photometric pass (in place) and raw noise generator.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_photometric(float *data, int64_t n, int64_t nz,
                                                          Photo P, float occ_lo, float occ_hi,
                                                          uint32_t vol, uint32_t k0, uint32_t k1,
                                                          int vec)
{
    const int64_t ngroups = (n + 3) >> 2;
    for (int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x; g < ngroups;
         g += (int64_t)gridDim.x * kThreads) {
        const int64_t v0 = g << 2;
        float nzs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (P.flags & kFlagNoise)
            gauss_group((uint64_t)g, vol, k0, k1, nzs);
        float x[4];
        if (vec) {
            const f32x4 w = *reinterpret_cast<const f32x4 *>(data + v0);
            x[0] = w.x;
            x[1] = w.y;
            x[2] = w.z;
            x[3] = w.w;
        } else {
            for (int k = 0; k < 4; ++k)
                x[k] = v0 + k < n ? data[v0 + k] : 0.0f;
        }
        if (P.flags & kFlagOcclude) {
            const int64_t z0 = v0 % nz;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float zf = (float)((z0 + k) % nz);
                if (zf >= occ_lo && zf <= occ_hi)
                    x[k] = 0.0f;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            x[k] = photometric(P, x[k], nzs[k]);
        if (vec) {
            *reinterpret_cast<f32x4 *>(data + v0) = f32x4{x[0], x[1], x[2], x[3]};
        } else {
            for (int k = 0; k < 4; ++k)
                if (v0 + k < n)
                    data[v0 + k] = x[k];
        }
    }
}

hipError_t launch_photometric(float *data, int64_t n, int64_t nz, const Photo &P, float occ_lo,
                              float occ_hi, uint32_t vol, uint32_t k0, uint32_t k1, bool vec,
                              hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const int64_t ngroups = (n + 3) >> 2;
    const int64_t blocks = std::min<int64_t>((ngroups + kThreads - 1) / kThreads, 256 * 64);
    hipLaunchKernelGGL(k_photometric, dim3((unsigned)blocks), dim3(kThreads), 0, s, data, n, nz, P,
                       occ_lo, occ_hi, vol, k0, k1, vec ? 1 : 0);
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

__global__ __launch_bounds__(kThreads) void k_box_muller(const uint32_t *__restrict__ w,
                                                         int64_t npairs, float *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < npairs;
         i += (int64_t)gridDim.x * kThreads) {
        float c, sn;
        box_muller(w[2 * i], w[2 * i + 1], c, sn);
        out[2 * i] = c;
        out[2 * i + 1] = sn;
    }
}

hipError_t launch_box_muller(const uint32_t *words, int64_t npairs, float *out, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>((npairs + kThreads - 1) / kThreads, 256 * 64);
    hipLaunchKernelGGL(k_box_muller, dim3((unsigned)blocks), dim3(kThreads), 0, s, words, npairs,
                       out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Plain streaming copy (measurement reference and cache eviction).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kThreads) void k_copy16(const float4 *__restrict__ src,
                                                     float4 *__restrict__ dst, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads)
        dst[i] = src[i];
}

__global__ __launch_bounds__(kThreads) void k_copy1(const uint8_t *__restrict__ src,
                                                    uint8_t *__restrict__ dst, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads)
        dst[i] = src[i];
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s)
{
    const bool aligned = ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst) |
                           bytes) & 15u) == 0;
    if (aligned) {
        const int64_t n = (int64_t)(bytes / 16);
        const int64_t blocks = std::min<int64_t>((n + kThreads - 1) / kThreads, 256 * 16);
        hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(kThreads), 0, s,
                           static_cast<const float4 *>(src), static_cast<float4 *>(dst), n);
    } else {
        const int64_t n = (int64_t)bytes;
        const int64_t blocks = std::min<int64_t>((n + kThreads - 1) / kThreads, 256 * 16);
        hipLaunchKernelGGL(k_copy1, dim3((unsigned)blocks), dim3(kThreads), 0, s,
                           static_cast<const uint8_t *>(src), static_cast<uint8_t *>(dst), n);
    }
    return hipGetLastError();
}

}  // namespace ctaug
