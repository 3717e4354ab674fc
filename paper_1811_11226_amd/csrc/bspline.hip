// bspline.hip -- uniform cubic B-spline displacement field and its adjoint
// (gfx950).  Separable evaluation: for an output row (x, y) the x/y weights
// contract the control grid to a row profile P[comp][gz] once (in LDS), and
// each voxel then needs only its 4 z-weights and 12 FMAs.  The adjoint runs
// the same factorisation backwards with fixed-order FP64 reductions, so the
// control-grid gradient is deterministic.
#include "device_common.h"
#include "launch.h"

namespace ctaug {

constexpr int kRowsPerWG = 4;          // upsample: rows (x, y..y+3) per workgroup
constexpr int kAdjRows = 64;           // adjoint: rows per workgroup chunk
constexpr int kMaxG = 64;

struct BsplineGeom {
    int32_t ox, oy, oz;
    int32_t gx, gy, gz;
    float inv_hx, inv_hy, inv_hz;      // (G - 3) / (n - 1), or 0 when n == 1
};

__device__ __forceinline__ void bs_cell(int32_t p, float inv_h, int32_t G, int32_t &i, float &t)
{
    const float s = (float)p * inv_h;
    const float f = fminf(floorf(s), (float)(G - 4));
    i = (int32_t)f;
    t = s - f;
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

__global__ __launch_bounds__(kThreads) void k_bspline_up(const float *__restrict__ ctrl,
                                                         BsplineGeom G, float *__restrict__ disp,
                                                         int vec)
{
    __shared__ float P[kRowsPerWG][3][kMaxG];
    const int x = blockIdx.x;
    const int y0 = blockIdx.y * kRowsPerWG;
    const int64_t nvox = (int64_t)G.ox * G.oy * G.oz;
    const int64_t gstride = (int64_t)G.gx * G.gy * G.gz;

    int32_t ix;
    float tx, Bx[4];
    bs_cell(x, G.inv_hx, G.gx, ix, tx);
    bs_basis(tx, Bx);
    for (int e = threadIdx.x; e < kRowsPerWG * 3 * G.gz; e += kThreads) {
        const int row = e / (3 * G.gz);
        const int rem = e - row * 3 * G.gz;
        const int comp = rem / G.gz, gz = rem - comp * G.gz;
        const int y = min(y0 + row, G.oy - 1);
        int32_t iy;
        float ty, By[4];
        bs_cell(y, G.inv_hy, G.gy, iy, ty);
        bs_basis(ty, By);
        float s = 0.0f;
        for (int a = 0; a < 4; ++a) {
            float sa = 0.0f;
            for (int b = 0; b < 4; ++b)
                sa = __builtin_fmaf(By[b],
                                    ctrl[comp * gstride + ((int64_t)(ix + a) * G.gy + (iy + b)) * G.gz + gz],
                                    sa);
            s = __builtin_fmaf(Bx[a], sa, s);
        }
        P[row][comp][gz] = s;
    }
    __syncthreads();

    const int row = threadIdx.x >> 6;          // 64 threads per row
    const int y = y0 + row;
    if (y >= G.oy)
        return;
    const int64_t rowbase = ((int64_t)x * G.oy + y) * G.oz;
    for (int z = (threadIdx.x & 63) * 4; z < G.oz; z += 256) {
        float u[3][4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int32_t iz;
            float tz, Bz[4];
            bs_cell(min(z + k, G.oz - 1), G.inv_hz, G.gz, iz, tz);
            bs_basis(tz, Bz);
#pragma unroll
            for (int comp = 0; comp < 3; ++comp) {
                float s = 0.0f;
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    s = __builtin_fmaf(Bz[c], P[row][comp][iz + c], s);
                u[comp][k] = s;
            }
        }
        if (vec) {
#pragma unroll
            for (int comp = 0; comp < 3; ++comp)
                *reinterpret_cast<float4 *>(disp + comp * nvox + rowbase + z) =
                    make_float4(u[comp][0], u[comp][1], u[comp][2], u[comp][3]);
        } else {
            for (int k = 0; k < 4; ++k)
                if (z + k < G.oz)
#pragma unroll
                    for (int comp = 0; comp < 3; ++comp)
                        disp[comp * nvox + rowbase + z + k] = u[comp][k];
        }
    }
}

// Adjoint, stage 1: for output plane x and a chunk of kAdjRows rows,
//   R[comp][gy][gz] = sum_{y in chunk} sum_z By_{gy-iy(y)} Bz_{gz-iz(z)} g[comp](x,y,z)
// written in FP64 to ws[x][chunk][comp][gy][gz].
__global__ __launch_bounds__(kThreads) void k_bspline_adj_rows(const float *__restrict__ g,
                                                               BsplineGeom G,
                                                               double *__restrict__ ws,
                                                               int32_t nchunks)
{
    __shared__ float Q[kAdjRows][3][kMaxG];
    const int x = blockIdx.x, chunk = blockIdx.y;
    const int64_t nvox = (int64_t)G.ox * G.oy * G.oz;
    for (int e = threadIdx.x; e < kAdjRows * 3 * kMaxG; e += kThreads)
        (&Q[0][0][0])[e] = 0.0f;
    __syncthreads();

    // Each of the first 3*kAdjRows threads streams one (row, component) along z,
    // accumulating the four weights of the current z-cell and flushing them to
    // Q when the cell index (nondecreasing in z) advances.
    if (threadIdx.x < 3 * kAdjRows) {
        const int row = threadIdx.x % kAdjRows, comp = threadIdx.x / kAdjRows;
        const int y = chunk * kAdjRows + row;
        if (y < G.oy && G.oz > 0) {
            const float *src = g + comp * nvox + ((int64_t)x * G.oy + y) * G.oz;
            float a[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            int32_t cur;
            float t0;
            bs_cell(0, G.inv_hz, G.gz, cur, t0);
            for (int z = 0; z < G.oz; ++z) {
                int32_t iz;
                float tz, Bz[4];
                bs_cell(z, G.inv_hz, G.gz, iz, tz);
                if (iz != cur) {
                    for (int c = 0; c < 4; ++c) {
                        Q[row][comp][cur + c] += a[c];
                        a[c] = 0.0f;
                    }
                    cur = iz;
                }
                bs_basis(tz, Bz);
                const float gv = src[z];
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    a[c] = __builtin_fmaf(Bz[c], gv, a[c]);
            }
            for (int c = 0; c < 4; ++c)
                Q[row][comp][cur + c] += a[c];
        }
    }
    __syncthreads();

    const int ne = 3 * G.gy * G.gz;
    double *dst = ws + ((int64_t)x * nchunks + chunk) * ne;
    for (int e = threadIdx.x; e < ne; e += kThreads) {
        const int comp = e / (G.gy * G.gz);
        const int rem = e - comp * G.gy * G.gz;
        const int gy = rem / G.gz, gz = rem - gy * G.gz;
        double s = 0.0;
        for (int row = 0; row < kAdjRows; ++row) {
            const int y = chunk * kAdjRows + row;
            if (y >= G.oy)
                break;
            int32_t iy;
            float ty, By[4];
            bs_cell(y, G.inv_hy, G.gy, iy, ty);
            const int b = gy - iy;
            if (b < 0 || b > 3)
                continue;
            bs_basis(ty, By);
            s += (double)By[b] * (double)Q[row][comp][gz];
        }
        dst[e] = s;
    }
}

// Adjoint, stage 2: grad_ctrl[comp][gx][gy][gz] = sum_x Bx_{gx-ix(x)} sum_chunk R.
__global__ __launch_bounds__(kThreads) void k_bspline_adj_final(const double *__restrict__ ws,
                                                                BsplineGeom G, int32_t nchunks,
                                                                float *__restrict__ grad_ctrl)
{
    const int ne_plane = 3 * G.gy * G.gz;
    const int total = G.gx * ne_plane;
    for (int e = blockIdx.x * kThreads + threadIdx.x; e < total; e += gridDim.x * kThreads) {
        const int comp = e / (G.gx * G.gy * G.gz);
        const int rem = e - comp * G.gx * G.gy * G.gz;
        const int gx = rem / (G.gy * G.gz);
        const int r2 = rem - gx * G.gy * G.gz;     // gy * Gz + gz
        double s = 0.0;
        for (int x = 0; x < G.ox; ++x) {
            int32_t ix;
            float tx, Bx[4];
            bs_cell(x, G.inv_hx, G.gx, ix, tx);
            const int a = gx - ix;
            if (a < 0 || a > 3)
                continue;
            bs_basis(tx, Bx);
            double r = 0.0;
            for (int c = 0; c < nchunks; ++c)
                r += ws[((int64_t)x * nchunks + c) * ne_plane + comp * G.gy * G.gz + r2];
            s += (double)Bx[a] * r;
        }
        grad_ctrl[e] = (float)s;
    }
}

static BsplineGeom geom(const int64_t G[3], const int64_t od[3])
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

int bspline_max_grid() { return kMaxG; }

int64_t bspline_adj_ws_bytes(const int64_t od[3], const int64_t G[3])
{
    const int64_t nchunks = (od[1] + kAdjRows - 1) / kAdjRows;
    return od[0] * nchunks * 3 * G[1] * G[2] * (int64_t)sizeof(double);
}

hipError_t launch_bspline_up(const float *ctrl, const int64_t G[3], const int64_t od[3],
                             float *disp, bool vec, hipStream_t s)
{
    if (od[0] == 0 || od[1] == 0 || od[2] == 0)
        return hipSuccess;
    const BsplineGeom g = geom(G, od);
    dim3 grid((unsigned)od[0], (unsigned)((od[1] + kRowsPerWG - 1) / kRowsPerWG));
    hipLaunchKernelGGL(k_bspline_up, grid, dim3(kThreads), 0, s, ctrl, g, disp, vec ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_bspline_adj(const float *grad_disp, const int64_t od[3], const int64_t G[3],
                              float *grad_ctrl, double *ws, hipStream_t s)
{
    const BsplineGeom g = geom(G, od);
    const int32_t nchunks = (int32_t)((od[1] + kAdjRows - 1) / kAdjRows);
    if (od[0] > 0 && od[1] > 0 && od[2] > 0) {
        hipLaunchKernelGGL(k_bspline_adj_rows, dim3((unsigned)od[0], (unsigned)nchunks),
                           dim3(kThreads), 0, s, grad_disp, g, ws, nchunks);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    BsplineGeom gf = g;
    if (od[1] == 0 || od[2] == 0)
        gf.ox = 0;                      // no voxels: every control gradient is 0
    const int total = (int)(3 * G[0] * G[1] * G[2]);
    hipLaunchKernelGGL(k_bspline_adj_final, dim3((unsigned)((total + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, ws, gf, nchunks, grad_ctrl);
    return hipGetLastError();
}

}  // namespace ctaug
