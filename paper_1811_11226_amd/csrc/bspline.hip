// bspline.hip -- uniform cubic B-spline displacement field and its adjoint
// (gfx950).  Separable evaluation: for an output row (x, y) the x/y weights
// contract the control grid to a row profile P[comp][gz] once (in LDS), and
// each voxel then needs only its 4 z-weights and 12 FMAs.  The adjoint runs
// the same factorisation backwards, one axis per pass (z in FP32 per row,
// then y and x in FP64, each in a fixed order), so the control-grid gradient
// is deterministic.
#include "bspline_eval.h"
#include "device_common.h"
#include "launch.h"

namespace ctaug {

constexpr int kRowsPerWG = 4;          // upsample: rows (x, y..y+3) per workgroup
constexpr int kMaxG = 64;

__global__ __launch_bounds__(kThreads) void k_bspline_up(const float *__restrict__ ctrl,
                                                         BsplineGeom G, float *__restrict__ disp,
                                                         int vec)
{
    __shared__ float P[kRowsPerWG][3][kMaxG];
    const int x = blockIdx.x;
    const int y0 = blockIdx.y * kRowsPerWG;
    const int64_t nvox = (int64_t)G.ox * G.oy * G.oz;

    for (int e = threadIdx.x; e < kRowsPerWG * 3 * G.gz; e += kThreads) {
        const int row = e / (3 * G.gz);
        const int rem = e - row * 3 * G.gz;
        const int comp = rem / G.gz, gz = rem - comp * G.gz;
        const int y = min(y0 + row, G.oy - 1);
        P[row][comp][gz] = bs_profile(ctrl, G, comp, x, y, gz);
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

// Adjoint, pass 1 (z): T1[comp][x][y][gz] = sum_z B_{gz - iz(z)}(t(z)) g[comp][x][y][z],
// one thread per (comp, x, y) row streaming z with 16-byte loads when the
// rows are aligned.  The z-cell index is nondecreasing along the row, so the
// four controls a voxel touches slide as a window of four FP32 accumulators;
// each control's sum is stored once, when the window moves past it.
__global__ __launch_bounds__(kThreads) void k_bspline_adj_z(const float *__restrict__ g,
                                                            BsplineGeom G, float *__restrict__ T1,
                                                            int vec)
{
    const int64_t nrows = 3 * (int64_t)G.ox * G.oy;
    const int64_t row = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (row >= nrows)
        return;
    const float *src = g + row * G.oz;
    float *dst = T1 + row * G.gz;
    float w[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    int32_t cur = 0;
    auto add = [&](int z, float v) {
        int32_t iz;
        float tz, Bz[4];
        bs_cell(z, G.inv_hz, G.gz, iz, tz);
        while (cur < iz) {             // controls below iz are complete
            dst[cur] = w[0];
            w[0] = w[1];
            w[1] = w[2];
            w[2] = w[3];
            w[3] = 0.0f;
            ++cur;
        }
        bs_basis(tz, Bz);
#pragma unroll
        for (int c = 0; c < 4; ++c)
            w[c] = __builtin_fmaf(Bz[c], v, w[c]);
    };
    if (vec) {
        for (int z = 0; z < G.oz; z += 4) {
            const f32x4 v = *reinterpret_cast<const f32x4 *>(src + z);
            add(z, v.x);
            add(z + 1, v.y);
            add(z + 2, v.z);
            add(z + 3, v.w);
        }
    } else {
        for (int z = 0; z < G.oz; ++z)
            add(z, src[z]);
    }
    for (int c = 0; c < 4; ++c)
        dst[cur + c] = w[c];
    for (int gz = cur + 4; gz < G.gz; ++gz)
        dst[gz] = 0.0f;
}

// Pass 2 (y): T2[comp][x][gy][gz] = sum_y B_{gy - iy(y)}(t(y)) T1[comp][x][y][gz], FP64,
// one thread per output, y in a fixed order.
__global__ __launch_bounds__(kThreads) void k_bspline_adj_y(const float *__restrict__ T1,
                                                            BsplineGeom G, double *__restrict__ T2)
{
    const int64_t total = 3 * (int64_t)G.ox * G.gy * G.gz;
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= total)
        return;
    const int gz = (int)(e % G.gz);
    const int gy = (int)((e / G.gz) % G.gy);
    const int64_t cx = e / ((int64_t)G.gz * G.gy);          // comp * ox + x
    // rows y whose cell reaches control gy: iy in [gy - 3, gy]
    double s = 0.0;
    for (int y = 0; y < G.oy; ++y) {
        int32_t iy;
        float ty, By[4];
        bs_cell(y, G.inv_hy, G.gy, iy, ty);
        const int b = gy - iy;
        if (b < 0 || b > 3)
            continue;
        bs_basis(ty, By);
        s += (double)By[b] * (double)T1[(cx * G.oy + y) * G.gz + gz];
    }
    T2[e] = s;
}

// Pass 3 (x): grad_ctrl[comp][gx][gy][gz] = sum_x B_{gx - ix(x)}(t(x)) T2[comp][x][gy][gz].
__global__ __launch_bounds__(kThreads) void k_bspline_adj_x(const double *__restrict__ T2,
                                                            BsplineGeom G,
                                                            float *__restrict__ grad_ctrl)
{
    const int total = 3 * G.gx * G.gy * G.gz;
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= total)
        return;
    const int plane = G.gy * G.gz;
    const int comp = e / (G.gx * plane);
    const int rem = e - comp * G.gx * plane;
    const int gx = rem / plane, r2 = rem - gx * plane;
    double s = 0.0;
    for (int x = 0; x < G.ox; ++x) {
        int32_t ix;
        float tx, Bx[4];
        bs_cell(x, G.inv_hx, G.gx, ix, tx);
        const int a = gx - ix;
        if (a < 0 || a > 3)
            continue;
        bs_basis(tx, Bx);
        s += (double)Bx[a] * T2[((int64_t)comp * G.ox + x) * plane + r2];
    }
    grad_ctrl[e] = (float)s;
}

int bspline_max_grid() { return kMaxG; }

// Workspace of the adjoint: T1 (FP32, 3 x ox x oy x Gz), then T2 (FP64,
// 3 x ox x Gy x Gz) at a 256-byte aligned offset.
static int64_t adj_t1_bytes(const int64_t od[3], const int64_t G[3])
{
    return ((3 * od[0] * od[1] * G[2] * (int64_t)sizeof(float)) + 255) & ~(int64_t)255;
}

int64_t bspline_adj_ws_bytes(const int64_t od[3], const int64_t G[3])
{
    return adj_t1_bytes(od, G) + 3 * od[0] * G[1] * G[2] * (int64_t)sizeof(double);
}

hipError_t launch_bspline_up(const float *ctrl, const int64_t G[3], const int64_t od[3],
                             float *disp, bool vec, hipStream_t s)
{
    if (od[0] == 0 || od[1] == 0 || od[2] == 0)
        return hipSuccess;
    const BsplineGeom g = bspline_geom(G, od);
    dim3 grid((unsigned)od[0], (unsigned)((od[1] + kRowsPerWG - 1) / kRowsPerWG));
    hipLaunchKernelGGL(k_bspline_up, grid, dim3(kThreads), 0, s, ctrl, g, disp, vec ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_bspline_adj(const float *grad_disp, const int64_t od[3], const int64_t G[3],
                              float *grad_ctrl, double *ws, hipStream_t s)
{
    BsplineGeom g = bspline_geom(G, od);
    if (od[0] == 0 || od[1] == 0 || od[2] == 0)
        g.ox = 0;                      // no voxels: every control gradient is 0
    float *T1 = reinterpret_cast<float *>(ws);
    double *T2 = reinterpret_cast<double *>(reinterpret_cast<char *>(ws) + adj_t1_bytes(od, G));
    if (g.ox > 0) {
        const int64_t rows = 3 * od[0] * od[1];
        const bool vec = od[2] % 4 == 0 && (reinterpret_cast<uintptr_t>(grad_disp) & 15u) == 0;
        hipLaunchKernelGGL(k_bspline_adj_z, dim3((unsigned)((rows + kThreads - 1) / kThreads)),
                           dim3(kThreads), 0, s, grad_disp, g, T1, vec ? 1 : 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        const int64_t n2 = 3 * od[0] * G[1] * G[2];
        hipLaunchKernelGGL(k_bspline_adj_y, dim3((unsigned)((n2 + kThreads - 1) / kThreads)),
                           dim3(kThreads), 0, s, T1, g, T2);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    const int total = (int)(3 * G[0] * G[1] * G[2]);
    hipLaunchKernelGGL(k_bspline_adj_x, dim3((unsigned)((total + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, T2, g, grad_ctrl);
    return hipGetLastError();
}

}  // namespace ctaug
