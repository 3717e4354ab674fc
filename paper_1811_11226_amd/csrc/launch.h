// launch.h -- host-side launchers of the gfx950 kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace ctaug {

hipError_t launch_warp_single(const FwdJob &J, const Tiling &TL, hipStream_t s);
// Labels alone (J.lbl, J.lout; J.img unused): see k_warp_labels.
hipError_t launch_warp_labels(const FwdJob &J, hipStream_t s);
// Input / LDS cell types shared by every job of a batch launch; the Spline
// modes warp B-spline jobs (displacement tiles, FP32 LDS cells).
enum : int { kBatchMixed = 0, kBatchI16F32 = 1, kBatchI16I16 = 2, kBatchF32 = 3,
             kBatchSplineI16 = 4, kBatchSplineF32 = 5, kBatchSplineMixed = 6 };
// Displacement warps: 8 x 8 x 16 tiles (one run of 4 z voxels per thread, so
// that a tile can reduce its coordinate range before staging) and a fixed
// reservation, since the footprint has no a-priori bound.
constexpr Tiling kDispTiling = {3, 3, 4};
constexpr int32_t kDispLdsCells = 10224;
hipError_t launch_warp_batch(const FwdJob *jobs_dev, const int32_t *prefix_dev, int32_t njobs,
                             int32_t total_tiles, int32_t grid, const Tiling &TL,
                             int32_t lds_cells, int32_t elem_bytes, int mode, bool aligned,
                             hipStream_t s);
// Largest LDS footprint (cells of input-type image + int8 label) any tile of J
// can need; the most cells a reservation of elem_bytes-wide cells can hold;
// the cells reserved for a bound; the LDS bytes of a reservation.
int32_t footprint_cells_bound(const FwdJob &J, const Tiling &TL);
int32_t lds_cells_cap(int32_t elem_bytes);
int32_t lds_cells_for(int32_t bound, int32_t elem_bytes);
size_t lds_bytes_for(int32_t cells, int32_t elem_bytes);
Tiling choose_subtile(const FwdJob &J, const Tiling &TL, int32_t lds_cells);
hipError_t launch_photometric(float *data, int64_t n, int64_t nz, const Photo &P, float occ_lo,
                              float occ_hi, uint32_t vol, uint32_t k0, uint32_t k1, bool vec,
                              hipStream_t s);
hipError_t launch_noise(uint64_t v0, int64_t n, uint32_t vol, uint32_t k0, uint32_t k1,
                        float *gauss, uint32_t *words, hipStream_t s);

hipError_t launch_box_muller(const uint32_t *words, int64_t npairs, float *out, hipStream_t s);
hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s);

// Rows of FP64 partials of grad_M the adjoint writes: one per persistent
// workgroup, at most kBwdMaxRows.
constexpr int64_t kBwdMaxRows = 2048;
int64_t bwd_partial_rows(int64_t ox, int64_t oy, int64_t oz);
// Adjoint of a warp.  A control grid (J.ctrl) requires bwd_spline_eval_ok(J.bs)
// (every tile's z window of controls fits the kernel's row profiles); its
// gradient g_ctrl is fused into the adjoint when bwd_ctrl_fused(J.bs) holds,
// with ctrl_part holding ctrl_reduce_doubles(bwd_partial_rows(), 3 Gx Gy Gz)
// doubles (the per-workgroup rows, then the row-group sums).
// Otherwise the caller materialises the field and uses the dense path.
hipError_t launch_warp_bwd(const FwdJob &J, const float *g, float *g_img, float *g_disp,
                           double *g_M, double *partials, double *ctrl_part, float *g_ctrl,
                           hipStream_t s);
int64_t ctrl_reduce_doubles(int64_t rows, int64_t nctrl);
// Batched affine adjoint (all jobs of one input dtype): per job its
// descriptor (tiles set by the launcher), grad_out, grad_img and grad_M
// (either may be null); partials: kBwdMaxRows * 12 doubles per job.
struct BwdJob {
    FwdJob J;
    const float *g;
    float *g_img;
    double *g_M;
};
constexpr int32_t kBwdBatchMax = 8;    // jobs per launch (the table travels in the kernel arguments)
struct BwdBatch {
    BwdJob jobs[kBwdBatchMax];
    int32_t prefix[kBwdBatchMax + 1];
    int32_t fix_bits[kBwdBatchMax];    // per job: 32-bit fixed-point exponent, or -1
    int32_t njobs;
};
hipError_t launch_warp_bwd_batch(const BwdJob *jobs, int32_t n, double *partials, hipStream_t s);
bool bwd_spline_eval_ok(const BsplineGeom &B);
bool bwd_ctrl_fused(const BsplineGeom &B);

int bspline_max_grid();
int64_t bspline_adj_ws_bytes(const int64_t od[3], const int64_t G[3]);
hipError_t launch_bspline_up(const float *ctrl, const int64_t G[3], const int64_t od[3],
                             float *disp, bool vec, hipStream_t s);
hipError_t launch_bspline_adj(const float *grad_disp, const int64_t od[3], const int64_t G[3],
                              float *grad_ctrl, double *ws, hipStream_t s);

// Gaussian smoothing of the resampling pre-step.
constexpr int kMaxGaussRadius = 160;
struct GaussTaps {
    int32_t R;                         // taps at offsets -R .. R
    float w[kMaxGaussRadius + 1];      // w[|d|], normalised to sum 1 over -R .. R
};
int32_t gauss_radius(float sigma);
GaussTaps gauss_taps(float sigma);
hipError_t launch_smooth_axis(const void *in, bool in_i16, float *out, const int32_t dim[3],
                              int axis, const GaussTaps &K, hipStream_t s);

}  // namespace ctaug
