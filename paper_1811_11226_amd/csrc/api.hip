// api.hip -- the C ABI declared in include/ctaug.h: argument validation, job
// descriptor construction, launch configuration and the batch plan
// (device job table + pinned staging + HIP graph + autotuner).
#include <cmath>
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ctaug.h"
#include "device_common.h"
#include "launch.h"

using namespace ctaug;

namespace {

constexpr int64_t kMaxElems = 2147483647LL;   // int32 linear indices in the kernels
constexpr int64_t kMaxF32In = 1073741823LL;   // FP32 input bytes must fit a 32-bit buffer range
constexpr int64_t kMax24 = 1LL << 24;          // operands of the kernels' 24-bit multiplies
constexpr Tiling kDefaultTiling = {3, 4, 4};   // 8 x 16 x 16 output voxels per workgroup

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

ctaug_status hip_status(hipError_t e) { return e == hipSuccess ? CTAUG_OK : CTAUG_EHIP; }

int64_t nelem(const int64_t d[3]) { return d[0] * d[1] * d[2]; }

bool dims_valid(const int64_t d[3])
{
    if (d[0] < 0 || d[1] < 0 || d[2] < 0)
        return false;
    if (d[0] == 0 || d[1] == 0 || d[2] == 0)
        return true;
    if (d[0] > kMaxElems || d[1] > kMaxElems || d[2] > kMaxElems)
        return false;
    return d[0] * d[1] <= kMaxElems && d[0] * d[1] * d[2] <= kMaxElems;
}

// Element strides of a volume: {0,0,0} = dense.  A strided layout keeps z
// contiguous and its x stride a whole number of y rows (any box cut out of a
// dense parent).  Writes the row pitch sy (elements between y rows) and the
// rows per x plane ry; false on a malformed layout.
bool vol_layout(const ctaug_vol *v, int64_t &ry, int64_t &sy)
{
    const int64_t *d = v->dim, *st = v->stride;
    if (st[0] == 0 && st[1] == 0 && st[2] == 0) {
        ry = d[1];
        sy = d[2];
        return true;
    }
    if (st[2] != 1 || st[1] < 1 || st[0] < 1 || st[1] > kMaxElems || st[0] > kMaxElems)
        return false;
    if (st[1] < d[2] || st[0] % st[1] != 0 || st[0] / st[1] < d[1])
        return false;
    ry = st[0] / st[1];
    sy = st[1];
    return true;
}

bool is_dense(const ctaug_vol *v)
{
    int64_t ry = 0, sy = 0;
    if (!vol_layout(v, ry, sy))
        return false;
    return nelem(v->dim) == 0 || (ry == v->dim[1] && sy == v->dim[2]);
}

// Elements from the first to one past the last element of the volume.
int64_t vol_extent(const ctaug_vol *v)
{
    int64_t ry = 0, sy = 0;
    if (nelem(v->dim) == 0 || !vol_layout(v, ry, sy))
        return 0;
    return ((v->dim[0] - 1) * ry + (v->dim[1] - 1)) * sy + v->dim[2];
}

// Validate a volume argument; `allowed` is a bit set of dtypes; `strided`:
// the argument may be a strided view (else it must be dense).
ctaug_status check_vol(const ctaug_vol *v, unsigned allowed, bool strided = false)
{
    if (!v || v->reserved != 0)
        return CTAUG_EINVAL;
    if (v->dtype < 0 || v->dtype > 2 || !(allowed & (1u << v->dtype)))
        return CTAUG_EDTYPE;
    if (!dims_valid(v->dim))
        return CTAUG_ESHAPE;
    int64_t ry = 0, sy = 0;
    if (!vol_layout(v, ry, sy) || (!strided && !is_dense(v)))
        return CTAUG_ESHAPE;
    if (nelem(v->dim) > 0) {           // extent within int32 element offsets
        const int64_t rows = (v->dim[0] - 1) * ry + (v->dim[1] - 1);
        if (rows > kMaxElems || rows * sy + v->dim[2] > kMaxElems)
            return CTAUG_ESHAPE;
    }
    if (!v->data && nelem(v->dim) > 0)
        return CTAUG_EINVAL;
    return CTAUG_OK;
}

// A gathered input: offsets (ix ry + iy) sy + iz are formed with 24-bit
// multiplies, whose operands must stay below 2^24.
bool gather_addressable(const ctaug_vol *v)
{
    int64_t ry = 0, sy = 0;
    if (nelem(v->dim) == 0)
        return true;
    if (!vol_layout(v, ry, sy))
        return false;
    return (v->dim[0] - 1) * ry + v->dim[1] <= kMax24 && sy < kMax24;
}

bool same_layout(const ctaug_vol *a, const ctaug_vol *b)
{
    int64_t ra = 0, sa = 0, rb = 0, sb = 0;
    return vol_layout(a, ra, sa) && vol_layout(b, rb, sb) && ra == rb && sa == sb;
}

bool same_dims(const ctaug_vol *a, const ctaug_vol *b)
{
    return a->dim[0] == b->dim[0] && a->dim[1] == b->dim[1] && a->dim[2] == b->dim[2];
}

bool finite_all(const float *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i]))
            return false;
    return true;
}

ctaug_status check_photo(const ctaug_photo *p)
{
    if (!p)
        return CTAUG_OK;
    const float vals[6] = {p->gain, p->offset, p->sigma, p->win_lo, p->win_hi, p->gamma};
    if (!finite_all(vals, 6) || p->sigma < 0.0f || !(p->gamma > 0.0f))
        return CTAUG_EINVAL;
    if (p->flags & ~(uint32_t)(CTAUG_PHOTO_WINDOW | CTAUG_PHOTO_OCCLUDE))
        return CTAUG_EINVAL;
    if ((p->flags & CTAUG_PHOTO_OCCLUDE) && !(std::isfinite(p->occ_lo) && std::isfinite(p->occ_hi)))
        return CTAUG_EINVAL;
    if ((p->flags & CTAUG_PHOTO_WINDOW) && !(p->win_hi > p->win_lo))
        return CTAUG_EINVAL;
    return CTAUG_OK;
}

void set_photo(FwdJob &J, const ctaug_photo *p)
{
    J.gain = 1.0f;
    J.offset = 0.0f;
    J.sigma = 0.0f;
    J.win_lo = 0.0f;
    J.inv_range = 1.0f;
    J.gamma = 1.0f;
    J.occ_lo = 0.0f;
    J.occ_hi = -1.0f;
    J.vol_id = J.key0 = J.key1 = 0;
    if (!p)
        return;
    J.flags |= kFlagPhoto;
    J.gain = p->gain;
    J.offset = p->offset;
    J.sigma = p->sigma;
    J.win_lo = p->win_lo;
    J.inv_range = (float)(1.0 / ((double)p->win_hi - (double)p->win_lo));
    J.gamma = p->gamma;
    J.vol_id = p->volume_id;
    J.key0 = (uint32_t)p->seed;
    J.key1 = (uint32_t)(p->seed >> 32);
    if (p->sigma > 0.0f)
        J.flags |= kFlagNoise;
    if (p->flags & CTAUG_PHOTO_WINDOW) {
        J.flags |= kFlagWindow;
        if (p->gamma != 1.0f)
            J.flags |= kFlagGamma;
    }
    if (p->flags & CTAUG_PHOTO_OCCLUDE) {
        J.flags |= kFlagOcclude;
        J.occ_lo = p->occ_lo;
        J.occ_hi = p->occ_hi;
    }
}

Photo photo_from_job(const FwdJob &J)
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

void set_tiles(FwdJob &J, const Tiling &TL)
{
    J.tiles_x = (J.ox + (1 << TL.lx) - 1) >> TL.lx;
    J.tiles_y = (J.oy + (1 << TL.ly) - 1) >> TL.ly;
    J.tiles_z = (J.oz + (1 << TL.lz) - 1) >> TL.lz;
    J.sub[0] = TL.lx;
    J.sub[1] = TL.ly;
    J.sub[2] = TL.lz;
}

// Stage each tile of J in sub-tiles whose footprint fits `cells` LDS cells.
void set_subtiles(FwdJob &J, const Tiling &TL, int32_t cells)
{
    const Tiling SL = choose_subtile(J, TL, cells);
    J.sub[0] = SL.lx;
    J.sub[1] = SL.ly;
    J.sub[2] = SL.lz;
}

// Validate the arguments of one forward warp and build its descriptor.
ctaug_status make_job(const ctaug_vol *img_in, const ctaug_vol *lbl_in, const float *M,
                      const float *disp, bool need_disp, float fill, int32_t label_fill,
                      const ctaug_photo *photo, const ctaug_vol *img_out,
                      const ctaug_vol *lbl_out, const Tiling &TL, FwdJob &J)
{
    ctaug_status st;
    if ((st = check_vol(img_in, 1u << CTAUG_F32 | 1u << CTAUG_I16, true)) != CTAUG_OK)
        return st;
    if (img_in->dtype == CTAUG_F32 && vol_extent(img_in) > kMaxF32In)
        return CTAUG_ESHAPE;
    if (!gather_addressable(img_in))
        return CTAUG_ESHAPE;
    if ((st = check_vol(img_out, 1u << CTAUG_F32)) != CTAUG_OK)
        return st;
    if (lbl_in) {
        if ((st = check_vol(lbl_in, 1u << CTAUG_I8, true)) != CTAUG_OK)
            return st;
        if (!same_dims(lbl_in, img_in))
            return CTAUG_ESHAPE;
        if (nelem(img_in->dim) > 0 && !same_layout(lbl_in, img_in))
            return CTAUG_ESHAPE;
        if (!lbl_out)
            return CTAUG_EINVAL;
        if ((st = check_vol(lbl_out, 1u << CTAUG_I8)) != CTAUG_OK)
            return st;
        if (!same_dims(lbl_out, img_out))
            return CTAUG_ESHAPE;
    }
    if (!M || !finite_all(M, 12) || !std::isfinite(fill))
        return CTAUG_EINVAL;
    if (label_fill < -128 || label_fill > 127)
        return CTAUG_EINVAL;
    if ((st = check_photo(photo)) != CTAUG_OK)
        return st;
    const int64_t nout = nelem(img_out->dim);
    if (need_disp) {
        if (!disp && nout > 0)
            return CTAUG_EINVAL;
        if (3 * nout > kMaxElems)
            return CTAUG_ESHAPE;
    }
    std::memset(&J, 0, sizeof J);
    J.img = img_in->data;
    J.lbl = lbl_in ? static_cast<const int8_t *>(lbl_in->data) : nullptr;
    J.out = static_cast<float *>(img_out->data);
    J.lout = lbl_in ? static_cast<int8_t *>(lbl_out->data) : nullptr;
    J.disp = need_disp ? disp : nullptr;
    J.dtype = img_in->dtype;
    J.nx = (int32_t)img_in->dim[0];
    J.ny = (int32_t)img_in->dim[1];
    J.nz = (int32_t)img_in->dim[2];
    {
        int64_t ry = 0, sy = 0;
        (void)vol_layout(img_in, ry, sy);
        J.in_ry = (int32_t)ry;
        J.in_sy = (int32_t)sy;
        J.in_extent = (int32_t)vol_extent(img_in);
    }
    J.ox = (int32_t)img_out->dim[0];
    J.oy = (int32_t)img_out->dim[1];
    J.oz = (int32_t)img_out->dim[2];
    std::memcpy(J.M, M, sizeof J.M);
    // Bound on the FP32 rounding of q over the output box: three fmaf roundings
    // of partial sums bounded by S_i = sum_j |A_ij| (n_j - 1) + |b_i|.
    const int64_t last[3] = {std::max<int64_t>(J.ox - 1, 0), std::max<int64_t>(J.oy - 1, 0),
                             std::max<int64_t>(J.oz - 1, 0)};
    for (int i = 0; i < 3; ++i) {
        double S = std::fabs((double)M[4 * i + 3]);
        for (int j = 0; j < 3; ++j)
            S += std::fabs((double)M[4 * i + j]) * (double)last[j];
        J.delta[i] = (float)((S + 1.0) * std::ldexp(1.0, -20));
    }
    J.fill = fill;
    J.label_fill = label_fill;
    if (fill >= -32768.0f && fill <= 32767.0f && (float)(int16_t)fill == fill)
        J.flags |= kFlagFillInT;
    if (J.lbl)
        J.flags |= kFlagLabels;
    set_photo(J, photo);
    const bool out_aligned = (reinterpret_cast<uintptr_t>(J.out) & 15u) == 0;
    const bool lbl_aligned = !J.lout || (reinterpret_cast<uintptr_t>(J.lout) & 3u) == 0;
    if (J.oz % 4 == 0 && out_aligned && lbl_aligned)
        J.flags |= kFlagVec;
    set_tiles(J, TL);
    return CTAUG_OK;
}

bool empty(const FwdJob &J) { return J.ox == 0 || J.oy == 0 || J.oz == 0; }

}  // namespace

// ---------------------------------------------------------------------------

extern "C" const char *ctaug_status_string(ctaug_status s)
{
    switch (s) {
    case CTAUG_OK: return "ok";
    case CTAUG_EINVAL: return "invalid argument";
    case CTAUG_EDTYPE: return "unsupported dtype";
    case CTAUG_ESHAPE: return "invalid or inconsistent shape";
    case CTAUG_EWORKSPACE: return "workspace missing or too small";
    case CTAUG_EHIP: return "HIP runtime error";
    case CTAUG_ENODEV: return "no usable gfx950 device";
    }
    return "unknown status";
}

extern "C" int ctaug_version(void) { return 10000; }

extern "C" ctaug_status ctaug_affine_matrix(const ctaug_affine_params *p, const int64_t in_dim[3],
                                            const int64_t out_dim[3], double M64[12],
                                            float M32[12])
{
    if (!p || !in_dim || !out_dim || (!M64 && !M32))
        return CTAUG_EINVAL;
    for (int i = 0; i < 3; ++i)
        if (in_dim[i] < 0 || out_dim[i] < 0)
            return CTAUG_ESHAPE;
    const double *all = reinterpret_cast<const double *>(p);
    for (size_t i = 0; i < sizeof(ctaug_affine_params) / sizeof(double); ++i)
        if (!std::isfinite(all[i]))
            return CTAUG_EINVAL;
    // factors, each a 3x3 row-major matrix
    double f[7][9];
    std::memcpy(f[0], p->generic, sizeof f[0]);
    const double cz = std::cos(p->rot[2]), sz = std::sin(p->rot[2]);
    const double cy = std::cos(p->rot[1]), sy = std::sin(p->rot[1]);
    const double cx = std::cos(p->rot[0]), sx = std::sin(p->rot[0]);
    const double Rz[9] = {cz, -sz, 0, sz, cz, 0, 0, 0, 1};
    const double Ry[9] = {cy, 0, sy, 0, 1, 0, -sy, 0, cy};
    const double Rx[9] = {1, 0, 0, 0, cx, -sx, 0, sx, cx};
    const double H[9] = {1, p->shear[0], p->shear[1], 0, 1, p->shear[2], 0, 0, 1};
    const double S[9] = {p->scale[0], 0, 0, 0, p->scale[1], 0, 0, 0, p->scale[2]};
    double F[9] = {0};
    for (int i = 0; i < 3; ++i)
        F[4 * i] = p->reflect[i] != 0.0 ? -1.0 : 1.0;
    std::memcpy(f[1], Rz, sizeof Rz);
    std::memcpy(f[2], Ry, sizeof Ry);
    std::memcpy(f[3], Rx, sizeof Rx);
    std::memcpy(f[4], H, sizeof H);
    std::memcpy(f[5], S, sizeof S);
    std::memcpy(f[6], F, sizeof F);
    double A[9];
    std::memcpy(A, f[0], sizeof A);
    for (int k = 1; k < 7; ++k) {
        double R[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                R[3 * i + j] = A[3 * i] * f[k][j] + A[3 * i + 1] * f[k][3 + j] +
                               A[3 * i + 2] * f[k][6 + j];
        std::memcpy(A, R, sizeof A);
    }
    double out[12];
    for (int i = 0; i < 3; ++i) {
        double Ac = 0.0;
        for (int j = 0; j < 3; ++j) {
            out[4 * i + j] = A[3 * i + j];
            Ac += A[3 * i + j] * (0.5 * (double)(out_dim[j] - 1));
        }
        out[4 * i + 3] = 0.5 * (double)(in_dim[i] - 1) + p->disp[i] + p->crop[i] - Ac;
    }
    for (int k = 0; k < 12; ++k) {
        if (M64)
            M64[k] = out[k];
        if (M32)
            M32[k] = (float)out[k];
    }
    return CTAUG_OK;
}

static bool grid_valid(const int64_t G[3])
{
    if (!G)
        return false;
    for (int i = 0; i < 3; ++i)
        if (G[i] < 4 || G[i] > bspline_max_grid())
            return false;
    return true;
}

static ctaug_status check_grid(const int64_t G[3], const int64_t od[3])
{
    if (!G || !od)
        return CTAUG_EINVAL;
    if (!dims_valid(od) || 3 * nelem(od) > kMaxElems)
        return CTAUG_ESHAPE;
    return grid_valid(G) ? CTAUG_OK : CTAUG_ESHAPE;
}

static ctaug_status warp_impl(const ctaug_vol *img_in, const ctaug_vol *lbl_in, const float M[12],
                              const float *disp, bool need_disp, float fill, int32_t label_fill,
                              const ctaug_photo *photo, ctaug_vol *img_out, ctaug_vol *lbl_out,
                              void *stream)
{
    FwdJob J;
    ctaug_status st = make_job(img_in, lbl_in, M, disp, need_disp, fill, label_fill, photo,
                               img_out, lbl_out, kDefaultTiling, J);
    if (st != CTAUG_OK)
        return st;
    if (empty(J))
        return CTAUG_OK;
    return hip_status(launch_warp_single(J, kDefaultTiling, as_stream(stream)));
}

extern "C" ctaug_status ctaug_warp_affine(const ctaug_vol *img_in, const ctaug_vol *lbl_in,
                                          const float M[12], float fill, int32_t label_fill,
                                          const ctaug_photo *photo, ctaug_vol *img_out,
                                          ctaug_vol *lbl_out, void *stream)
{
    return warp_impl(img_in, lbl_in, M, nullptr, false, fill, label_fill, photo, img_out, lbl_out,
                     stream);
}

extern "C" ctaug_status ctaug_warp_displacement(const ctaug_vol *img_in, const ctaug_vol *lbl_in,
                                                const float M[12], const float *disp, float fill,
                                                int32_t label_fill, const ctaug_photo *photo,
                                                ctaug_vol *img_out, ctaug_vol *lbl_out,
                                                void *stream)
{
    return warp_impl(img_in, lbl_in, M, disp, true, fill, label_fill, photo, img_out, lbl_out,
                     stream);
}

extern "C" ctaug_status ctaug_warp_labels(const ctaug_vol *lbl_in, const float M[12],
                                          int32_t label_fill, ctaug_vol *lbl_out, void *stream)
{
    ctaug_status st;
    if ((st = check_vol(lbl_in, 1u << CTAUG_I8, true)) != CTAUG_OK)
        return st;
    if (!gather_addressable(lbl_in))
        return CTAUG_ESHAPE;
    if ((st = check_vol(lbl_out, 1u << CTAUG_I8)) != CTAUG_OK)
        return st;
    if (!M || !finite_all(M, 12))
        return CTAUG_EINVAL;
    if (label_fill < -128 || label_fill > 127)
        return CTAUG_EINVAL;
    FwdJob J;
    std::memset(&J, 0, sizeof J);
    J.lbl = static_cast<const int8_t *>(lbl_in->data);
    J.lout = static_cast<int8_t *>(lbl_out->data);
    J.dtype = kI8;                     // labels only: no image
    J.nx = (int32_t)lbl_in->dim[0];
    J.ny = (int32_t)lbl_in->dim[1];
    J.nz = (int32_t)lbl_in->dim[2];
    int64_t ry = 0, sy = 0;
    (void)vol_layout(lbl_in, ry, sy);
    J.in_ry = (int32_t)ry;
    J.in_sy = (int32_t)sy;
    J.in_extent = (int32_t)vol_extent(lbl_in);
    J.ox = (int32_t)lbl_out->dim[0];
    J.oy = (int32_t)lbl_out->dim[1];
    J.oz = (int32_t)lbl_out->dim[2];
    std::memcpy(J.M, M, sizeof J.M);
    J.label_fill = label_fill;
    J.flags = kFlagLabels;
    if (J.oz % 4 == 0 && (reinterpret_cast<uintptr_t>(J.lout) & 3u) == 0)
        J.flags |= kFlagVec;
    if (empty(J))
        return CTAUG_OK;
    return hip_status(launch_warp_labels(J, as_stream(stream)));
}

extern "C" ctaug_status ctaug_warp_bspline(const ctaug_vol *img_in, const ctaug_vol *lbl_in,
                                           const float M[12], const float *ctrl,
                                           const int64_t G[3], float fill, int32_t label_fill,
                                           const ctaug_photo *photo, ctaug_vol *img_out,
                                           ctaug_vol *lbl_out, void *stream)
{
    FwdJob J;
    ctaug_status st = make_job(img_in, lbl_in, M, nullptr, false, fill, label_fill, photo,
                               img_out, lbl_out, kDefaultTiling, J);
    if (st != CTAUG_OK)
        return st;
    if (!G)
        return CTAUG_EINVAL;
    if (!grid_valid(G))
        return CTAUG_ESHAPE;
    if (empty(J))
        return CTAUG_OK;
    if (!ctrl)
        return CTAUG_EINVAL;
    J.ctrl = ctrl;
    J.bs = bspline_geom(G, img_out->dim);
    return hip_status(launch_warp_single(J, kDefaultTiling, as_stream(stream)));
}

extern "C" ctaug_status ctaug_photometric_noise(ctaug_vol *inout, const ctaug_photo *photo,
                                                void *stream)
{
    ctaug_status st;
    if ((st = check_vol(inout, 1u << CTAUG_F32)) != CTAUG_OK)
        return st;
    if (!photo)
        return CTAUG_EINVAL;
    if ((st = check_photo(photo)) != CTAUG_OK)
        return st;
    FwdJob J;
    std::memset(&J, 0, sizeof J);
    set_photo(J, photo);
    const int64_t n = nelem(inout->dim);
    if (n == 0)
        return CTAUG_OK;
    const bool vec = n % 4 == 0 && (reinterpret_cast<uintptr_t>(inout->data) & 15u) == 0;
    return hip_status(launch_photometric(static_cast<float *>(inout->data), n, inout->dim[2],
                                         photo_from_job(J), J.occ_lo, J.occ_hi, J.vol_id, J.key0,
                                         J.key1, vec, as_stream(stream)));
}

extern "C" ctaug_status ctaug_noise(uint64_t seed, uint32_t volume_id, uint64_t v0, int64_t n,
                                    float *gauss, uint32_t *words, void *stream)
{
    if (n < 0 || (uint64_t)n > ~(uint64_t)0 - v0)
        return CTAUG_EINVAL;
    if (n == 0 || (!gauss && !words))
        return CTAUG_OK;
    return hip_status(launch_noise(v0, n, volume_id, (uint32_t)seed, (uint32_t)(seed >> 32), gauss,
                                   words, as_stream(stream)));
}

extern "C" ctaug_status ctaug_box_muller(const uint32_t *words, int64_t npairs, float *out,
                                         void *stream)
{
    if (npairs < 0 || (npairs > 0 && (!words || !out)))
        return CTAUG_EINVAL;
    if (npairs == 0)
        return CTAUG_OK;
    return hip_status(launch_box_muller(words, npairs, out, as_stream(stream)));
}

extern "C" size_t ctaug_warp_backward_workspace(const int64_t out_dim[3])
{
    if (!out_dim || !dims_valid(out_dim))
        return 0;
    return (size_t)bwd_partial_rows(out_dim[0], out_dim[1], out_dim[2]) * 12 * sizeof(double);
}

// The backward passes differentiate the photometric chain only without the
// window (affine in the sampled value).
static ctaug_status check_photo_adjoint(const ctaug_photo *photo)
{
    const ctaug_status st = check_photo(photo);
    if (st != CTAUG_OK)
        return st;
    return photo && (photo->flags & CTAUG_PHOTO_WINDOW) ? CTAUG_EINVAL : CTAUG_OK;
}

namespace {
ctaug_status scratch_address(void **out);
constexpr size_t kScratchBytes = (size_t)kBwdMaxRows * 12 * sizeof(double);   // 192 KiB
}  // namespace

// use_scratch: the grad_M partials go to the library's static device array
// (ws / ws_bytes ignored), looked up after every argument is validated.
static ctaug_status backward_impl(const ctaug_vol *img_in, const float M[12], const float *disp,
                                  bool need_disp, float fill, const ctaug_photo *photo,
                                  const ctaug_vol *grad_out,
                                  ctaug_vol *grad_img, double *grad_M, float *grad_disp, void *ws,
                                  size_t ws_bytes, void *stream, bool use_scratch = false)
{
    ctaug_status st;
    if ((st = check_vol(img_in, 1u << CTAUG_F32 | 1u << CTAUG_I16, true)) != CTAUG_OK)
        return st;
    if ((st = check_vol(grad_out, 1u << CTAUG_F32)) != CTAUG_OK)
        return st;
    if (grad_img) {
        if ((st = check_vol(grad_img, 1u << CTAUG_F32)) != CTAUG_OK)
            return st;
        if (!same_dims(grad_img, img_in))
            return CTAUG_ESHAPE;
    }
    if (need_disp && grad_disp && 3 * nelem(grad_out->dim) > kMaxElems)
        return CTAUG_ESHAPE;
    if ((st = check_photo_adjoint(photo)) != CTAUG_OK)
        return st;
    if (grad_M) {
        const size_t need = ctaug_warp_backward_workspace(grad_out->dim);
        if (use_scratch && need > kScratchBytes)
            return CTAUG_EWORKSPACE;   // more partial rows than the static array holds
        if (!use_scratch && need > 0 && (!ws || ws_bytes < need))
            return CTAUG_EWORKSPACE;
    }
    FwdJob J;
    // the gradient volume plays the part of the forward output (dims only)
    ctaug_vol out_like = *grad_out;
    st = make_job(img_in, nullptr, M, disp, need_disp, fill, 0, photo, &out_like, nullptr,
                  kDefaultTiling, J);
    if (st != CTAUG_OK)
        return st;
    J.out = nullptr;
    if (empty(J) && !grad_M)
        return CTAUG_OK;
    if (use_scratch) {
        ws = nullptr;
        if (grad_M && (st = scratch_address(&ws)) != CTAUG_OK)
            return st;
    }
    return hip_status(launch_warp_bwd(J, static_cast<const float *>(grad_out->data),
                                      grad_img ? static_cast<float *>(grad_img->data) : nullptr,
                                      need_disp ? grad_disp : nullptr, grad_M,
                                      static_cast<double *>(ws), nullptr, nullptr,
                                      as_stream(stream)));
}

extern "C" ctaug_status ctaug_warp_affine_backward(const ctaug_vol *img_in, const float M[12],
                                                   float fill, const ctaug_photo *photo,
                                                   const ctaug_vol *grad_out, ctaug_vol *grad_img,
                                                   double *grad_M, void *ws, size_t ws_bytes,
                                                   void *stream)
{
    return backward_impl(img_in, M, nullptr, false, fill, photo, grad_out, grad_img, grad_M,
                         nullptr, ws, ws_bytes, stream);
}

extern "C" ctaug_status ctaug_warp_displacement_backward(const ctaug_vol *img_in,
                                                         const float M[12], const float *disp,
                                                         float fill, const ctaug_photo *photo,
                                                         const ctaug_vol *grad_out,
                                                         ctaug_vol *grad_img, double *grad_M,
                                                         float *grad_disp, void *ws,
                                                         size_t ws_bytes, void *stream)
{
    return backward_impl(img_in, M, disp, true, fill, photo, grad_out, grad_img, grad_M,
                         grad_disp, ws, ws_bytes, stream);
}

extern "C" size_t ctaug_warp_affine_backward_batch_workspace(int32_t n_jobs)
{
    if (n_jobs < 1 || n_jobs > (1 << 16))
        return 0;
    return (size_t)n_jobs * kBwdMaxRows * 12 * sizeof(double);
}

extern "C" ctaug_status ctaug_warp_affine_backward_batch(const ctaug_bwd_job *jobs, int32_t n_jobs,
                                                         void *ws, size_t ws_bytes, void *stream)
{
    if (!jobs || n_jobs < 1 || n_jobs > (1 << 16))
        return CTAUG_EINVAL;
    std::vector<BwdJob> B(n_jobs);
    bool any_M = false;
    for (int32_t k = 0; k < n_jobs; ++k) {
        const ctaug_bwd_job &j = jobs[k];
        ctaug_status st;
        if ((st = check_vol(&j.img_in, 1u << CTAUG_F32 | 1u << CTAUG_I16, true)) != CTAUG_OK)
            return st;
        if ((st = check_vol(&j.grad_out, 1u << CTAUG_F32)) != CTAUG_OK)
            return st;
        const bool want_img = j.grad_img.data != nullptr;
        if (want_img) {
            if ((st = check_vol(&j.grad_img, 1u << CTAUG_F32)) != CTAUG_OK)
                return st;
            if (!same_dims(&j.grad_img, &j.img_in))
                return CTAUG_ESHAPE;
        }
        const bool has_photo = !(j.photo.flags & CTAUG_PHOTO_NONE);
        if ((st = check_photo_adjoint(has_photo ? &j.photo : nullptr)) != CTAUG_OK)
            return st;
        if (j.img_in.dtype != jobs[0].img_in.dtype)
            return CTAUG_EDTYPE;           // one input dtype per batch
        ctaug_vol out_like = j.grad_out;   // the gradient plays the part of the output (dims only)
        FwdJob J;
        st = make_job(&j.img_in, nullptr, j.M, nullptr, false, j.fill, 0,
                      has_photo ? &j.photo : nullptr, &out_like, nullptr, kDefaultTiling, J);
        if (st != CTAUG_OK)
            return st;
        J.out = nullptr;
        B[k].J = J;
        B[k].g = static_cast<const float *>(j.grad_out.data);
        B[k].g_img = want_img ? static_cast<float *>(j.grad_img.data) : nullptr;
        B[k].g_M = j.grad_M;
        any_M = any_M || j.grad_M;
    }
    if (any_M && (!ws || ws_bytes < ctaug_warp_affine_backward_batch_workspace(n_jobs)))
        return CTAUG_EWORKSPACE;
    return hip_status(launch_warp_bwd_batch(B.data(), n_jobs, static_cast<double *>(ws),
                                            as_stream(stream)));
}

// ---------------------------------------------------------------------------
// Allocation-free adjoint: ctaug_warp_affine_backward with the grad_M partials
// (the only scratch memory the affine adjoint uses) in a static device array
// of the library instead of a caller workspace.  Each device holds its own
// copy of the array at its own address, looked up once per device; host code
// uses that address, never the array's name.
// ---------------------------------------------------------------------------

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of the current device's copy of `scratch`.
ctaug_status scratch_address(void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return CTAUG_EHIP;
    if (dev < 0 || dev >= kMaxDevices)
        return CTAUG_ENODEV;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return CTAUG_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CTAUG_OK;
}

}  // namespace

extern "C" ctaug_status ctaug_warp_affine_backward_noalloc(const ctaug_vol *img_in,
                                                           const float M[12], float fill,
                                                           const ctaug_photo *photo,
                                                           const ctaug_vol *grad_out,
                                                           ctaug_vol *grad_img, double *grad_M,
                                                           void *stream)
{
    return backward_impl(img_in, M, nullptr, false, fill, photo, grad_out, grad_img, grad_M,
                         nullptr, nullptr, 0, stream, true);
}

// Workspace of ctaug_warp_bspline_backward: grad_M partials, then either the
// per-workgroup control-grid rows (fused adjoint) or, for grids the fused
// kernel does not take, the dense field, its gradient and the B-spline
// adjoint's workspace.
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

extern "C" size_t ctaug_warp_bspline_backward_workspace(const int64_t out_dim[3],
                                                        const int64_t G[3])
{
    if (!out_dim || !dims_valid(out_dim) || !grid_valid(G))
        return 0;
    const int64_t rows = bwd_partial_rows(out_dim[0], out_dim[1], out_dim[2]);
    const size_t m = align256((size_t)rows * 12 * sizeof(double));
    const BsplineGeom B = bspline_geom(G, out_dim);
    if (bwd_ctrl_fused(B))
        return m + (size_t)ctrl_reduce_doubles(rows, 3 * G[0] * G[1] * G[2]) * sizeof(double);
    const size_t field = align256((size_t)(3 * nelem(out_dim)) * sizeof(float));
    return m + 2 * field + (size_t)bspline_adj_ws_bytes(out_dim, G);
}

extern "C" ctaug_status ctaug_warp_bspline_backward(const ctaug_vol *img_in, const float M[12],
                                                    const float *ctrl, const int64_t G[3],
                                                    float fill, const ctaug_photo *photo,
                                                    const ctaug_vol *grad_out,
                                                    ctaug_vol *grad_img, double *grad_M,
                                                    float *grad_ctrl, void *ws, size_t ws_bytes,
                                                    void *stream)
{
    ctaug_status st;
    if ((st = check_vol(img_in, 1u << CTAUG_F32 | 1u << CTAUG_I16, true)) != CTAUG_OK)
        return st;
    if ((st = check_vol(grad_out, 1u << CTAUG_F32)) != CTAUG_OK)
        return st;
    if (grad_img) {
        if ((st = check_vol(grad_img, 1u << CTAUG_F32)) != CTAUG_OK)
            return st;
        if (!same_dims(grad_img, img_in))
            return CTAUG_ESHAPE;
    }
    if (!G)
        return CTAUG_EINVAL;
    if (!grid_valid(G))
        return CTAUG_ESHAPE;
    if ((st = check_photo_adjoint(photo)) != CTAUG_OK)
        return st;
    const int64_t *od = grad_out->dim;
    const BsplineGeom B = bspline_geom(G, od);
    // fused kernel (field evaluated in the adjoint), or the dense route
    const bool fused = grad_ctrl ? bwd_ctrl_fused(B) : bwd_spline_eval_ok(B);
    if (!fused && 3 * nelem(od) > kMaxElems)
        return CTAUG_ESHAPE;
    const size_t need = ctaug_warp_bspline_backward_workspace(od, G);
    if ((grad_M || grad_ctrl || !fused) && need > 0 && (!ws || ws_bytes < need))
        return CTAUG_EWORKSPACE;
    FwdJob J;
    ctaug_vol out_like = *grad_out;    // the gradient plays the part of the output (dims only)
    st = make_job(img_in, nullptr, M, nullptr, false, fill, 0, photo, &out_like, nullptr,
                  kDefaultTiling, J);
    if (st != CTAUG_OK)
        return st;
    J.out = nullptr;
    if (!empty(J) && !ctrl)
        return CTAUG_EINVAL;
    if (empty(J) && !grad_M && !grad_ctrl)
        return CTAUG_OK;
    const float *g = static_cast<const float *>(grad_out->data);
    float *gi = grad_img ? static_cast<float *>(grad_img->data) : nullptr;
    char *w = static_cast<char *>(ws);
    double *partials = reinterpret_cast<double *>(w);
    const size_t m = align256((size_t)bwd_partial_rows(od[0], od[1], od[2]) * 12 * sizeof(double));
    hipStream_t s = as_stream(stream);
    if (fused) {
        J.ctrl = ctrl;
        J.bs = B;
        return hip_status(launch_warp_bwd(J, g, gi, nullptr, grad_M, partials,
                                          grad_ctrl ? reinterpret_cast<double *>(w + m) : nullptr,
                                          grad_ctrl, s));
    }
    // dense route: u = upsample(ctrl), adjoint with g_disp, then B^T g_disp
    const size_t field = align256((size_t)(3 * nelem(od)) * sizeof(float));
    float *u = reinterpret_cast<float *>(w + m);
    float *g_disp = reinterpret_cast<float *>(w + m + field);
    double *adj_ws = reinterpret_cast<double *>(w + m + 2 * field);
    if (!empty(J)) {
        const bool vec = od[2] % 4 == 0;   // workspace offsets are 256-byte aligned
        if ((st = hip_status(launch_bspline_up(ctrl, G, od, u, vec, s))) != CTAUG_OK)
            return st;
        J.disp = u;
    }
    st = hip_status(launch_warp_bwd(J, g, gi, grad_ctrl ? g_disp : nullptr, grad_M, partials,
                                    nullptr, nullptr, s));
    if (st != CTAUG_OK || !grad_ctrl)
        return st;
    return hip_status(launch_bspline_adj(g_disp, od, G, grad_ctrl, adj_ws, s));
}

extern "C" ctaug_status ctaug_bspline_upsample(const float *ctrl, const int64_t G[3],
                                               const int64_t out_dim[3], float *disp, void *stream)
{
    ctaug_status st = check_grid(G, out_dim);
    if (st != CTAUG_OK)
        return st;
    if (nelem(out_dim) == 0)
        return CTAUG_OK;
    if (!ctrl || !disp)
        return CTAUG_EINVAL;
    const bool vec = out_dim[2] % 4 == 0 && (reinterpret_cast<uintptr_t>(disp) & 15u) == 0;
    return hip_status(launch_bspline_up(ctrl, G, out_dim, disp, vec, as_stream(stream)));
}

extern "C" size_t ctaug_bspline_adjoint_workspace(const int64_t out_dim[3], const int64_t G[3])
{
    if (check_grid(G, out_dim) != CTAUG_OK)
        return 0;
    return (size_t)bspline_adj_ws_bytes(out_dim, G);
}

extern "C" ctaug_status ctaug_bspline_upsample_adjoint(const float *grad_disp,
                                                       const int64_t out_dim[3],
                                                       const int64_t G[3], float *grad_ctrl,
                                                       void *ws, size_t ws_bytes, void *stream)
{
    ctaug_status st = check_grid(G, out_dim);
    if (st != CTAUG_OK)
        return st;
    if (!grad_ctrl || (nelem(out_dim) > 0 && !grad_disp))
        return CTAUG_EINVAL;
    const size_t need = ctaug_bspline_adjoint_workspace(out_dim, G);
    if (need > 0 && (!ws || ws_bytes < need))
        return CTAUG_EWORKSPACE;
    return hip_status(launch_bspline_adj(grad_disp, out_dim, G, grad_ctrl,
                                         static_cast<double *>(ws), as_stream(stream)));
}

// ---------------------------------------------------------------------------
// Resampling pre-step
// ---------------------------------------------------------------------------

extern "C" ctaug_status ctaug_resample_sigma(const double spacing[3], double target,
                                             float sigma[3])
{
    if (!spacing || !sigma || !std::isfinite(target) || !(target > 0.0))
        return CTAUG_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(spacing[k]) || !(spacing[k] > 0.0))
            return CTAUG_EINVAL;
    for (int k = 0; k < 3; ++k)
        sigma[k] = (float)std::max((target / spacing[k] - 1.0) / 3.0, 0.0);
    return CTAUG_OK;
}

extern "C" size_t ctaug_gaussian_smooth_workspace(const int64_t dim[3])
{
    if (!dim || !dims_valid(dim))
        return 0;
    return (size_t)nelem(dim) * sizeof(float);
}

extern "C" ctaug_status ctaug_gaussian_smooth(const ctaug_vol *in, ctaug_vol *out,
                                              const float sigma[3], void *ws, size_t ws_bytes,
                                              void *stream)
{
    ctaug_status st;
    if ((st = check_vol(in, 1u << CTAUG_F32 | 1u << CTAUG_I16)) != CTAUG_OK)
        return st;
    if ((st = check_vol(out, 1u << CTAUG_F32)) != CTAUG_OK)
        return st;
    if (!same_dims(in, out))
        return CTAUG_ESHAPE;
    if (!sigma)
        return CTAUG_EINVAL;
    int active[3], m = 0;
    for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(sigma[k]) || sigma[k] < 0.0f)
            return CTAUG_EINVAL;
        if (gauss_radius(sigma[k]) > kMaxGaussRadius)
            return CTAUG_EINVAL;
        if (gauss_radius(sigma[k]) > 0)
            active[m++] = k;
    }
    const int64_t n = nelem(in->dim);
    if (n == 0)
        return CTAUG_OK;
    if (in->dim[0] > 65535 || in->dim[1] > 65535)
        return CTAUG_ESHAPE;               // grid y / z extents
    if (in->data == out->data)
        return CTAUG_EINVAL;               // out must not alias in
    if (m >= 2 && (!ws || ws_bytes < (size_t)n * sizeof(float)))
        return CTAUG_EWORKSPACE;
    const int32_t d[3] = {(int32_t)in->dim[0], (int32_t)in->dim[1], (int32_t)in->dim[2]};
    hipStream_t s = as_stream(stream);
    float *dst = static_cast<float *>(out->data);
    float *tmp = static_cast<float *>(ws);
    if (m == 0)                            // no smoothing: a converting copy
        return hip_status(launch_smooth_axis(in->data, in->dtype == CTAUG_I16, dst, d, 2,
                                             gauss_taps(0.0f), s));
    // ping-pong so that the last pass writes `out`
    const void *src = in->data;
    bool src_i16 = in->dtype == CTAUG_I16;
    for (int p = 0; p < m; ++p) {
        float *o = ((m - 1 - p) % 2 == 0) ? dst : tmp;
        hipError_t e = launch_smooth_axis(src, src_i16, o, d, active[p],
                                          gauss_taps(sigma[active[p]]), s);
        if (e != hipSuccess)
            return CTAUG_EHIP;
        src = o;
        src_i16 = false;
    }
    return CTAUG_OK;
}

// ---------------------------------------------------------------------------
// Batch plan
// ---------------------------------------------------------------------------

struct ctaug_batch_plan {
    int32_t n = 0;
    std::vector<int32_t> out_dims;      // 3 per job, fixed at creation
    std::vector<FwdJob> jobs;           // current descriptors (host copy)
    FwdJob *staging = nullptr;          // pinned host
    FwdJob *table = nullptr;            // device
    int32_t *prefix_dev = nullptr;      // device, n + 1
    int32_t total = 0;
    ctaug_tuning tune{};
    Tiling TL = kDefaultTiling;
    int32_t grid = 0;
    int32_t lds_cells = 0;              // LDS footprint cells reserved per workgroup
    int32_t elem_bytes = 4;             // LDS cell width: 2 when int16 cells are used
    bool all_i16 = true;                // every job has an int16 input
    bool all_f32 = true;                // every job has an FP32 input
    bool aligned = true;                // every job's output z extent is a multiple of 4
    bool spline = false;                // B-spline jobs (displacement tiles)
    int num_cu = 256;
    hipEvent_t upload_done = nullptr;
    bool upload_recorded = false;
    hipGraphExec_t exec = nullptr;
    std::string arch;                   // device architecture name (autotune cache key)
    uint64_t generation = 0;            // bumped by every (re)tiling
};

namespace {

int ilog2(int v)
{
    int l = 0;
    while ((1 << l) < v)
        ++l;
    return (1 << l) == v ? l : -1;
}

ctaug_status tiling_of(const ctaug_tuning *t, Tiling &TL)
{
    if (!t) {
        TL = kDefaultTiling;
        return CTAUG_OK;
    }
    const int lx = ilog2(t->tile[0]), ly = ilog2(t->tile[1]), lz = ilog2(t->tile[2]);
    if (lx < 0 || ly < 0 || lz < 2 || lx + ly + lz > 14 || t->wg_per_cu < 0 || t->wg_per_cu > 32 ||
        t->lds_cells < -1 || t->lds_cells > lds_cells_cap(2) || t->lds_format < 0 ||
        t->lds_format > 1)
        return CTAUG_EINVAL;
    TL = {lx, ly, lz};
    return CTAUG_OK;
}

ctaug_status job_from_public(const ctaug_job &j, const Tiling &TL, FwdJob &J)
{
    const bool has_lbl = j.lbl_in.data != nullptr;
    const bool has_photo = !(j.photo.flags & CTAUG_PHOTO_NONE);
    ctaug_status st = make_job(&j.img_in, has_lbl ? &j.lbl_in : nullptr, j.M, nullptr, false,
                               j.fill, j.label_fill, has_photo ? &j.photo : nullptr, &j.img_out,
                               has_lbl ? &j.lbl_out : nullptr, TL, J);
    if (st != CTAUG_OK || !j.ctrl)
        return st;
    if (!grid_valid(j.grid))
        return CTAUG_ESHAPE;
    J.ctrl = j.ctrl;
    J.bs = bspline_geom(j.grid, j.img_out.dim);
    return CTAUG_OK;
}

void destroy_graph(ctaug_batch_plan *p)
{
    if (p->exec) {
        (void)hipGraphExecDestroy(p->exec);
        p->exec = nullptr;
    }
}

// Recompute tile counts / prefix sums / grid for the plan's tiling and upload
// the prefix and job tables (synchronous: only at creation and retuning).
// Both uploads wait for the plan's last launch, run or replay first, so that
// no kernel still running reads a prefix table of one tiling beside a job
// table of another; afterwards the device tables agree with the new tiling,
// so a later run() (no upload) decodes tiles consistently.
ctaug_status apply_tiling(ctaug_batch_plan *p, const ctaug_tuning &t)
{
    Tiling TL;
    ctaug_status st = tiling_of(&t, TL);
    if (st != CTAUG_OK)
        return st;
    if (p->spline)                      // B-spline jobs: displacement tiles, FP32 cells
        TL = kDispTiling;
    std::vector<int32_t> prefix(p->n + 1, 0);
    int64_t total = 0;
    p->elem_bytes = (t.lds_format == 1 && p->all_i16 && !p->spline) ? 2 : 4;
    for (int i = 0; i < p->n; ++i) {
        set_tiles(p->jobs[i], TL);
        if (p->elem_bytes == 2)
            p->jobs[i].flags |= kFlagLds16;
        else
            p->jobs[i].flags &= ~kFlagLds16;
        prefix[i] = (int32_t)total;
        total += (int64_t)p->jobs[i].tiles_x * p->jobs[i].tiles_y * p->jobs[i].tiles_z;
    }
    if (total > (int64_t)kMaxElems)
        return CTAUG_ESHAPE;
    prefix[p->n] = (int32_t)total;
    int32_t cells = t.lds_cells < 0 ? 0 : t.lds_cells;
    if (p->spline) {
        cells = lds_cells_for(kDispLdsCells, 4);
    } else if (t.lds_cells == 0) {
        // the largest footprint of the current jobs, with headroom for later
        // updates; tiles that still exceed it take the direct-gather path
        int64_t need = 0;
        for (int i = 0; i < p->n; ++i)
            need = std::max<int64_t>(need, footprint_cells_bound(p->jobs[i], TL));
        cells = lds_cells_for((int32_t)std::min<int64_t>(need + need / 4 + 64, 1 << 20),
                              p->elem_bytes);
    } else if (cells > lds_cells_cap(p->elem_bytes)) {
        return CTAUG_EINVAL;
    }
    for (int i = 0; i < p->n; ++i)
        set_subtiles(p->jobs[i], TL, cells);
    if (p->upload_recorded && hipEventSynchronize(p->upload_done) != hipSuccess)
        return CTAUG_EHIP;
    std::memcpy(p->staging, p->jobs.data(), sizeof(FwdJob) * p->n);
    if (hipMemcpy(p->prefix_dev, prefix.data(), sizeof(int32_t) * (p->n + 1),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->table, p->staging, sizeof(FwdJob) * p->n, hipMemcpyHostToDevice) !=
            hipSuccess)
        return CTAUG_EHIP;
    p->TL = TL;
    p->tune = t;
    p->tune.lds_cells = t.lds_cells < 0 && !p->spline ? -1 : cells;
    if (p->spline) {
        p->tune.tile[0] = 1 << TL.lx;
        p->tune.tile[1] = 1 << TL.ly;
        p->tune.tile[2] = 1 << TL.lz;
        p->tune.lds_format = 0;
    }
    p->lds_cells = cells;
    p->total = (int32_t)total;
    ++p->generation;                    // descriptors prepared for the old tiling are stale
    const int64_t tiles8 = 8 * (int64_t)xcd_slots((int)total);
    int64_t grid = t.wg_per_cu > 0 ? (int64_t)p->num_cu * t.wg_per_cu : tiles8;
    grid = std::max<int64_t>(8, (grid / 8) * 8);
    p->grid = (int32_t)std::min<int64_t>(grid, std::max<int64_t>(tiles8, 8));
    destroy_graph(p);
    return CTAUG_OK;
}

int batch_mode(const ctaug_batch_plan *p)
{
    if (p->spline)
        return p->all_i16 ? kBatchSplineI16 : p->all_f32 ? kBatchSplineF32 : kBatchSplineMixed;
    if (p->all_i16)
        return p->elem_bytes == 2 ? kBatchI16I16 : kBatchI16F32;
    return p->all_f32 ? kBatchF32 : kBatchMixed;
}

ctaug_status enqueue(ctaug_batch_plan *p, hipStream_t s)
{
    if (hipMemcpyAsync(p->table, p->staging, sizeof(FwdJob) * p->n, hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return CTAUG_EHIP;
    return hip_status(
        launch_warp_batch(p->table, p->prefix_dev, p->n, p->total, p->grid, p->TL, p->lds_cells,
                          p->elem_bytes, batch_mode(p), p->aligned, s));
}

}  // namespace

// ---------------------------------------------------------------------------
// Autotune cache: the launch shape ctaug_batch_plan_autotune chose, keyed by
// the device (architecture name, compute units) and a class of batch shapes
// (input dtype specialisation, job count and largest output rounded to powers
// of two, labels / noise present).  ctaug_batch_plan_create consults it when
// given no tuning; save / load persist it as text.  The only mutable state of
// the library besides plans and pipelines; guarded by a mutex.
// ---------------------------------------------------------------------------

namespace {

struct TuneKey {
    std::string arch;
    int32_t cus, mode, njobs_log, vox_log, flags;
    bool operator==(const TuneKey &o) const
    {
        return arch == o.arch && cus == o.cus && mode == o.mode && njobs_log == o.njobs_log &&
               vox_log == o.vox_log && flags == o.flags;
    }
};

std::mutex g_cache_mu;
std::vector<std::pair<TuneKey, ctaug_tuning>> g_cache;

int ceil_log2(int64_t v)
{
    int l = 0;
    while (((int64_t)1 << l) < v)
        ++l;
    return l;
}

// Key of a batch: mode 0 mixed, 1 all int16, 3 all FP32 (the launch's dtype
// specialisations), +8 for B-spline jobs.
TuneKey tune_key(const std::string &arch, int cus, const std::vector<FwdJob> &jobs, bool spline)
{
    bool all_i16 = true, all_f32 = true, labels = false, noise = false;
    int64_t vox = 1;
    for (const FwdJob &J : jobs) {
        all_i16 = all_i16 && J.dtype == kI16;
        all_f32 = all_f32 && J.dtype == kF32;
        labels = labels || (J.flags & kFlagLabels);
        noise = noise || (J.flags & kFlagNoise);
        vox = std::max<int64_t>(vox, (int64_t)J.ox * J.oy * J.oz);
    }
    TuneKey k;
    k.arch = arch;
    k.cus = cus;
    k.mode = (all_i16 ? 1 : all_f32 ? 3 : 0) + (spline ? 8 : 0);
    k.njobs_log = ceil_log2((int64_t)jobs.size());
    k.vox_log = ceil_log2(vox);
    k.flags = (labels ? 1 : 0) | (noise ? 2 : 0);
    return k;
}

bool cache_find(const TuneKey &k, ctaug_tuning &out)
{
    std::lock_guard<std::mutex> lock(g_cache_mu);
    for (const auto &e : g_cache)
        if (e.first == k) {
            out = e.second;
            return true;
        }
    return false;
}

void cache_put(const TuneKey &k, const ctaug_tuning &t)
{
    std::lock_guard<std::mutex> lock(g_cache_mu);
    for (auto &e : g_cache)
        if (e.first == k) {
            e.second = t;
            return;
        }
    g_cache.emplace_back(k, t);
}

bool device_id(std::string &arch, int &cus)
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return false;
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos)
        arch.resize(colon);            // gfx950, without target features
    cus = prop.multiProcessorCount;
    return true;
}

constexpr const char *kCacheHeader = "# ctaug autotune cache v1";

}  // namespace

extern "C" ctaug_status ctaug_autotune_cache_save(const char *path)
{
    if (!path)
        return CTAUG_EINVAL;
    std::vector<std::pair<TuneKey, ctaug_tuning>> snap;
    {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        snap = g_cache;
    }
    FILE *f = std::fopen(path, "w");
    if (!f)
        return CTAUG_EINVAL;
    bool ok = std::fprintf(f, "%s\n", kCacheHeader) > 0;
    for (const auto &e : snap) {
        const TuneKey &k = e.first;
        const ctaug_tuning &t = e.second;
        ok = ok && std::fprintf(f, "%s %d %d %d %d %d %d %d %d %d %d %d\n", k.arch.c_str(), k.cus,
                                k.mode, k.njobs_log, k.vox_log, k.flags, t.tile[0], t.tile[1],
                                t.tile[2], t.wg_per_cu, t.lds_cells, t.lds_format) > 0;
    }
    ok = (std::fclose(f) == 0) && ok;
    return ok ? CTAUG_OK : CTAUG_EINVAL;
}

extern "C" ctaug_status ctaug_autotune_cache_load(const char *path, int32_t *n_entries)
{
    if (!path)
        return CTAUG_EINVAL;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return CTAUG_EINVAL;
    std::vector<std::pair<TuneKey, ctaug_tuning>> read;
    char line[512];
    bool ok = std::fgets(line, sizeof line, f) != nullptr &&
              std::strncmp(line, kCacheHeader, std::strlen(kCacheHeader)) == 0;
    while (ok && std::fgets(line, sizeof line, f)) {
        if (line[0] == '\n' || line[0] == '#')
            continue;
        char arch[64];
        TuneKey k;
        ctaug_tuning t;
        const int got = std::sscanf(line, "%63s %d %d %d %d %d %d %d %d %d %d %d", arch, &k.cus,
                                    &k.mode, &k.njobs_log, &k.vox_log, &k.flags, &t.tile[0],
                                    &t.tile[1], &t.tile[2], &t.wg_per_cu, &t.lds_cells,
                                    &t.lds_format);
        Tiling TL;
        ok = got == 12 && tiling_of(&t, TL) == CTAUG_OK && k.cus > 0;
        k.arch = arch;
        if (ok)
            read.emplace_back(k, t);
    }
    std::fclose(f);
    if (!ok)
        return CTAUG_EINVAL;           // nothing merged from a malformed file
    for (const auto &e : read)
        cache_put(e.first, e.second);
    if (n_entries)
        *n_entries = (int32_t)read.size();
    return CTAUG_OK;
}

extern "C" ctaug_status ctaug_autotune_cache_clear(void)
{
    std::lock_guard<std::mutex> lock(g_cache_mu);
    g_cache.clear();
    return CTAUG_OK;
}

extern "C" ctaug_status ctaug_autotune_cache_lookup(const ctaug_job *jobs, int32_t n_jobs,
                                                    ctaug_tuning *out, int32_t *found)
{
    if (!jobs || !out || !found || n_jobs <= 0 || n_jobs > (1 << 20))
        return CTAUG_EINVAL;
    std::vector<FwdJob> js(n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
        if ((jobs[i].ctrl != nullptr) != (jobs[0].ctrl != nullptr))
            return CTAUG_EINVAL;
        const ctaug_status st = job_from_public(jobs[i], kDefaultTiling, js[i]);
        if (st != CTAUG_OK)
            return st;
    }
    std::string arch;
    int cus = 0;
    if (!device_id(arch, cus))
        return CTAUG_ENODEV;
    *found = cache_find(tune_key(arch, cus, js, jobs[0].ctrl != nullptr), *out) ? 1 : 0;
    return CTAUG_OK;
}

extern "C" ctaug_status ctaug_batch_plan_destroy(ctaug_batch_plan *p)
{
    if (!p)
        return CTAUG_EINVAL;
    destroy_graph(p);
    if (p->upload_done)
        (void)hipEventDestroy(p->upload_done);
    if (p->staging)
        (void)hipHostFree(p->staging);
    if (p->table)
        (void)hipFree(p->table);
    if (p->prefix_dev)
        (void)hipFree(p->prefix_dev);
    delete p;
    return CTAUG_OK;
}

extern "C" ctaug_status ctaug_batch_plan_create(const ctaug_job *jobs, int32_t n_jobs,
                                                const ctaug_tuning *tune, ctaug_batch_plan **out)
{
    if (!jobs || !out || n_jobs <= 0 || n_jobs > (1 << 20))
        return CTAUG_EINVAL;
    Tiling TL;
    ctaug_status st = tiling_of(tune, TL);
    if (st != CTAUG_OK)
        return st;
    for (int i = 1; i < n_jobs; ++i)
        if ((jobs[i].ctrl != nullptr) != (jobs[0].ctrl != nullptr))
            return CTAUG_EINVAL;           // affine and B-spline jobs in one plan
    if (jobs[0].ctrl)
        TL = kDispTiling;
    ctaug_batch_plan *p = new (std::nothrow) ctaug_batch_plan();
    if (!p)
        return CTAUG_EINVAL;
    p->n = n_jobs;
    p->spline = jobs[0].ctrl != nullptr;
    p->jobs.resize(n_jobs);
    p->out_dims.resize(3 * (size_t)n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
        st = job_from_public(jobs[i], TL, p->jobs[i]);
        if (st != CTAUG_OK) {
            delete p;
            return st;
        }
        p->out_dims[3 * i + 0] = p->jobs[i].ox;
        p->out_dims[3 * i + 1] = p->jobs[i].oy;
        p->out_dims[3 * i + 2] = p->jobs[i].oz;
        p->aligned = p->aligned && p->jobs[i].oz % 4 == 0;
        if (p->jobs[i].dtype != CTAUG_I16)
            p->all_i16 = false;
        if (p->jobs[i].dtype != CTAUG_F32)
            p->all_f32 = false;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete p;
        return CTAUG_ENODEV;
    }
    p->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    p->arch = prop.gcnArchName;
    if (p->arch.find(':') != std::string::npos)
        p->arch.resize(p->arch.find(':'));
    if (hipHostMalloc(reinterpret_cast<void **>(&p->staging), sizeof(FwdJob) * n_jobs,
                      hipHostMallocDefault) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&p->table), sizeof(FwdJob) * n_jobs) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&p->prefix_dev), sizeof(int32_t) * (n_jobs + 1)) !=
            hipSuccess ||
        hipEventCreateWithFlags(&p->upload_done, hipEventDisableTiming) != hipSuccess) {
        ctaug_batch_plan_destroy(p);
        return CTAUG_EHIP;
    }
    // no tuning given: the cached autotune result for this device and batch
    // class, else the default shape
    ctaug_tuning t = ctaug_tuning{{8, 16, 16}, 0, 0, 0};
    if (tune)
        t = *tune;
    else
        (void)cache_find(tune_key(p->arch, p->num_cu, p->jobs, p->spline), t);
    st = apply_tiling(p, t);
    if (st != CTAUG_OK) {
        ctaug_batch_plan_destroy(p);
        return st;
    }
    *out = p;
    return CTAUG_OK;
}

namespace {

// Validate jobs against plan p and build their descriptors for its current
// tiling (sub-tile shapes included): no device work, no waiting.
ctaug_status prepare_jobs(const ctaug_batch_plan *p, const ctaug_job *jobs,
                          std::vector<FwdJob> &next)
{
    next.resize(p->n);
    for (int i = 0; i < p->n; ++i) {
        if ((jobs[i].ctrl != nullptr) != p->spline)
            return CTAUG_EINVAL;           // the plan holds only affine or only B-spline jobs
        ctaug_status st = job_from_public(jobs[i], p->TL, next[i]);
        if (st != CTAUG_OK)
            return st;
        if (next[i].ox != p->out_dims[3 * i] || next[i].oy != p->out_dims[3 * i + 1] ||
            next[i].oz != p->out_dims[3 * i + 2])
            return CTAUG_ESHAPE;
        if (next[i].dtype != CTAUG_I16 && p->elem_bytes < 4)
            return CTAUG_EDTYPE;           // the LDS reservation was sized for int16 cells
        if ((p->all_i16 && next[i].dtype != CTAUG_I16) ||
            (p->all_f32 && next[i].dtype != CTAUG_F32))
            return CTAUG_EDTYPE;           // the launch was specialised for the creation dtypes
    }
    for (int i = 0; i < p->n; ++i) {
        if (p->elem_bytes == 2)
            next[i].flags |= kFlagLds16;
        set_subtiles(next[i], p->TL, p->lds_cells);
    }
    return CTAUG_OK;
}

// Wait until the plan's last launch / run / replay no longer reads staging or
// table, then install the descriptors.
ctaug_status commit_jobs(ctaug_batch_plan *p, const std::vector<FwdJob> &next)
{
    if (p->upload_recorded && hipEventSynchronize(p->upload_done) != hipSuccess)
        return CTAUG_EHIP;
    p->jobs = next;
    std::memcpy(p->staging, p->jobs.data(), sizeof(FwdJob) * p->n);
    return CTAUG_OK;
}

}  // namespace

struct ctaug_batch_jobs {
    const ctaug_batch_plan *plan = nullptr;
    uint64_t generation = 0;            // the plan's tiling generation at prepare time
    std::vector<FwdJob> jobs;
};

extern "C" ctaug_status ctaug_batch_plan_update(ctaug_batch_plan *p, const ctaug_job *jobs)
{
    if (!p || !jobs)
        return CTAUG_EINVAL;
    std::vector<FwdJob> next;
    const ctaug_status st = prepare_jobs(p, jobs, next);
    return st != CTAUG_OK ? st : commit_jobs(p, next);
}

extern "C" ctaug_status ctaug_batch_plan_prepare(ctaug_batch_plan *p, const ctaug_job *jobs,
                                                 ctaug_batch_jobs **out)
{
    if (!p || !jobs || !out)
        return CTAUG_EINVAL;
    ctaug_batch_jobs *b = new (std::nothrow) ctaug_batch_jobs();
    if (!b)
        return CTAUG_EINVAL;
    const ctaug_status st = prepare_jobs(p, jobs, b->jobs);
    if (st != CTAUG_OK) {
        delete b;
        return st;
    }
    b->plan = p;
    b->generation = p->generation;
    *out = b;
    return CTAUG_OK;
}

extern "C" ctaug_status ctaug_batch_plan_update_prepared(ctaug_batch_plan *p,
                                                         const ctaug_batch_jobs *b)
{
    if (!p || !b || b->plan != p || b->generation != p->generation)
        return CTAUG_EINVAL;
    return commit_jobs(p, b->jobs);
}

extern "C" ctaug_status ctaug_batch_jobs_destroy(ctaug_batch_jobs *b)
{
    if (!b)
        return CTAUG_EINVAL;
    delete b;
    return CTAUG_OK;
}

extern "C" ctaug_status ctaug_batch_plan_launch(ctaug_batch_plan *p, void *stream)
{
    if (!p)
        return CTAUG_EINVAL;
    hipStream_t s = as_stream(stream);
    ctaug_status st = enqueue(p, s);
    if (st != CTAUG_OK)
        return st;
    if (hipEventRecord(p->upload_done, s) != hipSuccess)
        return CTAUG_EHIP;
    p->upload_recorded = true;
    return CTAUG_OK;
}

extern "C" ctaug_status ctaug_batch_plan_run(ctaug_batch_plan *p, void *stream)
{
    if (!p || !p->upload_recorded)
        return CTAUG_EINVAL;
    hipStream_t s = as_stream(stream);
    ctaug_status st = hip_status(launch_warp_batch(p->table, p->prefix_dev, p->n, p->total,
                                                   p->grid, p->TL, p->lds_cells, p->elem_bytes,
                                                   batch_mode(p), p->aligned, s));
    if (st != CTAUG_OK)
        return st;
    // a later update must also wait for this launch's reads of the table
    return hip_status(hipEventRecord(p->upload_done, s));
}

extern "C" ctaug_status ctaug_copy(const void *src, void *dst, size_t bytes, void *stream)
{
    if (bytes == 0)
        return CTAUG_OK;
    if (!src || !dst)
        return CTAUG_EINVAL;
    return hip_status(launch_copy(src, dst, bytes, as_stream(stream)));
}

extern "C" ctaug_status ctaug_batch_plan_capture(ctaug_batch_plan *p, void *stream)
{
    if (!p)
        return CTAUG_EINVAL;
    hipStream_t s = as_stream(stream);
    if (!s)
        return CTAUG_EINVAL;             // the null stream cannot be captured
    destroy_graph(p);
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return CTAUG_EHIP;
    ctaug_status st = enqueue(p, s);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (st != CTAUG_OK || e != hipSuccess) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return st != CTAUG_OK ? st : CTAUG_EHIP;
    }
    e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        p->exec = nullptr;
        return CTAUG_EHIP;
    }
    return CTAUG_OK;
}

extern "C" ctaug_status ctaug_batch_plan_replay(ctaug_batch_plan *p, void *stream)
{
    if (!p || !p->exec)
        return CTAUG_EINVAL;
    hipStream_t s = as_stream(stream);
    if (hipGraphLaunch(p->exec, s) != hipSuccess)
        return CTAUG_EHIP;
    if (hipEventRecord(p->upload_done, s) != hipSuccess)
        return CTAUG_EHIP;
    p->upload_recorded = true;
    return CTAUG_OK;
}

extern "C" ctaug_status ctaug_batch_plan_get_tuning(const ctaug_batch_plan *p, ctaug_tuning *out)
{
    if (!p || !out)
        return CTAUG_EINVAL;
    *out = p->tune;
    return CTAUG_OK;
}

extern "C" ctaug_status ctaug_batch_plan_autotune(ctaug_batch_plan *p, const ctaug_tuning *cand,
                                                  int32_t n_cand, int32_t reps, void *stream,
                                                  ctaug_tuning *best, float *times_ms)
{
    if (!p || !cand || n_cand <= 0 || reps <= 0)
        return CTAUG_EINVAL;
    for (int i = 0; i < n_cand; ++i) {
        Tiling TL;
        if (tiling_of(&cand[i], TL) != CTAUG_OK)
            return CTAUG_EINVAL;
    }
    hipStream_t s = as_stream(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return CTAUG_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return CTAUG_EHIP;
    }
    const ctaug_tuning original = p->tune;
    int best_i = -1;
    float best_ms = 0.0f;
    ctaug_status st = CTAUG_OK;
    for (int i = 0; i < n_cand && st == CTAUG_OK; ++i) {
        st = apply_tiling(p, cand[i]);
        if (st != CTAUG_OK)
            break;
        st = ctaug_batch_plan_launch(p, stream);           // warm-up
        if (st != CTAUG_OK)
            break;
        if (hipEventRecord(e0, s) != hipSuccess) {
            st = CTAUG_EHIP;
            break;
        }
        for (int r = 0; r < reps && st == CTAUG_OK; ++r)
            st = ctaug_batch_plan_launch(p, stream);
        if (st != CTAUG_OK)
            break;
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = CTAUG_EHIP;
            break;
        }
        ms /= (float)reps;
        if (times_ms)
            times_ms[i] = ms;
        if (best_i < 0 || ms < best_ms) {
            best_i = i;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != CTAUG_OK) {
        (void)apply_tiling(p, original);
        return st;
    }
    st = apply_tiling(p, cand[best_i]);
    if (st != CTAUG_OK)
        return st;
    cache_put(tune_key(p->arch, p->num_cu, p->jobs, p->spline), cand[best_i]);
    if (best)
        *best = cand[best_i];
    return CTAUG_OK;
}

// ---------------------------------------------------------------------------
// Host-to-device FIFO: pinned host slots filled by the caller, device slots
// read by the warps, a copy stream and a compute stream.  Slot s is reused
// only after the warp that read it has finished (event done[s]); the copy of
// slot s+1 proceeds on the copy engine while the warp of slot s runs.
// ---------------------------------------------------------------------------

struct ctaug_pipeline {
    int32_t depth = 0;
    size_t slot_bytes = 0;
    std::vector<void *> host;          // pinned (hipHostMalloc)
    std::vector<void *> dev;
    std::vector<hipEvent_t> copied;    // H2D of the slot's volume finished
    std::vector<hipEvent_t> done;      // the warp reading the slot finished
    std::vector<char> pending;         // done[] recorded and not yet waited for
    hipStream_t copy = nullptr;
    hipStream_t compute = nullptr;
    int32_t next = 0;                  // slot the next acquire hands out
    int32_t held = -1;                 // slot handed out and not yet submitted
};

namespace {

void pipeline_free(ctaug_pipeline *p)
{
    if (p->copy)
        (void)hipStreamSynchronize(p->copy);
    if (p->compute)
        (void)hipStreamSynchronize(p->compute);
    for (void *h : p->host)
        if (h)
            (void)hipHostFree(h);
    for (void *d : p->dev)
        if (d)
            (void)hipFree(d);
    for (hipEvent_t e : p->copied)
        if (e)
            (void)hipEventDestroy(e);
    for (hipEvent_t e : p->done)
        if (e)
            (void)hipEventDestroy(e);
    if (p->copy)
        (void)hipStreamDestroy(p->copy);
    if (p->compute)
        (void)hipStreamDestroy(p->compute);
    delete p;
}

// Byte range of a volume's data inside [base, base + size), as an offset.
bool slot_offset(const ctaug_vol *v, const void *base, size_t size, size_t &off, size_t &bytes)
{
    const size_t esz = v->dtype == CTAUG_F32 ? 4 : v->dtype == CTAUG_I16 ? 2 : 1;
    bytes = (size_t)nelem(v->dim) * esz;
    const uintptr_t b = reinterpret_cast<uintptr_t>(base), d = reinterpret_cast<uintptr_t>(v->data);
    if (bytes == 0)
        return true;
    if (d < b || d - b > size || bytes > size - (d - b))
        return false;
    off = (size_t)(d - b);
    return true;
}

}  // namespace

extern "C" ctaug_status ctaug_pipeline_create(int32_t depth, size_t slot_bytes,
                                              ctaug_pipeline **out)
{
    if (!out || depth < 2 || depth > 64 || slot_bytes == 0)
        return CTAUG_EINVAL;
    ctaug_pipeline *p = new (std::nothrow) ctaug_pipeline();
    if (!p)
        return CTAUG_EINVAL;
    p->depth = depth;
    p->slot_bytes = slot_bytes;
    p->host.assign(depth, nullptr);
    p->dev.assign(depth, nullptr);
    p->copied.assign(depth, nullptr);
    p->done.assign(depth, nullptr);
    p->pending.assign(depth, 0);
    bool ok = hipStreamCreateWithFlags(&p->copy, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&p->compute, hipStreamNonBlocking) == hipSuccess;
    for (int i = 0; ok && i < depth; ++i)
        ok = hipHostMalloc(&p->host[i], slot_bytes, hipHostMallocDefault) == hipSuccess &&
             hipMalloc(&p->dev[i], slot_bytes) == hipSuccess &&
             hipEventCreateWithFlags(&p->copied[i], hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&p->done[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        pipeline_free(p);
        return CTAUG_EHIP;
    }
    *out = p;
    return CTAUG_OK;
}

extern "C" ctaug_status ctaug_pipeline_acquire(ctaug_pipeline *p, void **host_slot)
{
    if (!p || !host_slot || p->held >= 0)
        return CTAUG_EINVAL;
    const int32_t s = p->next;
    if (p->pending[s]) {
        if (hipEventSynchronize(p->done[s]) != hipSuccess)
            return CTAUG_EHIP;
        p->pending[s] = 0;
    }
    p->held = s;
    *host_slot = p->host[s];
    return CTAUG_OK;
}

extern "C" ctaug_status ctaug_pipeline_submit(ctaug_pipeline *p, const ctaug_vol *img_host,
                                              const ctaug_vol *lbl_host, const float M[12],
                                              float fill, int32_t label_fill,
                                              const ctaug_photo *photo, ctaug_vol *img_out,
                                              ctaug_vol *lbl_out)
{
    if (!p || p->held < 0 || !img_host)
        return CTAUG_EINVAL;
    if (!is_dense(img_host) || (lbl_host && !is_dense(lbl_host)))
        return CTAUG_ESHAPE;           // slot volumes are copied as dense byte ranges
    const int32_t s = p->held;
    size_t io = 0, ib = 0, lo = 0, lb = 0;
    if (!slot_offset(img_host, p->host[s], p->slot_bytes, io, ib))
        return CTAUG_EINVAL;
    if (lbl_host && !slot_offset(lbl_host, p->host[s], p->slot_bytes, lo, lb))
        return CTAUG_EINVAL;
    // the same volumes at the device slot's addresses
    char *dbase = static_cast<char *>(p->dev[s]);
    ctaug_vol img_dev = *img_host, lbl_dev{};
    img_dev.data = ib ? dbase + io : nullptr;
    if (lbl_host) {
        lbl_dev = *lbl_host;
        lbl_dev.data = lb ? dbase + lo : nullptr;
    }
    FwdJob J;
    ctaug_status st = make_job(&img_dev, lbl_host ? &lbl_dev : nullptr, M, nullptr, false, fill,
                               label_fill, photo, img_out, lbl_out, kDefaultTiling, J);
    if (st != CTAUG_OK)
        return st;
    const char *hbase = static_cast<const char *>(p->host[s]);
    hipError_t e = hipSuccess;
    if (ib)
        e = hipMemcpyAsync(dbase + io, hbase + io, ib, hipMemcpyHostToDevice, p->copy);
    if (e == hipSuccess && lb)
        e = hipMemcpyAsync(dbase + lo, hbase + lo, lb, hipMemcpyHostToDevice, p->copy);
    if (e == hipSuccess)
        e = hipEventRecord(p->copied[s], p->copy);
    if (e == hipSuccess)
        e = hipStreamWaitEvent(p->compute, p->copied[s], 0);
    if (e == hipSuccess && !empty(J))
        e = launch_warp_single(J, kDefaultTiling, p->compute);
    if (e == hipSuccess)
        e = hipEventRecord(p->done[s], p->compute);
    if (e != hipSuccess)
        return CTAUG_EHIP;
    p->pending[s] = 1;
    p->held = -1;
    p->next = (s + 1) % p->depth;
    return CTAUG_OK;
}

extern "C" ctaug_status ctaug_pipeline_stream(ctaug_pipeline *p, void **stream)
{
    if (!p || !stream)
        return CTAUG_EINVAL;
    *stream = p->compute;
    return CTAUG_OK;
}

extern "C" ctaug_status ctaug_pipeline_sync(ctaug_pipeline *p)
{
    if (!p)
        return CTAUG_EINVAL;
    if (hipStreamSynchronize(p->copy) != hipSuccess ||
        hipStreamSynchronize(p->compute) != hipSuccess)
        return CTAUG_EHIP;
    std::fill(p->pending.begin(), p->pending.end(), 0);
    return CTAUG_OK;
}

extern "C" ctaug_status ctaug_pipeline_destroy(ctaug_pipeline *p)
{
    if (!p)
        return CTAUG_EINVAL;
    pipeline_free(p);
    return CTAUG_OK;
}
