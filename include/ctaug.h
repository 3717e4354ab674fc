/*
 * ctaug.h -- C ABI of the MI355X (gfx950) CT data-augmentation library.
 *
 * The library implements the GPU augmentation path of Rister et al., "CT organ
 * segmentation using GPU data augmentation, unsupervised labels and IOU loss"
 * (arXiv:1811.11226), Sec. "GPU-accelerated data augmentation": a 3-D CT
 * volume is resampled through a random affine coordinate map x' = A x + b
 * with trilinear interpolation, the label volume is warped through the same
 * map by nearest-neighbour lookup, and photometric transforms and generated
 * Gaussian noise are applied, all in one pass per output voxel.  Additions
 * beyond the paper: gain/offset/gamma, a dense or cubic-B-spline displacement
 * added to the affine map, adjoints (image, affine parameters, displacement,
 * control grid), and a batched launch over volumes of uneven sizes.
 *
 * Conventions shared by every call
 * ---------------------------------
 *  - Volumes are dense C-order arrays [X][Y][Z] (z fastest).  Output voxel
 *    p = (x, y, z) has linear index v = (x*Y + y)*Z + z.
 *  - Data pointers named "device" are HIP device pointers owned by the caller;
 *    the library never frees or retains them.  Small parameter blocks (the
 *    3x4 matrix, photometric parameters, dimension triples) are host pointers
 *    read before the call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every compute call is asynchronous and stream-ordered; none synchronises.
 *  - Arguments are validated before anything is enqueued.  On any error the
 *    call returns a nonzero ctaug_status and leaves every output untouched.
 *    No exception crosses the ABI and the library never prints.
 *  - The only calls that allocate device or pinned memory are
 *    ctaug_batch_plan_create and ctaug_pipeline_create (owned by the plan or
 *    pipeline, freed by its destroy call); compute calls take caller
 *    workspace.
 *  - Empty volumes (a zero dimension) are valid and make a call a no-op.
 *  - The sampling coordinate of output voxel p is, per axis i,
 *        q_i = fmaf(A_i2, z, fmaf(A_i1, y, fmaf(A_i0, x, b_i)))
 *    in FP32 (plus u_i(p) as one FP32 addition when a displacement is given),
 *    so that results are reproducible bit for bit across launch shapes.
 *    Integer coordinates are voxel centres.  M = [A|b] maps OUTPUT voxel
 *    coordinates to INPUT voxel coordinates (I_out(p) = I_in(A p + b)).
 */
#ifndef CTAUG_H
#define CTAUG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CTAUG_OK = 0,
    CTAUG_EINVAL = 1,      /* null pointer, non-finite parameter, bad flag, ... */
    CTAUG_EDTYPE = 2,      /* unsupported dtype for this argument */
    CTAUG_ESHAPE = 3,      /* negative / inconsistent / too large dimensions */
    CTAUG_EWORKSPACE = 4,  /* workspace missing or smaller than required */
    CTAUG_EHIP = 5,        /* a HIP runtime call or kernel launch failed */
    CTAUG_ENODEV = 6       /* no usable gfx950 device */
} ctaug_status;

typedef enum {
    CTAUG_F32 = 0,         /* float32 */
    CTAUG_I16 = 1,         /* int16 (e.g. 12-bit CT in HU) */
    CTAUG_I8 = 2           /* int8 labels */
} ctaug_dtype;

/* A volume.  data: device pointer to element (0,0,0); dim: X, Y, Z (each
 * >= 0); stride: element strides along X, Y, Z.  stride = {0, 0, 0} means
 * dense C order ({Y*Z, Z, 1}).
 *
 * Strided volumes (e.g. a random training crop, Sec. "Pre- and
 * post-processing", passed as a view of the whole scan) are accepted for the
 * INPUT image and label of the warps, their batch jobs and the image read by
 * the adjoints; every other volume argument must be dense (ESHAPE
 * otherwise).  A strided volume keeps z contiguous: stride[2] == 1,
 * stride[1] >= dim[2], and stride[0] a multiple of stride[1] with
 * stride[0] / stride[1] >= dim[1] (the layout of any box cut out of a dense
 * parent volume).  A label input must have its image's strides.
 *
 * Size limits (ESHAPE beyond them):
 *  - every volume: at most 2^31 - 1 elements, and its extent
 *    (X-1) stride[0] + (Y-1) stride[1] + Z at most 2^31 - 1 (FP32 input
 *    images: 2^30 - 1, so that their byte extent fits a 32-bit buffer range);
 *  - gathered inputs (image and labels of the warps, the adjoints' image):
 *    their offsets are formed with 24-bit multiplies, so the row count
 *    (X-1) stride[0]/stride[1] + Y must be at most 2^24 and the row pitch
 *    stride[1] below 2^24 (dense: X*Y <= 2^24 and Z < 2^24). */
typedef struct {
    void *data;
    int32_t dtype;         /* ctaug_dtype */
    int32_t reserved;      /* must be 0 */
    int64_t dim[3];
    int64_t stride[3];     /* elements; {0, 0, 0} = dense */
} ctaug_vol;

#define CTAUG_PHOTO_WINDOW 1u   /* apply window [win_lo, win_hi] -> [0,1] and gamma */
#define CTAUG_PHOTO_OCCLUDE 2u  /* random occlusion of the output slab occ_lo <= z <= occ_hi */
#define CTAUG_PHOTO_NONE 0x80000000u  /* in a job descriptor: no photometric chain */

/* Photometric parameters of one volume (Sec. "GPU-accelerated data
 * augmentation", occlusion, noise and window paragraphs; gain, offset and
 * gamma are additions).  For each output voxel p = (x, y, z) with
 * interpolated value V:
 *     if OCCLUDE and occ_lo <= z <= occ_hi (FP32 comparisons): V = 0
 *         (the I_occ equation, its slab read as a closed interval on the
 *         output's third axis; labels are not occluded)
 *     v = gain * V + offset
 *     v = v + sigma * n(v_index)          n ~ N(0,1), see ctaug_noise
 *     if WINDOW: t = min(max((v - win_lo) / (win_hi - win_lo), 0), 1)
 *                out = t^gamma  (0^gamma = 0)
 *     else       out = v  (Hounsfield units)
 * Requirements: all values finite; sigma >= 0; gamma > 0; win_hi > win_lo
 * when WINDOW is set.  sigma == 0 adds no noise (the result is exactly the
 * noiseless value).  occ_lo / occ_hi are read only with OCCLUDE (an empty
 * slab, occ_hi < occ_lo, occludes nothing). */
typedef struct {
    float gain, offset, sigma, win_lo, win_hi, gamma;
    uint32_t flags;        /* CTAUG_PHOTO_* bits */
    uint32_t volume_id;    /* Philox counter word 2 */
    uint64_t seed;         /* Philox key */
    float occ_lo, occ_hi;  /* occluded output slab (OCCLUDE) */
} ctaug_photo;

/* Raw draws of the random affine transform (Sec. "GPU-accelerated data
 * augmentation", first paragraph and footnote; crop from Sec. "Pre- and
 * post-processing").  All FP64. */
typedef struct {
    double rot[3];         /* rotation angles about x, y, z (radians) */
    double scale[3];       /* scale factors along x, y, z */
    double shear[3];       /* h_xy, h_xz, h_yz of [[1,h_xy,h_xz],[0,1,h_yz],[0,0,1]] */
    double reflect[3];     /* 0 or 1: reflect about the centre plane of axis i */
    double generic[9];     /* generic 3x3 matrix G, row-major (identity if unused) */
    double disp[3];        /* displacement d of the volume centre (input voxels) */
    double crop[3];        /* crop shift k (input voxels) */
} ctaug_affine_params;

/* ------------------------------------------------------------------------ */
/* Host-side helpers                                                         */
/* ------------------------------------------------------------------------ */

const char *ctaug_status_string(ctaug_status s);
/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int ctaug_version(void);

/* Transform composition (the paper composes rotation, scaling, shearing,
 * reflection and a generic affine, and sets b = c + d - A c so that the
 * volume centre c moves by d; the crop generalises c to separate input and
 * output centres):
 *     A = G Rz(rot_z) Ry(rot_y) Rx(rot_x) H diag(scale) F
 *     c_in = (in_dim - 1)/2,  c_out = (out_dim - 1)/2
 *     b = c_in + disp + crop - A c_out        (so A c_out + b = c_in + disp + crop)
 * Rx(t) = [[1,0,0],[0,cos t,-sin t],[0,sin t,cos t]] and cyclically for y, z;
 * F = diag(1 - 2*reflect).  Host only, synchronous.  Writes M = [A|b]
 * row-major 3x4 in FP64 to M64 and/or FP32 (round to nearest) to M32 (either
 * may be NULL).  Errors: EINVAL (null prm or both outputs NULL, non-finite
 * value), ESHAPE (negative dimension). */
ctaug_status ctaug_affine_matrix(const ctaug_affine_params *prm, const int64_t in_dim[3],
                                 const int64_t out_dim[3], double M64[12], float M32[12]);

/* ------------------------------------------------------------------------ */
/* Forward warps                                                             */
/* ------------------------------------------------------------------------ */

/* Fused affine augmentation of one volume (Sec. "GPU-accelerated data
 * augmentation": I_affine(x) = I_in(A x + b), trilinear image, nearest
 * labels, then noise and window).  Per output voxel p with coordinate q:
 *   image: if on any axis q_i is not strictly inside (-1, n_i) (or is NaN),
 *          V = fill; otherwise V is the trilinear interpolation of the eight
 *          voxels around floor(q), with `fill` substituted for every corner
 *          outside the volume (constant border).  Then the photometric chain
 *          of `photo` (NULL = identity, out = V).
 *   labels: j_i = floorf(q_i + 0.5f) (FP32; ties round up); lbl_out(p) =
 *          lbl_in(j) if j is inside the volume, else label_fill.
 * img_in: device, F32 or I16, any dims.  lbl_in: device I8 with img_in's dims,
 * or NULL.  M: host float[12].  img_out: device F32 (output dims).  lbl_out:
 * device I8 with img_out's dims, required iff lbl_in is given.  img_out and
 * lbl_out must not alias the inputs.
 * Errors: EINVAL (null required pointer, non-finite M or fill, bad photo,
 * reserved != 0, label_fill outside int8), EDTYPE, ESHAPE (dims mismatch,
 * > 2^31-1 elements), EHIP. */
ctaug_status ctaug_warp_affine(const ctaug_vol *img_in, const ctaug_vol *lbl_in,
                               const float M[12], float fill, int32_t label_fill,
                               const ctaug_photo *photo, ctaug_vol *img_out,
                               ctaug_vol *lbl_out, void *stream);

/* Nearest-neighbour warp of a label volume alone (Sec. "Pre- and
 * post-processing": predicted label maps are resampled back to the original
 * resolution by nearest-neighbour interpolation, with M the map from that
 * grid into the prediction's).  Per output voxel p with coordinate q = A p + b
 * in FP32 as ctaug_warp_affine: lbl_out(p) = lbl_in(j), j_i = floorf(q_i +
 * 0.5f), if q is strictly inside (-1, n) on every axis and j is inside the
 * volume, else label_fill; bit for bit the labels ctaug_warp_affine writes for
 * the same M, with no image read or written.  lbl_in: device I8, any dims,
 * strides allowed (as for gathered inputs).  M: host float[12].  lbl_out:
 * device I8, dense, output dims; must not alias lbl_in.
 * Errors: EINVAL (null pointer, non-finite M, reserved != 0, label_fill
 * outside int8), EDTYPE, ESHAPE (> 2^31-1 elements, a layout beyond the
 * gather limits), EHIP. */
ctaug_status ctaug_warp_labels(const ctaug_vol *lbl_in, const float M[12], int32_t label_fill,
                               ctaug_vol *lbl_out, void *stream);

/* As ctaug_warp_affine with a dense displacement field added to the affine
 * coordinate: q_i = (A p + b)_i + u_i(p) (one FP32 addition).  disp: device
 * float32 SoA [3][Xo][Yo][Zo] on the OUTPUT grid, in input-voxel units.
 * Errors: as ctaug_warp_affine, plus EINVAL for a NULL disp. */
ctaug_status ctaug_warp_displacement(const ctaug_vol *img_in, const ctaug_vol *lbl_in,
                                     const float M[12], const float *disp, float fill,
                                     int32_t label_fill, const ctaug_photo *photo,
                                     ctaug_vol *img_out, ctaug_vol *lbl_out, void *stream);

/* ------------------------------------------------------------------------ */
/* Photometric transform and noise                                           */
/* ------------------------------------------------------------------------ */

/* In-place photometric chain (see ctaug_photo, occlusion included) on a F32
 * volume, voxel index v = linear index in the volume, z = v mod dim[2].
 * Bit-identical to the same chain fused into ctaug_warp_affine.  Errors:
 * EINVAL, EDTYPE (not F32), ESHAPE, EHIP. */
ctaug_status ctaug_photometric_noise(ctaug_vol *inout, const ctaug_photo *photo, void *stream);

/* Noise generator (replaces the per-thread cuRAND generators of the paper's
 * noise paragraph by a stateless counter-based generator).  For voxel index
 * v, Philox4x32-10 (Salmon et al., SC'11) is evaluated at counter
 * (lo32(v>>2), hi32(v>>2), volume_id, 0) with key (lo32(seed), hi32(seed)),
 * giving words w0..w3.  Uniforms U(w) = ((w >> 9) + 0.5) * 2^-23.  Box-Muller
 * on pair k = (v & 3) >> 1: r = sqrt(-2 ln U(w_2k)), theta = 2 pi U(w_2k+1);
 * n(v) = r cos(theta) for even v, r sin(theta) for odd v.
 * Writes, for v = v0 .. v0+n-1, gauss[v - v0] = n(v) (device float*, may be
 * NULL) and, for the groups g = v0>>2 .. (v0+n-1)>>2, words[4*(g - (v0>>2)) + k]
 * = w_k (device uint32*, may be NULL).  Errors: EINVAL (n < 0, overflow), EHIP. */
ctaug_status ctaug_noise(uint64_t seed, uint32_t volume_id, uint64_t v0, int64_t n,
                         float *gauss, uint32_t *words, void *stream);

/* The Box-Muller step of ctaug_noise on caller-supplied words: for pair i,
 * out[2i] = r cos(theta), out[2i+1] = r sin(theta) with r = sqrt(-2 ln U(w[2i])),
 * theta = 2 pi U(w[2i+1]).  words, out: device arrays of 2*npairs elements.
 * Lets callers check or reuse the normal transform on any uniform input.
 * Errors: EINVAL (npairs < 0, null pointer with npairs > 0), EHIP. */
ctaug_status ctaug_box_muller(const uint32_t *words, int64_t npairs, float *out, void *stream);

/* ------------------------------------------------------------------------ */
/* Adjoints (not in the paper)                                               */
/* ------------------------------------------------------------------------ */

/* Workspace bytes needed by the backward calls for an output volume of
 * out_dim (0 for an empty volume, or on bad dims). */
size_t ctaug_warp_backward_workspace(const int64_t out_dim[3]);

/* Adjoint of the affine warp, including the photometric chain when it is
 * differentiable.  With photo (NULL = none) the forward output is
 * gain * V' + offset + sigma * n, V' = 0 on the occluded slab and V' = V
 * elsewhere (ctaug_photo without WINDOW: affine in V, the noise a constant),
 * so the gradient reaching V is g(p) = gain * grad_out(p) off the slab and 0
 * on it (computed in FP32 in the kernel); photo == NULL gives
 * g = grad_out.  With weights w_c(p) of the in-volume corners c of the cell
 * floor(q(p)):
 *   grad_img[c] += sum_p w_c(p) g(p)              (accumulates; see below)
 *   grad_M[i][j] = sum_p g(p) dV/dq_i(p) [x,y,z,1]_j   (overwritten)
 * dV/dq is the derivative of the interpolant on the cell floor(q) (fill
 * corners included, i.e. the right derivative at integer q); samples outside
 * (-1, n) contribute nothing.  grad_img is summed per output tile in fixed
 * point scaled by the tile's largest |g| (gmax), independent of the order of
 * the additions, and tiles meet in FP32 atomics.  Where the map bounds how
 * many of a tile's samples share an input cell by 2^b, b <= 7 (the usual
 * augmentation range; not for strong upsampling or a near-singular A), the
 * tile sums are 32-bit: each contribution is rounded to within 2^(b - 30)
 * gmax.  Otherwise they are 64-bit and exact to 2^-51 gmax.  A tile with a
 * non-finite g adds per corner in FP32 (NaN and infinities reach every
 * in-volume corner of the voxel's cell, as 0 * NaN = NaN).
 * img_in: device F32/I16 (may be strided); photo: host, WINDOW not allowed
 * (EINVAL); grad_out: device F32 with the output dims; grad_img: device F32
 * with img_in's dims (dense), or NULL; grad_M: device double[12], or NULL.
 * ws: device workspace of at least ctaug_warp_backward_workspace(out dims)
 * bytes (required when grad_M is given).  grad_M is reduced
 * deterministically in FP64.
 * Errors: EINVAL, EDTYPE, ESHAPE, EWORKSPACE, EHIP. */
ctaug_status ctaug_warp_affine_backward(const ctaug_vol *img_in, const float M[12], float fill,
                                        const ctaug_photo *photo, const ctaug_vol *grad_out,
                                        ctaug_vol *grad_img, double *grad_M, void *ws,
                                        size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same adjoint
 * as ctaug_warp_affine_backward, bit for bit in grad_M, without a workspace
 * argument.  Its only scratch memory, the FP64 partial rows of grad_M (at
 * most 2048 rows of 12 doubles), lives in a 192 KiB static device array of
 * the library, one copy per GPU, held until the process ends.  The call
 * allocates nothing (no hipMalloc / hipFree, no library allocation).  Every
 * call on a GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (on different streams, or from
 * several threads) race and must be serialised by the caller; each call
 * overwrites every row it reads.  Errors: as ctaug_warp_affine_backward;
 * EWORKSPACE if the output would need more partial rows than the array
 * holds (no output shape does today). */
ctaug_status ctaug_warp_affine_backward_noalloc(const ctaug_vol *img_in, const float M[12],
                                                float fill, const ctaug_photo *photo,
                                                const ctaug_vol *grad_out, ctaug_vol *grad_img,
                                                double *grad_M, void *stream);

/* Batched adjoint of the affine warp (an addition: one launch for a training
 * batch's volumes rather than one per volume, so that the per-launch ramp,
 * tail and reduction are paid once).  Job k holds exactly the arguments of
 * ctaug_warp_affine_backward for one volume: grad_img.data == NULL means no
 * image gradient, grad_M == NULL no parameter gradient, photo.flags with
 * CTAUG_PHOTO_NONE no photometric chain.  Results: as one call per job;
 * grad_img tile sums are fixed point and meet in FP32 atomics (32-bit sums
 * when every job of the launch has the single call's bound, else 64-bit),
 * grad_M is reduced in FP64 in a fixed order over the launch's workgroups
 * (deterministic for a given device and batch; its rounding may differ from
 * the single call's, which reduces over a different set of rows).  Every
 * input image must have the same dtype (EDTYPE otherwise); output volumes
 * of different jobs must not overlap.  Up to 8 jobs go into one launch
 * (their descriptors travel in the kernel arguments: no upload, no
 * allocation, graph-capturable); larger batches take one launch per 8.
 * ws: device workspace of ctaug_warp_affine_backward_batch_workspace(n_jobs)
 * bytes (FP64 partial rows), required when any job wants grad_M.
 * Errors: EINVAL (null pointer, n_jobs < 1, bad job), EDTYPE, ESHAPE,
 * EWORKSPACE, EHIP. */
typedef struct {
    ctaug_vol img_in;      /* device F32 / I16, may be strided */
    ctaug_vol grad_out;    /* device F32, the forward output's dims */
    ctaug_vol grad_img;    /* device F32, img_in's dims, accumulated into; data NULL = none */
    double *grad_M;        /* device double[12], overwritten; NULL = none */
    float M[12];
    float fill;
    ctaug_photo photo;     /* without WINDOW; flags CTAUG_PHOTO_NONE = none */
} ctaug_bwd_job;

size_t ctaug_warp_affine_backward_batch_workspace(int32_t n_jobs);
ctaug_status ctaug_warp_affine_backward_batch(const ctaug_bwd_job *jobs, int32_t n_jobs,
                                              void *ws, size_t ws_bytes, void *stream);

/* Adjoint of ctaug_warp_displacement: as above (photo likewise), plus
 * grad_disp[i](p) = g(p) dV/dq_i(p) (device float SoA [3][Xo][Yo][Zo],
 * overwritten, or NULL). */
ctaug_status ctaug_warp_displacement_backward(const ctaug_vol *img_in, const float M[12],
                                              const float *disp, float fill,
                                              const ctaug_photo *photo,
                                              const ctaug_vol *grad_out, ctaug_vol *grad_img,
                                              double *grad_M, float *grad_disp, void *ws,
                                              size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Cubic B-spline displacement (uniform cubic free-form deformation,         */
/* Rueckert et al., IEEE TMI 1999; not in the paper)                         */
/* ------------------------------------------------------------------------ */

/* disp[i](p) = sum_{a,b,c=0..3} B_a(t_x) B_b(t_y) B_c(t_z) ctrl[i][ix+a][iy+b][iz+c]
 * where, per axis k, h = (n_k - 1)/(G_k - 3), s = p_k / h, i = min(floor(s),
 * G_k - 4), t = s - i (t = 0, i = 0 when n_k = 1), and B0 = (1-t)^3/6,
 * B1 = (3t^3 - 6t^2 + 4)/6, B2 = (-3t^3 + 3t^2 + 3t + 1)/6, B3 = t^3/6: control
 * j sits at output coordinate (j - 1) h.  ctrl: device float [3][Gx][Gy][Gz]
 * with 4 <= G_k <= 64; disp: device float SoA [3][Xo][Yo][Zo].
 * Errors: EINVAL, ESHAPE, EHIP. */
ctaug_status ctaug_bspline_upsample(const float *ctrl, const int64_t G[3],
                                    const int64_t out_dim[3], float *disp, void *stream);

/* Fused nonrigid warp: ctaug_warp_displacement with the displacement of
 * ctaug_bspline_upsample(ctrl, G, img_out dims) evaluated inside the warp
 * kernel instead of read from a dense field (the nonrigid deformation the
 * paper applies on top of the affine map, built from a coarse control grid).
 * The field is computed with the same FP32 operations in the same order as
 * ctaug_bspline_upsample, so outputs and labels equal those of the two
 * unfused calls bit for bit; no field is stored.  ctrl: device float
 * [3][Gx][Gy][Gz] with 4 <= G_k <= 64; other arguments as ctaug_warp_affine.
 * Errors: as ctaug_warp_affine, plus EINVAL for a NULL ctrl with a nonempty
 * output and ESHAPE for a bad grid. */
ctaug_status ctaug_warp_bspline(const ctaug_vol *img_in, const ctaug_vol *lbl_in,
                                const float M[12], const float *ctrl, const int64_t G[3],
                                float fill, int32_t label_fill, const ctaug_photo *photo,
                                ctaug_vol *img_out, ctaug_vol *lbl_out, void *stream);

/* Workspace bytes for ctaug_warp_bspline_backward (0 on bad arguments). */
size_t ctaug_warp_bspline_backward_workspace(const int64_t out_dim[3], const int64_t G[3]);

/* Adjoint of ctaug_warp_bspline: grad_img and grad_M as in
 * ctaug_warp_affine_backward (photo likewise; q now includes the spline
 * displacement), and
 *   grad_ctrl = B^T grad_disp,  grad_disp[i](p) = g(p) dV/dq_i(p)
 * (device float [3][Gx][Gy][Gz], overwritten, or NULL): the gradient with
 * respect to the control grid, without a dense field in memory when the
 * grid has at most 2048 entries and no 8 x 8 x 16 output tile touches more
 * than 8 controls along an axis (otherwise grad_disp is staged in the
 * workspace and contracted by the B-spline adjoint).  Reduced in FP64 in a
 * fixed order (deterministic).  ws: device workspace of at least
 * ctaug_warp_bspline_backward_workspace(grad_out dims, G) bytes, required
 * when grad_M or grad_ctrl is given.
 * Errors: EINVAL (null required pointer, non-finite M or fill), EDTYPE,
 * ESHAPE (dims mismatch, bad grid), EWORKSPACE, EHIP. */
ctaug_status ctaug_warp_bspline_backward(const ctaug_vol *img_in, const float M[12],
                                         const float *ctrl, const int64_t G[3], float fill,
                                         const ctaug_photo *photo,
                                         const ctaug_vol *grad_out, ctaug_vol *grad_img,
                                         double *grad_M, float *grad_ctrl, void *ws,
                                         size_t ws_bytes, void *stream);

/* Workspace bytes for ctaug_bspline_upsample_adjoint. */
size_t ctaug_bspline_adjoint_workspace(const int64_t out_dim[3], const int64_t G[3]);

/* Adjoint: grad_ctrl = B^T grad_disp (device float [3][Gx][Gy][Gz], overwritten),
 * reduced deterministically in FP64.  Errors: EINVAL, ESHAPE, EWORKSPACE, EHIP. */
ctaug_status ctaug_bspline_upsample_adjoint(const float *grad_disp, const int64_t out_dim[3],
                                            const int64_t G[3], float *grad_ctrl, void *ws,
                                            size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Resampling pre-step (Sec. "Pre- and post-processing")                     */
/* ------------------------------------------------------------------------ */

/* Smoothing widths before resampling a volume of voxel spacing spacing[k]
 * (any unit) to the coarser spacing `target` (same unit):
 *     sigma_k = max(target / spacing_k - 1, 0) / 3   (input voxels)
 * Host only.  Errors: EINVAL (null pointer, non-finite or non-positive
 * spacing or target). */
ctaug_status ctaug_resample_sigma(const double spacing[3], double target, float sigma[3]);

/* Separable Gaussian smoothing g(x) ~ exp(-sum_k x_k^2 / sigma_k^2) (the
 * section's kernel as printed: standard deviation sigma_k / sqrt(2) per axis),
 * sampled at integer offsets |d| <= R_k = floor(3 sigma_k / sqrt(2) + 0.5) and
 * normalised to sum 1; voxels beyond the volume repeat the nearest edge voxel;
 * an axis with R_k = 0 is left unchanged.  Resampling itself is then
 * ctaug_warp_affine with A = diag(target / spacing) (ctaug_affine_matrix with
 * those scale factors aligns the volume centres).
 * in: device F32 or I16; out: device F32 with in's dims, not aliasing in;
 * ws: device workspace of ctaug_gaussian_smooth_workspace(dims) bytes, needed
 * when two or more axes are smoothed (else may be NULL).  X and Y extents up
 * to 65535.  FP32 accumulation.
 * Errors: EINVAL (bad sigma, R_k > 160, aliasing), EDTYPE, ESHAPE,
 * EWORKSPACE, EHIP. */
size_t ctaug_gaussian_smooth_workspace(const int64_t dim[3]);
ctaug_status ctaug_gaussian_smooth(const ctaug_vol *in, ctaug_vol *out, const float sigma[3],
                                   void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Batched augmentation of volumes of uneven sizes (the paper augments a     */
/* whole training batch through a job queue; here one launch covers it)      */
/* ------------------------------------------------------------------------ */

/* One job: exactly the arguments of ctaug_warp_affine, or of
 * ctaug_warp_bspline when ctrl is not NULL (grid = its G).  lbl_in.data ==
 * NULL means no labels (then lbl_out is ignored); photo.flags bit 31 set means
 * "no photometrics".  A plan holds either only affine jobs or only B-spline
 * jobs; B-spline plans always use 8 x 8 x 16 tiles and FP32 LDS cells. */
typedef struct {
    ctaug_vol img_in, lbl_in, img_out, lbl_out;
    float M[12];
    float fill;
    int32_t label_fill;
    ctaug_photo photo;
    const float *ctrl;     /* device [3][Gx][Gy][Gz], or NULL */
    int64_t grid[3];
} ctaug_job;


/* Launch shape: output tile (voxels along x, y, z; each a power of two, z at
 * least 4, at most 2^14 voxels), the number of resident workgroups per CU for
 * the persistent launch (0 = one workgroup per tile, non-persistent), and the
 * LDS footprint reserved per workgroup in input cells (0 = sized from the
 * jobs; -1 = no LDS staging), and the cell format: 0 = FP32 cells (4 bytes
 * per cell; at most 15344 cells in the 60 KB reservation), 1 = int16 cells
 * when every input is int16 (2 bytes per cell, at most 30704 cells; half the
 * LDS, more conversions per corner read).  Labels are not staged: they are
 * gathered from global memory while sampling.  Tiles whose footprint
 * exceeds the reservation, and int16-cell jobs whose fill value is not an
 * int16, gather directly from global memory, with identical results. */
typedef struct {
    int32_t tile[3];
    int32_t wg_per_cu;
    int32_t lds_cells;
    int32_t lds_format;
} ctaug_tuning;

typedef struct ctaug_batch_plan ctaug_batch_plan;

/* Create a plan for n_jobs jobs whose shapes are those of jobs[] (host
 * array).  Allocates the device job table and pinned staging (freed by
 * ctaug_batch_plan_destroy).  tune == NULL takes the autotune cache's entry
 * for this device and batch class (see ctaug_autotune_cache_lookup), else the
 * default launch shape (8 x 16 x 16 tiles, one workgroup per tile, LDS sized
 * from the jobs, FP32 cells).  Errors: EINVAL, EDTYPE, ESHAPE, EHIP. */
ctaug_status ctaug_batch_plan_create(const ctaug_job *jobs, int32_t n_jobs,
                                     const ctaug_tuning *tune, ctaug_batch_plan **plan);

/* Replace the jobs' contents (pointers, matrices, photometrics).  Every job
 * must keep the output dims it had at plan creation (else ESHAPE), and an
 * FP32 input is refused (EDTYPE) in a plan created with only int16 inputs.
 * Waits (host side) until the plan's last launch, run or replay has finished
 * on the GPU (its upload reads the staging buffer, its kernel the table)
 * before overwriting staging. */
ctaug_status ctaug_batch_plan_update(ctaug_batch_plan *plan, const ctaug_job *jobs);

/* Updates prepared ahead of time: ctaug_batch_plan_prepare validates jobs
 * against the plan and builds their descriptors once (host memory owned by
 * *out, no device work); ctaug_batch_plan_update_prepared then installs them
 * exactly as ctaug_batch_plan_update would (same wait for the plan's last
 * launch, run or replay), with no per-call validation: one copy into the
 * pinned staging buffer.  A prepared set belongs to its plan and to the
 * plan's current launch shape: after ctaug_batch_plan_autotune it is stale
 * and update_prepared returns EINVAL (prepare again).  The caller keeps the
 * jobs' buffers alive and unchanged in shape while a prepared set may be
 * installed.  Errors: as ctaug_batch_plan_update; EINVAL for another plan's
 * or a stale set. */
typedef struct ctaug_batch_jobs ctaug_batch_jobs;
ctaug_status ctaug_batch_plan_prepare(ctaug_batch_plan *plan, const ctaug_job *jobs,
                                      ctaug_batch_jobs **out);
ctaug_status ctaug_batch_plan_update_prepared(ctaug_batch_plan *plan,
                                              const ctaug_batch_jobs *jobs);
ctaug_status ctaug_batch_jobs_destroy(ctaug_batch_jobs *jobs);

/* Enqueue: upload the job table (async copy from pinned staging) and run one
 * persistent launch that warps every job.  Results equal ctaug_warp_affine
 * (ctaug_warp_bspline) on each job, bit for bit. */
ctaug_status ctaug_batch_plan_launch(ctaug_batch_plan *plan, void *stream);

/* Enqueue only the persistent launch, reading the job table uploaded by the
 * last launch, replay or autotune (no upload): re-runs the same descriptors,
 * e.g. after the caller refilled the same input buffers in place.  EINVAL
 * before the first launch or replay. */
ctaug_status ctaug_batch_plan_run(ctaug_batch_plan *plan, void *stream);

/* Capture ctaug_batch_plan_launch on `stream` into a HIP graph owned by the
 * plan (replacing any earlier one); ctaug_batch_plan_replay then launches it.
 * The graph reads the staging buffer at replay time, so updates between
 * replays need no re-capture. */
ctaug_status ctaug_batch_plan_capture(ctaug_batch_plan *plan, void *stream);
ctaug_status ctaug_batch_plan_replay(ctaug_batch_plan *plan, void *stream);

/* Time each candidate launch shape on the plan's current jobs (HIP events,
 * `reps` launches each, after one warm-up) and keep the fastest in the plan
 * and in the autotune cache (under this device and the plan's batch class).
 * The jobs' outputs are overwritten (with identical results).  Synchronises
 * `stream`.  best (host, may be NULL) receives the choice; times_ms (host
 * float[n_cand], may be NULL) the mean time per launch of each candidate. */
ctaug_status ctaug_batch_plan_autotune(ctaug_batch_plan *plan, const ctaug_tuning *cand,
                                       int32_t n_cand, int32_t reps, void *stream,
                                       ctaug_tuning *best, float *times_ms);

ctaug_status ctaug_batch_plan_get_tuning(const ctaug_batch_plan *plan, ctaug_tuning *out);
ctaug_status ctaug_batch_plan_destroy(ctaug_batch_plan *plan);

/* Autotune cache: the library's only state beyond plans and pipelines (one per
 * process, thread-safe).  An entry maps (device architecture name and compute
 * unit count; batch class) to the launch shape ctaug_batch_plan_autotune
 * chose.  The batch class is: the inputs' dtype specialisation (all int16,
 * all FP32, mixed; B-spline jobs apart), ceil(log2(n_jobs)),
 * ceil(log2(largest output voxel count)), and whether any job warps labels or
 * draws noise.
 *
 * lookup: *found = 1 and *out = the entry for these jobs on the current
 * device, else *found = 0 (jobs validated as by ctaug_batch_plan_create;
 * ENODEV without a device).  save: write every entry as text to path (a
 * header line, then one line per entry).  load: read such a file and merge
 * its entries (replacing equal keys); *n_entries (may be NULL) receives the
 * count; a malformed file (bad header, field count or launch shape) merges
 * nothing and returns EINVAL.  clear: drop every entry.  Host only. */
ctaug_status ctaug_autotune_cache_lookup(const ctaug_job *jobs, int32_t n_jobs, ctaug_tuning *out,
                                         int32_t *found);
ctaug_status ctaug_autotune_cache_save(const char *path);
ctaug_status ctaug_autotune_cache_load(const char *path, int32_t *n_entries);
ctaug_status ctaug_autotune_cache_clear(void);

/* ------------------------------------------------------------------------ */
/* Host-to-device FIFO (Sec. "GPU-accelerated data augmentation": volumes    */
/* are queued on the host while the GPU augments earlier ones, so that       */
/* transfers overlap the warps)                                              */
/* ------------------------------------------------------------------------ */

typedef struct ctaug_pipeline ctaug_pipeline;

/* Not thread-safe: one producer thread drives a pipeline.
 *
 * Create a FIFO of `depth` >= 2 slots of `slot_bytes` bytes each: pinned host
 * buffers the caller fills, device buffers the warps read, a copy stream and
 * a compute stream (default priority), and per-slot events.  Owned by the
 * pipeline, freed by ctaug_pipeline_destroy.  Errors: EINVAL (depth < 2 or >
 * 64, slot_bytes 0, null out), EHIP (allocation). */
ctaug_status ctaug_pipeline_create(int32_t depth, size_t slot_bytes, ctaug_pipeline **out);

/* Hand out the next slot's pinned host buffer (*host_slot, slot_bytes bytes)
 * for the caller to fill with one volume (image, optionally labels, at any
 * offsets).  Blocks the calling host thread until the warp that last read the
 * slot has finished.  Errors: EINVAL (null argument, a slot already handed
 * out and not submitted), EHIP. */
ctaug_status ctaug_pipeline_acquire(ctaug_pipeline *p, void **host_slot);

/* Queue the acquired slot: copy the bytes of img (and lbl) from the host
 * slot to the device slot on the copy stream, then run the fused affine warp
 * (as ctaug_warp_affine, same results bit for bit) on the compute stream once
 * the copy has landed.  img->data / lbl->data are HOST pointers inside the
 * acquired slot; img_out / lbl_out are device volumes owned by the caller,
 * written asynchronously on the compute stream (ctaug_pipeline_sync, or an
 * event on ctaug_pipeline_stream's stream, orders later work after them).
 * Errors: as ctaug_warp_affine, plus EINVAL when no slot is acquired or an
 * input does not lie inside it; on an error the slot stays acquired and
 * nothing is queued, so a corrected submit may follow. */
ctaug_status ctaug_pipeline_submit(ctaug_pipeline *p, const ctaug_vol *img_host,
                                   const ctaug_vol *lbl_host, const float M[12], float fill,
                                   int32_t label_fill, const ctaug_photo *photo,
                                   ctaug_vol *img_out, ctaug_vol *lbl_out);

/* The compute stream (hipStream_t as void*) the pipeline's warps run on. */
ctaug_status ctaug_pipeline_stream(ctaug_pipeline *p, void **stream);

/* Block until every submitted copy and warp has finished.  Errors: EINVAL, EHIP. */
ctaug_status ctaug_pipeline_sync(ctaug_pipeline *p);

/* Wait for outstanding work, then free every buffer, stream and event. */
ctaug_status ctaug_pipeline_destroy(ctaug_pipeline *p);

/* ------------------------------------------------------------------------ */
/* Measurement helper                                                        */
/* ------------------------------------------------------------------------ */

/* Plain device-to-device copy of `bytes` bytes by a streaming kernel (16-byte
 * vector loads and stores when both pointers are 16-byte aligned).  Used as the
 * reference kernel of known traffic when scaling hardware byte counters, and
 * to evict the Infinity Cache between timed runs.  Errors: EINVAL, EHIP. */
ctaug_status ctaug_copy(const void *src, void *dst, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CTAUG_H */
