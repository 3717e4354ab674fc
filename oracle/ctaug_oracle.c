/*
 * ctaug_oracle.c -- plain CPU oracle for the CT data-augmentation hot path of
 * Rister et al., "CT organ segmentation using GPU data augmentation,
 * unsupervised labels and IOU loss" (arXiv:1811.11226).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file.  It exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the GPU library against a slow,
 * obviously correct reading of the paper.  It shares no code, header, table
 * or constant with the GPU library.
 *
 * Arithmetic: FP64 everywhere, except for expressions that the GPU must
 * reproduce bit for bit and which are therefore pinned to FP32 here as well:
 *   - the sampling coordinate q = A x + b (one fmaf chain per axis),
 *   - the nearest-neighbour label rounding floorf(q + 0.5f), and
 *   - the parity-mode B-spline field of warps that evaluate it themselves
 *     (orc_bspline_upsample_f32; the FP64 field is orc_bspline_upsample).
 * "exact" mode replaces the pinned FP32 coordinate with FP64 and is used only
 * to validate gradient formulas by finite differences.
 *
 * Layout: every volume is a dense C-order array [X][Y][Z] (z fastest).
 * Voxel p = (x, y, z) has linear index v = (x*Y + y)*Z + z.
 *
 * Citations are to sections / equations of the paper:
 *   Sec. "GPU-accelerated data augmentation" (GPU-AUG):
 *     affine map x' = A x + b, b = c + d - A c, I_affine(x) = I_in(A x + b),
 *     trilinear image / nearest-neighbour labels, additive Gaussian noise
 *     I_noise = I_occ + n, window equation I_window = min(max((I-a)/(b-a),0),1).
 *   Sec. "Pre- and post-processing": random 120x120x160 training crop.
 * Gain/offset/gamma, the Philox counter mapping, the displacement field, its
 * cubic B-spline parameterisation and the adjoints are NOT in the paper; they
 * follow the definitions written next to each function below.
 *
 * Parity status: every function here is pinned by tests in
 * tests/test_oracle_pins.py (closed forms, invariants, brute force, SciPy /
 * torch-CPU / rocRAND-host cross-checks).  The relation to the paper's own
 * outputs is parity unpinned: its data, texture precision and RNG are not
 * available.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Replaces the per-thread cuRAND generators of   */
/* Sec. GPU-AUG (noise paragraph) by a stateless counter-based generator.    */
/* ------------------------------------------------------------------------ */

static void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

/* One application of the 10-round bijection to a 128-bit counter under a
 * 64-bit key.  Each round multiplies counter words 0 and 2 by the two Philox
 * multipliers, and forms the new counter from the high halves xor-ed with the
 * other two words and the round key, and the low halves.  The key advances by
 * the two Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t MUL0 = 0xD2511F53u, MUL1 = 0xCD9E8D57u;
    const uint32_t WEYL0 = 0x9E3779B9u, WEYL1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(MUL0, c0, &hi0, &lo0);
        mulhilo32(MUL1, c2, &hi1, &lo1);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += WEYL0;
        k1 += WEYL1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter of the noise draw for output voxel v of volume `vol`: the 4-voxel
 * group index v >> 2 fills counter words 0-1, the volume id word 2, and word 3
 * is a stream tag (0 = additive noise).  Key = (lo32(seed), hi32(seed)). */
static void noise_words(uint64_t seed, uint32_t vol, uint64_t group, uint32_t w[4])
{
    uint32_t ctr[4] = { (uint32_t)group, (uint32_t)(group >> 32), vol, 0u };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    orc_philox4x32_10(ctr, key, w);
}

void orc_noise_words(uint64_t seed, uint32_t vol, uint64_t group0, int64_t ngroups, uint32_t *out)
{
    for (int64_t i = 0; i < ngroups; ++i)
        noise_words(seed, vol, group0 + (uint64_t)i, out + 4 * i);
}

/* Uniform on the open interval (0,1): ((w >> 9) + 1/2) * 2^-23.  The 23 top
 * bits select one of 2^23 equal cells and the value is the cell's centre, so
 * it is exact in FP32 and never 0 or 1. */
double orc_uniform(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* Standard normal for output voxel v (Box & Muller, 1958), FP64.
 * Words (w0,w1) form pair 0, (w2,w3) pair 1; voxel v uses pair ((v & 3) >> 1):
 * radius r = sqrt(-2 ln U(w_even)), angle theta = 2 pi U(w_odd);
 * the even voxel of the pair takes r cos(theta), the odd one r sin(theta). */
double orc_gauss(uint64_t seed, uint32_t vol, uint64_t v)
{
    uint32_t w[4];
    noise_words(seed, vol, v >> 2, w);
    int pair = (int)((v & 3u) >> 1);
    double u_r = orc_uniform(w[2 * pair]);
    double u_t = orc_uniform(w[2 * pair + 1]);
    double r = sqrt(-2.0 * log(u_r));
    double theta = 2.0 * M_PI * u_t;
    return (v & 1u) ? r * sin(theta) : r * cos(theta);
}

/* Box-Muller on explicit words: out[2i] = r cos(theta), out[2i+1] = r sin(theta). */
void orc_box_muller(const uint32_t *w, int64_t npairs, double *out)
{
    for (int64_t i = 0; i < npairs; ++i) {
        double r = sqrt(-2.0 * log(orc_uniform(w[2 * i])));
        double theta = 2.0 * M_PI * orc_uniform(w[2 * i + 1]);
        out[2 * i] = r * cos(theta);
        out[2 * i + 1] = r * sin(theta);
    }
}

void orc_gauss_range(uint64_t seed, uint32_t vol, uint64_t v0, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = orc_gauss(seed, vol, v0 + (uint64_t)i);
}

/* ------------------------------------------------------------------------ */
/* Photometric chain (Sec. GPU-AUG noise and window paragraphs; gain,       */
/* offset and gamma are additions): v = g V + o; v += sigma n(v);            */
/* windowed: t = min(max((v - a)/(b - a), 0), 1), out = t^gamma (0^gamma=0); */
/* otherwise out = v in HU.  photo = {gain, offset, sigma, a, b, gamma}.      */
/* ------------------------------------------------------------------------ */

static double photometric(double V, const double *photo, int window,
                          uint64_t seed, uint32_t vol, uint64_t v)
{
    double gain = photo[0], offset = photo[1], sigma = photo[2];
    double a = photo[3], b = photo[4], gamma = photo[5];
    double val = gain * V + offset;
    val = val + sigma * orc_gauss(seed, vol, v);
    if (!window)
        return val;
    double t = (val - a) / (b - a);
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    return t == 0.0 ? 0.0 : pow(t, gamma);
}

/* ------------------------------------------------------------------------ */
/* Random occlusion (Sec. GPU-AUG, occlusion paragraph and its I_occ         */
/* equation).  The occluded region is the slab of output voxels whose third  */
/* coordinate x_3 (z here) lies in [lo, hi] = [z_start, z_start + delta]; the */
/* equation's printed inequality cannot hold for delta > 0, and it is read as */
/* lo <= z <= hi (closed).  Occluded voxels take the value 0 in place of the  */
/* warped image; noise and window follow as for every voxel, since the noise */
/* equation adds n to I_occ.  occ = {lo, hi} or NULL (no occlusion).         */
/* ------------------------------------------------------------------------ */

static int occluded(const double *occ, int64_t z)
{
    return occ && (double)z >= occ[0] && (double)z <= occ[1];
}

/* Photometric chain over a volume whose z extent is Z (the occlusion test
 * uses z = v mod Z). */
int orc_photometric(const double *vin, int64_t n, const double *photo, int window,
                    uint64_t seed, uint32_t vol, const double *occ, int64_t Z, double *out)
{
    if (!vin || !out || !photo || n < 0 || (occ && Z <= 0))
        return ORC_EINVAL;
    for (int64_t v = 0; v < n; ++v) {
        double V = occluded(occ, occ ? v % Z : 0) ? 0.0 : vin[v];
        out[v] = photometric(V, photo, window, seed, vol, (uint64_t)v);
    }
    return ORC_OK;
}

/* Adjoint of the photometric chain without the window (an addition; the   */
/* paper has no gradients).  Off the window, out = gain * V' + offset +      */
/* sigma * n with V' = 0 on the occluded slab and V' = V elsewhere: affine   */
/* in V, the noise a constant.  So dout/dV = gain off the slab and 0 on it,  */
/* and g_V(p) = gain * g(p) or 0.  The window clamp and gamma are not        */
/* differentiated (EINVAL).  photo, occ, Z as orc_photometric.               */
int orc_photometric_adjoint(const double *g, int64_t n, const double *photo, int window,
                            const double *occ, int64_t Z, double *g_V)
{
    if (!g || !g_V || !photo || n < 0 || window || (occ && Z <= 0))
        return ORC_EINVAL;
    for (int64_t v = 0; v < n; ++v)
        g_V[v] = occluded(occ, occ ? v % Z : 0) ? 0.0 : photo[0] * g[v];
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Transform sampling (Sec. GPU-AUG, first paragraph and footnote; crop from */
/* Sec. Pre- and post-processing).                                           */
/* prm (27 doubles):                                                          */
/*   [0..2]  rotation angles about x, y, z (radians)                          */
/*   [3..5]  scale factors along x, y, z                                      */
/*   [6..8]  shears h_xy, h_xz, h_yz (upper-triangular shear matrix)          */
/*   [9..11] reflection flags for x, y, z (0 or 1)                            */
/*   [12..20] generic 3x3 matrix G, row-major (identity = no generic warp)    */
/*   [21..23] displacement d of the volume centre (input voxels)              */
/*   [24..26] crop shift k (input voxels)                                     */
/* A = G Rz Ry Rx H S F, c = (n - 1)/2 per axis, b = c_in + d + k - A c_out,  */
/* so that A c_out + b = c_in + d + k.  Output M = [A|b] row-major 3x4.      */
/* ------------------------------------------------------------------------ */

static void matmul3(const double *L, const double *R, double *out)
{
    double tmp[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k)
                s += L[3 * i + k] * R[3 * k + j];
            tmp[3 * i + j] = s;
        }
    memcpy(out, tmp, sizeof tmp);
}

int orc_affine_matrix(const double *prm, const int64_t *in_dim, const int64_t *out_dim, double *M)
{
    if (!prm || !in_dim || !out_dim || !M)
        return ORC_EINVAL;
    double cx = cos(prm[0]), sx = sin(prm[0]);
    double cy = cos(prm[1]), sy = sin(prm[1]);
    double cz = cos(prm[2]), sz = sin(prm[2]);
    double Rx[9] = { 1, 0, 0, 0, cx, -sx, 0, sx, cx };
    double Ry[9] = { cy, 0, sy, 0, 1, 0, -sy, 0, cy };
    double Rz[9] = { cz, -sz, 0, sz, cz, 0, 0, 0, 1 };
    double H[9] = { 1, prm[6], prm[7], 0, 1, prm[8], 0, 0, 1 };
    double S[9] = { prm[3], 0, 0, 0, prm[4], 0, 0, 0, prm[5] };
    double F[9] = { prm[9] != 0.0 ? -1.0 : 1.0, 0, 0,
                    0, prm[10] != 0.0 ? -1.0 : 1.0, 0,
                    0, 0, prm[11] != 0.0 ? -1.0 : 1.0 };
    double A[9];
    memcpy(A, prm + 12, sizeof A);      /* G */
    matmul3(A, Rz, A);
    matmul3(A, Ry, A);
    matmul3(A, Rx, A);
    matmul3(A, H, A);
    matmul3(A, S, A);
    matmul3(A, F, A);
    for (int i = 0; i < 3; ++i) {
        double c_in = 0.5 * (double)(in_dim[i] - 1);
        double Ac = 0.0;
        for (int j = 0; j < 3; ++j)
            Ac += A[3 * i + j] * 0.5 * (double)(out_dim[j] - 1);
        for (int j = 0; j < 3; ++j)
            M[4 * i + j] = A[3 * i + j];
        M[4 * i + 3] = c_in + prm[21 + i] + prm[24 + i] - Ac;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Sampling coordinate and trilinear / nearest-neighbour sampling            */
/* (Sec. GPU-AUG: I_affine(x) = I_in(A x + b); trilinear image, nearest      */
/* labels).  Integer coordinates are voxel centres.  Out-of-volume corners   */
/* take the constant `fill` (constant border).                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    const float *Mf;     /* parity mode: FP32 [A|b] */
    const double *Md;    /* exact mode: FP64 [A|b] */
    int exact;
    const float *disp;   /* optional SoA displacement [3][X][Y][Z] on the output grid */
    int64_t out_n;       /* output voxel count (SoA component stride) */
} coord_ctx;

/* q for output voxel (x,y,z) with linear index v.  Parity mode evaluates
 * q_i = fmaf(A_i2, z, fmaf(A_i1, y, fmaf(A_i0, x, b_i))) in FP32 and then adds
 * the displacement as one FP32 addition; exact mode does the same in FP64. */
static void coord(const coord_ctx *cc, int64_t x, int64_t y, int64_t z, int64_t v,
                  double q[3], float qf[3])
{
    for (int i = 0; i < 3; ++i) {
        if (cc->exact) {
            const double *r = cc->Md + 4 * i;
            double t = r[3] + r[0] * (double)x + r[1] * (double)y + r[2] * (double)z;
            if (cc->disp)
                t += (double)cc->disp[i * cc->out_n + v];
            q[i] = t;
            qf[i] = (float)t;
        } else {
            const float *r = cc->Mf + 4 * i;
            float t = fmaf(r[2], (float)z, fmaf(r[1], (float)y, fmaf(r[0], (float)x, r[3])));
            if (cc->disp)
                t = t + cc->disp[i * cc->out_n + v];
            q[i] = (double)t;
            qf[i] = t;
        }
    }
}

/* True when q lies strictly inside (-1, n) on every axis.  Outside that box
 * all eight corners are out of the volume, so the sample equals fill; the
 * test also rejects NaN/inf. */
static int inside_guard(const double q[3], const int64_t n[3])
{
    for (int i = 0; i < 3; ++i)
        if (!(q[i] > -1.0 && q[i] < (double)n[i]))
            return 0;
    return 1;
}

static double lerp(double a, double b, double t) { return a + t * (b - a); }

static double corner(const double *img, const int64_t n[3], int64_t cx, int64_t cy, int64_t cz,
                     double fill)
{
    if (cx < 0 || cy < 0 || cz < 0 || cx >= n[0] || cy >= n[1] || cz >= n[2])
        return fill;
    return img[(cx * n[1] + cy) * n[2] + cz];
}

/* Trilinear value at q (FP64), interpolating z, then y, then x.  Also returns
 * the partial derivatives of the interpolant inside the cell floor(q) (the
 * right derivative at integer coordinates) when dV != NULL. */
static double trilinear(const double *img, const int64_t n[3], const double q[3], double fill,
                        double dV[3])
{
    if (!inside_guard(q, n)) {
        if (dV) dV[0] = dV[1] = dV[2] = 0.0;
        return fill;
    }
    int64_t i0[3];
    double t[3];
    for (int i = 0; i < 3; ++i) {
        double f = floor(q[i]);
        i0[i] = (int64_t)f;
        t[i] = q[i] - f;
    }
    double K[2][2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c)
                K[a][b][c] = corner(img, n, i0[0] + a, i0[1] + b, i0[2] + c, fill);
    double e[2][2];     /* after z */
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            e[a][b] = lerp(K[a][b][0], K[a][b][1], t[2]);
    double f0 = lerp(e[0][0], e[0][1], t[1]);   /* after y */
    double f1 = lerp(e[1][0], e[1][1], t[1]);
    double V = lerp(f0, f1, t[0]);              /* after x */
    if (dV) {
        dV[0] = f1 - f0;
        double gy0 = e[0][1] - e[0][0], gy1 = e[1][1] - e[1][0];
        dV[1] = lerp(gy0, gy1, t[0]);
        double gz[2][2];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                gz[a][b] = K[a][b][1] - K[a][b][0];
        dV[2] = lerp(lerp(gz[0][0], gz[0][1], t[1]), lerp(gz[1][0], gz[1][1], t[1]), t[0]);
    }
    return V;
}

/* Nearest-neighbour label: j_i = floorf(q_i + 0.5f) in FP32 (round half up,
 * including the rounding of the FP32 addition).  Defined only for finite
 * |q_i| < 2^24; anything else, or j outside the volume, gives label_fill. */
static int nn_label(const int8_t *lbl, const int64_t n[3], const float qf[3], int label_fill)
{
    int64_t j[3];
    for (int i = 0; i < 3; ++i) {
        if (!(fabsf(qf[i]) < 16777216.0f))
            return label_fill;
        float h = qf[i] + 0.5f;
        j[i] = (int64_t)floorf(h);
        if (j[i] < 0 || j[i] >= n[i])
            return label_fill;
    }
    return lbl[(j[0] * n[1] + j[1]) * n[2] + j[2]];
}

static int dims_ok(const int64_t *d)
{
    return d && d[0] >= 0 && d[1] >= 0 && d[2] >= 0;
}

typedef struct {
    const double *img;
    const int64_t *in_dim;
    const int8_t *lbl;
    double fill;
    int label_fill;
    const double *photo;
    int window;
    uint64_t seed;
    uint32_t vol;
    const double *occ;
} warp_ctx;

/* One output voxel (x, y, z) with linear index v of the forward warp. */
static void warp_voxel(const coord_ctx *cc, const warp_ctx *w, int64_t x, int64_t y, int64_t z,
                       int64_t v, double *out, int8_t *lbl_out)
{
    double q[3];
    float qf[3];
    coord(cc, x, y, z, v, q, qf);
    if (out) {
        /* I_occ: the occluded slab is 0, elsewhere the warped image */
        double V = occluded(w->occ, z) ? 0.0 : trilinear(w->img, w->in_dim, q, w->fill, NULL);
        *out = w->photo ? photometric(V, w->photo, w->window, w->seed, w->vol, (uint64_t)v) : V;
    }
    if (lbl_out)
        *lbl_out = (int8_t)nn_label(w->lbl, w->in_dim, qf, w->label_fill);
}

static int warp_args_ok(const double *img, const int64_t *in_dim, const int8_t *lbl,
                        const float *Mf, const double *Md, int exact, const int64_t *out_dim,
                        const double *out, const int8_t *lbl_out)
{
    if (!dims_ok(in_dim) || !dims_ok(out_dim))
        return 0;
    if ((exact && !Md) || (!exact && !Mf))
        return 0;
    if ((out && !img) || (lbl_out && !lbl))
        return 0;
    return 1;
}

/* Forward warp: out(p) = photometric(I_in(q(p))), lbl_out(p) = L_in(nn(q(p))).
 * img/out may be NULL independently of lbl/lbl_out.  photo == NULL leaves
 * the interpolated value unchanged (identity photometrics). */
int orc_warp(const double *img, const int64_t *in_dim, const int8_t *lbl,
             const float *Mf, const double *Md, int exact, const float *disp,
             double fill, int label_fill,
             const double *photo, int window, uint64_t seed, uint32_t vol, const double *occ,
             const int64_t *out_dim, double *out, int8_t *lbl_out)
{
    if (!warp_args_ok(img, in_dim, lbl, Mf, Md, exact, out_dim, out, lbl_out))
        return ORC_EINVAL;
    const int64_t X = out_dim[0], Y = out_dim[1], Z = out_dim[2];
    coord_ctx cc = { Mf, Md, exact, disp, X * Y * Z };
    warp_ctx w = { img, in_dim, lbl, fill, label_fill, photo, window, seed, vol, occ };
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < X; ++x)
        for (int64_t y = 0; y < Y; ++y)
            for (int64_t z = 0; z < Z; ++z) {
                int64_t v = (x * Y + y) * Z + z;
                warp_voxel(&cc, &w, x, y, z, v, out ? out + v : NULL, lbl_out ? lbl_out + v : NULL);
            }
    return ORC_OK;
}

/* The same warp evaluated only at the npts output voxels with linear indices
 * idx[k] (each in [0, X*Y*Z)); out[k] / lbl_out[k] receive voxel idx[k].  A
 * displacement field, when given, is still the whole [3][X][Y][Z] field. */
int orc_warp_points(const double *img, const int64_t *in_dim, const int8_t *lbl,
                    const float *Mf, const double *Md, int exact, const float *disp,
                    double fill, int label_fill,
                    const double *photo, int window, uint64_t seed, uint32_t vol,
                    const double *occ, const int64_t *out_dim, const int64_t *idx, int64_t npts,
                    double *out, int8_t *lbl_out)
{
    if (!warp_args_ok(img, in_dim, lbl, Mf, Md, exact, out_dim, out, lbl_out) || npts < 0 ||
        (npts > 0 && !idx))
        return ORC_EINVAL;
    const int64_t X = out_dim[0], Y = out_dim[1], Z = out_dim[2];
    for (int64_t k = 0; k < npts; ++k)
        if (idx[k] < 0 || idx[k] >= X * Y * Z)
            return ORC_EINVAL;
    coord_ctx cc = { Mf, Md, exact, disp, X * Y * Z };
    warp_ctx w = { img, in_dim, lbl, fill, label_fill, photo, window, seed, vol, occ };
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < npts; ++k) {
        const int64_t v = idx[k];
        const int64_t z = v % Z, y = (v / Z) % Y, x = v / (Y * Z);
        warp_voxel(&cc, &w, x, y, z, v, out ? out + k : NULL, lbl_out ? lbl_out + k : NULL);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the warp with respect to the image, the 12 entries of [A|b]    */
/* and the displacement field (an addition; the paper has no gradients).    */
/* With V(p) = sum_c w_c(p) I[c] + fill * (1 - sum_c w_c(p)) for the         */
/* in-volume corners c of the cell floor(q(p)):                               */
/*   g_img[c]  += w_c(p) g(p)                                                 */
/*   g_M[i][j]  = sum_p g(p) dV/dq_i(p) [x, y, z, 1]_j                        */
/*   g_u[i](p)  = g(p) dV/dq_i(p)                                             */
/* dV/dq is the derivative of the interpolant on the cell floor(q) (fill     */
/* corners included), i.e. the right derivative at integer q.  Samples       */
/* outside the (-1, n) box have zero gradient.                               */
/* ------------------------------------------------------------------------ */

int orc_warp_backward(const double *img, const int64_t *in_dim,
                      const float *Mf, const double *Md, int exact, const float *disp,
                      double fill, const double *g, const int64_t *out_dim,
                      double *g_img, double *g_M, double *g_u)
{
    if (!dims_ok(in_dim) || !dims_ok(out_dim) || !g || !img)
        return ORC_EINVAL;
    if ((exact && !Md) || (!exact && !Mf))
        return ORC_EINVAL;
    const int64_t X = out_dim[0], Y = out_dim[1], Z = out_dim[2];
    const int64_t *n = in_dim;
    coord_ctx cc = { Mf, Md, exact, disp, X * Y * Z };
    double acc[12];
    memset(acc, 0, sizeof acc);
    for (int64_t x = 0; x < X; ++x)
        for (int64_t y = 0; y < Y; ++y)
            for (int64_t z = 0; z < Z; ++z) {
                int64_t v = (x * Y + y) * Z + z;
                double q[3], dV[3];
                float qf[3];
                coord(&cc, x, y, z, v, q, qf);
                trilinear(img, n, q, fill, dV);
                double gp = g[v];
                if (g_u)
                    for (int i = 0; i < 3; ++i)
                        g_u[i * cc.out_n + v] = gp * dV[i];
                double pos[4] = { (double)x, (double)y, (double)z, 1.0 };
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 4; ++j)
                        acc[4 * i + j] += gp * dV[i] * pos[j];
                if (!g_img || !inside_guard(q, n))
                    continue;
                int64_t i0[3];
                double t[3];
                for (int i = 0; i < 3; ++i) {
                    double f = floor(q[i]);
                    i0[i] = (int64_t)f;
                    t[i] = q[i] - f;
                }
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        for (int c = 0; c < 2; ++c) {
                            int64_t cx = i0[0] + a, cy = i0[1] + b, cz = i0[2] + c;
                            if (cx < 0 || cy < 0 || cz < 0 || cx >= n[0] || cy >= n[1] || cz >= n[2])
                                continue;
                            double w = (a ? t[0] : 1.0 - t[0]) * (b ? t[1] : 1.0 - t[1]) *
                                       (c ? t[2] : 1.0 - t[2]);
                            g_img[(cx * n[1] + cy) * n[2] + cz] += w * gp;
                        }
            }
    if (g_M)
        memcpy(g_M, acc, sizeof acc);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Uniform cubic B-spline free-form displacement (Rueckert et al., IEEE TMI  */
/* 1999), an addition to the paper.  Control grid C[3][Gx][Gy][Gz]; control  */
/* j of axis k sits at output coordinate (j - 1) h_k, h_k = (n_k - 1)/(G_k-3) */
/* so that the grid spans the output volume.  For p_k: s = p_k / h_k,        */
/* i = min(floor(s), G_k - 4), t = s - i, and                                */
/*   u(p) = sum_{a,b,c=0..3} B_a(t_x) B_b(t_y) B_c(t_z) C[i_x+a][i_y+b][i_z+c] */
/* with B0=(1-t)^3/6, B1=(3t^3-6t^2+4)/6, B2=(-3t^3+3t^2+3t+1)/6, B3=t^3/6.  */
/* ------------------------------------------------------------------------ */

static void bspline_basis(double t, double B[4])
{
    double t2 = t * t, t3 = t2 * t, m = 1.0 - t;
    B[0] = m * m * m / 6.0;
    B[1] = (3.0 * t3 - 6.0 * t2 + 4.0) / 6.0;
    B[2] = (-3.0 * t3 + 3.0 * t2 + 3.0 * t + 1.0) / 6.0;
    B[3] = t3 / 6.0;
}

static void bspline_cell(int64_t p, int64_t n, int64_t G, int64_t *i, double *t)
{
    if (n <= 1) {
        *i = 0;
        *t = 0.0;
        return;
    }
    double h = (double)(n - 1) / (double)(G - 3);
    double s = (double)p / h;
    double f = floor(s);
    if (f > (double)(G - 4))
        f = (double)(G - 4);
    *i = (int64_t)f;
    *t = s - f;
}

int orc_bspline_upsample(const double *ctrl, const int64_t *G, const int64_t *out_dim, double *u)
{
    if (!ctrl || !u || !dims_ok(out_dim) || !G || G[0] < 4 || G[1] < 4 || G[2] < 4)
        return ORC_EINVAL;
    const int64_t X = out_dim[0], Y = out_dim[1], Z = out_dim[2], N = X * Y * Z;
    const int64_t GN = G[0] * G[1] * G[2];
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < X; ++x)
        for (int64_t y = 0; y < Y; ++y)
            for (int64_t z = 0; z < Z; ++z) {
                int64_t ix, iy, iz;
                double tx, ty, tz, Bx[4], By[4], Bz[4];
                bspline_cell(x, X, G[0], &ix, &tx);
                bspline_cell(y, Y, G[1], &iy, &ty);
                bspline_cell(z, Z, G[2], &iz, &tz);
                bspline_basis(tx, Bx);
                bspline_basis(ty, By);
                bspline_basis(tz, Bz);
                int64_t v = (x * Y + y) * Z + z;
                for (int comp = 0; comp < 3; ++comp) {
                    double s = 0.0;
                    for (int a = 0; a < 4; ++a)
                        for (int b = 0; b < 4; ++b)
                            for (int c = 0; c < 4; ++c)
                                s += Bx[a] * By[b] * Bz[c] *
                                     ctrl[comp * GN + ((ix + a) * G[1] + (iy + b)) * G[2] + (iz + c)];
                    u[comp * N + v] = s;
                }
            }
    return ORC_OK;
}

/* Parity mode of the field, for warps that evaluate it themselves: the same
 * definition in FP32 with every rounding fixed, so that a kernel that follows
 * the same steps agrees bit for bit (as the pinned coordinate map does).
 * Per axis: inv_h = (float)((G - 3) / (n - 1)) (0 when n = 1); s = (float)p *
 * inv_h; i = min(floor(s), G - 4); t = s - i.  Basis with m = 1 - t, t2 = t*t,
 * t3 = t2*t, k = 1/6 rounded to FP32: B0 = ((m*m)*m)*k, B1 = fmaf(3, t3,
 * fmaf(-6, t2, 4))*k, B2 = fmaf(-3, t3, fmaf(3, t2, fmaf(3, t, 1)))*k,
 * B3 = t3*k.  Sums: P(gz) = sum_a Bx_a (sum_b By_b C[ix+a][iy+b][gz]) and
 * u = sum_c Bz_c P(iz+c), each a chain of fmaf from 0 in index order. */
static void bspline_cell_f32(int64_t p, int64_t n, int64_t G, int64_t *i, float *t)
{
    const float inv_h = n > 1 ? (float)((double)(G - 3) / (double)(n - 1)) : 0.0f;
    const float s = (float)p * inv_h;
    const float f = fminf(floorf(s), (float)(G - 4));
    *i = (int64_t)f;
    *t = s - f;
}

static void bspline_basis_f32(float t, float B[4])
{
    const float t2 = t * t, t3 = t2 * t, m = 1.0f - t, k = 1.0f / 6.0f;
    B[0] = m * m * m * k;
    B[1] = fmaf(3.0f, t3, fmaf(-6.0f, t2, 4.0f)) * k;
    B[2] = fmaf(-3.0f, t3, fmaf(3.0f, t2, fmaf(3.0f, t, 1.0f))) * k;
    B[3] = t3 * k;
}

int orc_bspline_upsample_f32(const float *ctrl, const int64_t *G, const int64_t *out_dim, float *u)
{
    if (!ctrl || !u || !dims_ok(out_dim) || !G || G[0] < 4 || G[1] < 4 || G[2] < 4)
        return ORC_EINVAL;
    const int64_t X = out_dim[0], Y = out_dim[1], Z = out_dim[2], N = X * Y * Z;
    const int64_t GN = G[0] * G[1] * G[2];
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < X; ++x)
        for (int64_t y = 0; y < Y; ++y)
            for (int64_t z = 0; z < Z; ++z) {
                int64_t ix, iy, iz;
                float tx, ty, tz, Bx[4], By[4], Bz[4];
                bspline_cell_f32(x, X, G[0], &ix, &tx);
                bspline_cell_f32(y, Y, G[1], &iy, &ty);
                bspline_cell_f32(z, Z, G[2], &iz, &tz);
                bspline_basis_f32(tx, Bx);
                bspline_basis_f32(ty, By);
                bspline_basis_f32(tz, Bz);
                const int64_t v = (x * Y + y) * Z + z;
                for (int comp = 0; comp < 3; ++comp) {
                    float s = 0.0f;
                    for (int c = 0; c < 4; ++c) {
                        float P = 0.0f;
                        for (int a = 0; a < 4; ++a) {
                            float sa = 0.0f;
                            for (int b = 0; b < 4; ++b)
                                sa = fmaf(By[b],
                                          ctrl[comp * GN + ((ix + a) * G[1] + (iy + b)) * G[2] +
                                               (iz + c)],
                                          sa);
                            P = fmaf(Bx[a], sa, P);
                        }
                        s = fmaf(Bz[c], P, s);
                    }
                    u[comp * N + v] = s;
                }
            }
    return ORC_OK;
}

/* Adjoint of the upsampling: g_C = B^T g_u, the literal transpose sum. */
int orc_bspline_adjoint(const double *g_u, const int64_t *out_dim, const int64_t *G, double *g_ctrl)
{
    if (!g_u || !g_ctrl || !dims_ok(out_dim) || !G || G[0] < 4 || G[1] < 4 || G[2] < 4)
        return ORC_EINVAL;
    const int64_t X = out_dim[0], Y = out_dim[1], Z = out_dim[2], N = X * Y * Z;
    const int64_t GN = G[0] * G[1] * G[2];
    memset(g_ctrl, 0, sizeof(double) * 3 * (size_t)GN);
    for (int64_t x = 0; x < X; ++x)
        for (int64_t y = 0; y < Y; ++y)
            for (int64_t z = 0; z < Z; ++z) {
                int64_t ix, iy, iz;
                double tx, ty, tz, Bx[4], By[4], Bz[4];
                bspline_cell(x, X, G[0], &ix, &tx);
                bspline_cell(y, Y, G[1], &iy, &ty);
                bspline_cell(z, Z, G[2], &iz, &tz);
                bspline_basis(tx, Bx);
                bspline_basis(ty, By);
                bspline_basis(tz, Bz);
                int64_t v = (x * Y + y) * Z + z;
                for (int comp = 0; comp < 3; ++comp)
                    for (int a = 0; a < 4; ++a)
                        for (int b = 0; b < 4; ++b)
                            for (int c = 0; c < 4; ++c)
                                g_ctrl[comp * GN + ((ix + a) * G[1] + (iy + b)) * G[2] + (iz + c)] +=
                                    Bx[a] * By[b] * Bz[c] * g_u[comp * N + v];
            }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Resampling pre-step (Sec. "Pre- and post-processing"): before a volume of */
/* voxel spacing u_k is resampled to spacing r, it is smoothed by a Gaussian */
/* g(x) proportional to exp(-sum_k x_k^2 / sigma_k^2) with                    */
/* sigma_k = max(r / u_k - 1, 0) / 3 (in input voxels).  The kernel as        */
/* printed has no factor 2 in the exponent, so its standard deviation per     */
/* axis is sigma_k / sqrt(2).  Readings: the separable kernel is sampled at  */
/* integer offsets |d| <= R_k = floor(3 sigma_k / sqrt(2) + 0.5) (three       */
/* standard deviations) and normalised to sum 1; voxels beyond the volume    */
/* repeat the nearest edge voxel; sigma_k = 0 leaves axis k unchanged.        */
/* ------------------------------------------------------------------------ */

void orc_resample_sigma(const double *spacing, double target, double *sigma)
{
    for (int k = 0; k < 3; ++k) {
        double s = (target / spacing[k] - 1.0) / 3.0;
        sigma[k] = s > 0.0 ? s : 0.0;
    }
}

static int64_t gauss_radius(double sigma)
{
    return sigma > 0.0 ? (int64_t)floor(3.0 * sigma / sqrt(2.0) + 0.5) : 0;
}

/* One axis of the separable smoothing, in place through a scratch line. */
static void smooth_axis(double *vol, const int64_t *dim, int axis, double sigma)
{
    const int64_t R = gauss_radius(sigma);
    if (R == 0)
        return;
    double *w = malloc(sizeof(double) * (size_t)(R + 1));
    double sum = 0.0;
    for (int64_t d = 0; d <= R; ++d) {
        w[d] = exp(-(double)(d * d) / (sigma * sigma));
        sum += d == 0 ? w[d] : 2.0 * w[d];
    }
    for (int64_t d = 0; d <= R; ++d)
        w[d] /= sum;
    const int64_t n = dim[axis];
    const int64_t stride = axis == 0 ? dim[1] * dim[2] : axis == 1 ? dim[2] : 1;
    const int64_t lines = dim[0] * dim[1] * dim[2] / n;
#pragma omp parallel
    {
        double *line = malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t l = 0; l < lines; ++l) {
            /* base of line l: the other two coordinates in C order */
            int64_t base;
            if (axis == 2)
                base = l * n;
            else if (axis == 1)
                base = (l / dim[2]) * dim[1] * dim[2] + (l % dim[2]);
            else
                base = l;
            for (int64_t i = 0; i < n; ++i)
                line[i] = vol[base + i * stride];
            for (int64_t i = 0; i < n; ++i) {
                double acc = 0.0;
                for (int64_t d = -R; d <= R; ++d) {
                    int64_t j = i + d;
                    j = j < 0 ? 0 : (j > n - 1 ? n - 1 : j);
                    acc += w[d < 0 ? -d : d] * line[j];
                }
                vol[base + i * stride] = acc;
            }
        }
        free(line);
    }
    free(w);
}

int orc_gaussian_smooth(const double *img, const int64_t *dim, const double *sigma, double *out)
{
    if (!img || !out || !dims_ok(dim) || !sigma)
        return ORC_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (!(sigma[k] >= 0.0))
            return ORC_EINVAL;
    const int64_t N = dim[0] * dim[1] * dim[2];
    memcpy(out, img, sizeof(double) * (size_t)N);
    if (N == 0)
        return ORC_OK;
    for (int k = 0; k < 3; ++k)
        smooth_axis(out, dim, k, sigma[k]);
    return ORC_OK;
}
