"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bars: labels and Philox words bit-exact; Box-Muller Gaussians within
1e-6 * max(1, |n|); intensities within 1e-5 * max(|ref|, R) with R = 1 for
windowed [0,1] output and R = 1000 HU for HU output; gradients within 1e-4
normwise per tensor (and elementwise 1e-4 * max(|ref|, 1e-2 ||ref||_inf)).
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_1811_11226_amd as ctaug
from synth import AugmentRanges, PhotoParams, configs, draw_affine_params, draw_photo, \
    identity_affine_params, phantom_pair

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def assert_intensity(got, ref, windowed, what=""):
    R = 1.0 if windowed else 1000.0
    err = np.abs(got.astype(np.float64) - ref) / np.maximum(np.abs(ref), R)
    i = int(np.argmax(err)) if err.size else 0
    assert err.size == 0 or err.max() <= 1e-5, \
        f"{what}: max scaled error {err.max():.3e} at {np.unravel_index(i, err.shape)}: " \
        f"got {got.ravel()[i]!r} ref {ref.ravel()[i]!r}"


def assert_grad(got, ref, what=""):
    got = got.astype(np.float64)
    nref = np.linalg.norm(ref)
    assert np.linalg.norm(got - ref) <= 1e-4 * max(nref, 1e-30), \
        f"{what}: normwise {np.linalg.norm(got - ref) / max(nref, 1e-30):.3e}"
    # (an all-zero reference takes the normwise bar above: got must be zero)
    floor = max(1e-2 * np.abs(ref).max() if ref.size else 0.0, np.finfo(np.float64).tiny)
    err = np.abs(got - ref) / np.maximum(np.abs(ref), floor)
    assert err.size == 0 or err.max() <= 1e-4, f"{what}: elementwise {err.max():.3e}"


def run_job(job, M=None, out_dim=None, photo="job"):
    if M is None:
        _, M = ctaug.affine_matrix(job.prm, job.in_dim, job.out_dim)
    ph = job.photo if photo == "job" else photo
    od = job.out_dim if out_dim is None else out_dim
    img = _t(job.img)
    lbl = _t(job.lbl) if job.lbl is not None else None
    out, lout = ctaug.warp_affine(img, M, lbl=lbl, fill=job.fill, label_fill=job.label_fill,
                                  photo=ph, out_dim=od)
    ref, lref = oracle.warp(job.img, M, od, lbl=job.lbl, fill=job.fill,
                            label_fill=job.label_fill, photo=ph)
    return M, _np(out), (_np(lout) if lout is not None else None), ref, lref


# ---------------------------------------------------------------------------
# Noise: Philox words bit-exact, Gaussians within 1e-6
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed,vol,v0,n", [
    (0, 0, 0, 4096),
    (20181129, 3, 1, 10001),                      # unaligned start, ragged end
    (2 ** 64 - 1, 2 ** 32 - 1, 2 ** 34 + 2, 777),  # high counter word in use
    (123456789, 15, 84 * 2 ** 20 - 5, 1 << 16),
])
def test_noise_words_and_gaussians(seed, vol, v0, n):
    g, w = ctaug.noise(seed, vol, v0, n, gauss=True, words=True)
    words = _np(w).view(np.uint32)
    ng = ((v0 + n - 1) >> 2) - (v0 >> 2) + 1
    ref_w = oracle.noise_words(seed, vol, v0 >> 2, ng)
    assert np.array_equal(words, ref_w)
    ref_g = oracle.gauss(seed, vol, v0, n)
    err = np.abs(_np(g).astype(np.float64) - ref_g) / np.maximum(1.0, np.abs(ref_g))
    assert err.max() <= 1e-6, f"gaussian error {err.max():.3e}"


def test_gaussians_many_samples_within_bound():
    n = 1 << 22
    g, _ = ctaug.noise(987654321, 7, 0, n)
    ref = oracle.gauss(987654321, 7, 0, n)
    err = np.abs(_np(g).astype(np.float64) - ref) / np.maximum(1.0, np.abs(ref))
    assert err.max() <= 1e-6, f"gaussian error {err.max():.3e} at |n|={abs(ref[np.argmax(err)])}"


def _bm_check(words):
    got = _np(ctaug.box_muller(_t(words.view(np.int32)))).astype(np.float64)
    ref = oracle.box_muller(words)
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    return err.max(), ref[np.argmax(err)]


def test_box_muller_exhaustive_uniforms():
    """Every one of the 2^23 uniforms as the radius word (paired with a
    permutation of all angle uniforms), then the largest radius paired with
    every angle uniform."""
    n = 1 << 23
    rng = np.random.default_rng(13)
    k = np.arange(n, dtype=np.uint32)
    low = rng.integers(0, 512, size=(2, n), dtype=np.uint32)
    w = np.empty(2 * n, dtype=np.uint32)
    w[0::2] = (k << 9) | low[0]
    w[1::2] = (rng.permutation(k) << 9) | low[1]
    e1, at1 = _bm_check(w)
    w[0::2] = 0                                   # U = 2^-24: r = sqrt(48 ln 2)
    w[1::2] = k << 9
    e2, at2 = _bm_check(w)
    assert e1 <= 1e-6 and e2 <= 1e-6, (e1, at1, e2, at2)


# ---------------------------------------------------------------------------
# Forward warp: C1 full size, exact invariants, ragged and edge cases
# ---------------------------------------------------------------------------

def test_c1_full_size_parity():
    job = configs.c1()[0]
    _, out, lout, ref, lref = run_job(job)
    assert np.array_equal(lout, lref)
    assert_intensity(out, ref, windowed=True, what="c1")


def test_c1_hu_output_no_window():
    job = configs.c1()[0]
    ph = PhotoParams(**{**job.photo.__dict__, "window": False})
    _, out, lout, ref, lref = run_job(job, photo=ph)
    assert np.array_equal(lout, lref)
    assert_intensity(out, ref, windowed=False, what="c1-hu")


def test_identity_and_integer_shift_bit_exact():
    img, lbl = phantom_pair((37, 29, 23), seed=3)
    for shift in [(0, 0, 0), (3, -2, 5), (-40, 0, 0)]:
        M = np.zeros((3, 4), np.float32)
        M[:, :3] = np.eye(3)
        M[:, 3] = shift
        out, lout = ctaug.warp_affine(_t(img), M.ravel(), lbl=_t(lbl), fill=-1000.0)
        ref, lref = oracle.warp(img, M.ravel(), img.shape, lbl=lbl, fill=-1000.0)
        assert np.array_equal(_np(out).astype(np.float64), ref)
        assert np.array_equal(_np(lout), lref)


def test_rot90_bit_exact():
    n = 32
    img, lbl = phantom_pair((n, n, 20), seed=4)
    A = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], np.float64)
    c = (np.array(img.shape) - 1) / 2
    M = np.concatenate([A, (c - A @ c)[:, None]], axis=1).astype(np.float32).ravel()
    out, lout = ctaug.warp_affine(_t(img), M, lbl=_t(lbl))
    assert np.array_equal(_np(out), np.rot90(img, k=-1, axes=(0, 1)).astype(np.float32))
    assert np.array_equal(_np(lout), np.rot90(lbl, k=-1, axes=(0, 1)))


@pytest.mark.parametrize("in_dim,out_dim,dtype", [
    ((33, 29, 21), (31, 27, 19), np.float32),     # ragged tiles, Zo % 4 != 0
    ((40, 36, 30), (17, 9, 7), np.int16),
    ((96, 101, 130), (120, 120, 160), np.int16),  # crop larger than some axes
    ((5, 6, 7), (64, 64, 64), np.float32),        # mostly outside
    ((64, 64, 64), (1, 1, 1), np.float32),
    ((64, 48, 32), (4, 8, 32), np.int16),         # exactly one tile
])
def test_ragged_shapes_parity(in_dim, out_dim, dtype):
    rng = np.random.default_rng(sum(in_dim) + sum(out_dim))
    img, lbl = phantom_pair(in_dim, seed=int(rng.integers(1 << 30)))
    prm = draw_affine_params(rng, AugmentRanges(), in_dim, out_dim)
    ph = draw_photo(rng, AugmentRanges(), seed=int(rng.integers(1 << 62)), volume_id=5)
    job = configs.Job(img=img.astype(dtype), lbl=lbl, out_dim=out_dim, prm=prm, photo=ph)
    _, out, lout, ref, lref = run_job(job)
    assert np.array_equal(lout, lref)
    assert_intensity(out, ref, windowed=True, what=str(out_dim))


@pytest.mark.parametrize("scale", [(3.5, 4.0), (0.3, 0.4)])
def test_large_and_small_footprints(scale):
    """Strong downsampling makes tile footprints exceed the LDS reservation
    (direct-gather fallback); strong upsampling makes them tiny."""
    rng = np.random.default_rng(int(scale[0] * 10))
    in_dim, out_dim = (200, 180, 160), (44, 40, 36)
    img, lbl = phantom_pair(in_dim, seed=12)
    prm = draw_affine_params(rng, AugmentRanges(scale=scale), in_dim, out_dim)
    ph = draw_photo(rng, AugmentRanges(), seed=5, volume_id=1)
    job = configs.Job(img=img, lbl=lbl, out_dim=out_dim, prm=prm, photo=ph)
    _, out, lout, ref, lref = run_job(job)
    assert np.array_equal(lout, lref)
    assert_intensity(out, ref, windowed=True)


@pytest.mark.parametrize("shift", [-0.5, 0.5, -0.75, 0.25])
@pytest.mark.parametrize("dtype", [np.float32, np.int16])
@pytest.mark.parametrize("lds", [0, -1])
def test_first_and_last_volume_elements(shift, dtype, lds):
    """Half-voxel shifts put valid corners at the very first / last element of
    the volume next to out-of-volume corners (regression: merged wide loads
    must never straddle the buffer ends)."""
    dims = (12, 10, 8)
    rng = np.random.default_rng(3)
    img = rng.integers(-1000, 1500, dims).astype(dtype)
    lbl = rng.integers(0, 6, dims).astype(np.int8)
    M = np.zeros((3, 4), np.float32)
    M[:, :3] = np.eye(3)
    M[:, 3] = shift
    M = M.ravel()
    out = torch.empty(dims, dtype=torch.float32, device=DEV)
    lout = torch.empty(dims, dtype=torch.int8, device=DEV)
    plan = ctaug.BatchPlan([ctaug.make_job(_t(img), M, out, _t(lbl), lout, fill=-1000.0)],
                           tile=(4, 8, 8), lds_cells=lds, lds_format=int(dtype == np.int16))
    plan.launch()
    ref, lref = oracle.warp(img, M, dims, lbl=lbl, fill=-1000.0)
    assert np.array_equal(_np(lout), lref)
    assert_intensity(_np(out), ref, windowed=False)
    plan.close()
    g = rng.standard_normal(dims).astype(np.float32)
    g_img, g_M = ctaug.warp_affine_backward(_t(img), M, _t(g))
    r_img, r_M, _ = oracle.warp_backward(img, M, g)
    assert_grad(_np(g_img), r_img, "g_img")
    assert_grad(_np(g_M), r_M, "g_M")


def test_unaligned_output_pointer_uses_scalar_path():
    job = configs.c1(dims=(24, 20, 16))[0]
    _, M = ctaug.affine_matrix(job.prm, job.in_dim, job.out_dim)
    base = torch.empty(int(np.prod(job.out_dim)) + 1, dtype=torch.float32, device=DEV)
    out = base[1:].view(job.out_dim)                 # 4-byte but not 16-byte aligned
    lbase = torch.empty(int(np.prod(job.out_dim)) + 1, dtype=torch.int8, device=DEV)
    lout = lbase[1:].view(job.out_dim)
    ctaug.warp_affine(_t(job.img), M, lbl=_t(job.lbl), fill=job.fill, photo=job.photo, out=out,
                      lbl_out=lout)
    ref, lref = oracle.warp(job.img, M, job.out_dim, lbl=job.lbl, fill=job.fill, photo=job.photo)
    assert np.array_equal(_np(lout), lref)
    assert_intensity(_np(out), ref, windowed=True)


def test_no_labels_no_photo():
    job = configs.c1(dims=(40, 40, 24))[0]
    _, M = ctaug.affine_matrix(job.prm, job.in_dim, job.out_dim)
    out, lout = ctaug.warp_affine(_t(job.img), M, fill=job.fill)
    assert lout is None
    ref, _ = oracle.warp(job.img, M, job.out_dim, fill=job.fill)
    assert_intensity(_np(out), ref, windowed=False)


def test_empty_volumes_are_noops():
    img = torch.zeros((0, 4, 4), dtype=torch.float32, device=DEV)
    out, _ = ctaug.warp_affine(img, np.eye(3, 4).ravel(), fill=7.0, out_dim=(3, 4, 5))
    assert np.all(_np(out) == 7.0)                   # empty input: everything is fill
    img = torch.zeros((4, 4, 4), dtype=torch.float32, device=DEV)
    out, _ = ctaug.warp_affine(img, np.eye(3, 4).ravel(), out_dim=(0, 4, 4))
    assert out.numel() == 0


def test_fused_equals_unfused_bit_exact():
    job = configs.c1(dims=(64, 48, 40))[0]
    _, M = ctaug.affine_matrix(job.prm, job.in_dim, job.out_dim)
    fused, _ = ctaug.warp_affine(_t(job.img), M, fill=job.fill, photo=job.photo)
    plain, _ = ctaug.warp_affine(_t(job.img), M, fill=job.fill)
    ctaug.photometric_noise(plain, job.photo)
    assert torch.equal(fused, plain)


@pytest.mark.parametrize("occ", [(3.0, 11.0), (-5.5, 0.25), (20.5, 20.7), (30.0, 99.0)])
@pytest.mark.parametrize("dtype,odd", [(np.float32, False), (np.int16, True)])
def test_occlusion_parity(occ, dtype, odd):
    """Random occlusion of an output z-slab: labels bit-exact, intensities
    against the oracle, fused = unfused through photometric_noise."""
    dims = (40, 36, 37 if odd else 40)
    job = configs.c1(dims=dims)[0]
    job.img = job.img.astype(dtype)
    ph = job.photo
    ph.occlude, ph.occ_lo, ph.occ_hi = True, occ[0], occ[1]
    _, out, lout, ref, lref = run_job(job)
    assert np.array_equal(lout, lref)
    assert_intensity(out, ref, windowed=True, what=f"occlusion {occ}")
    _, M = ctaug.affine_matrix(job.prm, job.in_dim, job.out_dim)
    plain, _ = ctaug.warp_affine(_t(job.img), M, fill=job.fill)
    ctaug.photometric_noise(plain, ph)
    fused, _ = ctaug.warp_affine(_t(job.img), M, fill=job.fill, photo=ph)
    assert torch.equal(fused, plain)


def test_occlusion_in_batch_plan():
    T = _batch_jobs(n=3, out_dim=(36, 30, 44))
    rng = np.random.default_rng(77)
    jobs, phs = [], []
    for (j, M, img, lbl, out, lout) in T:
        ph = draw_photo(rng, AugmentRanges(occlusion=12.0), seed=9, volume_id=j.volume_id,
                        out_z=44)
        phs.append(ph)
        jobs.append(ctaug.make_job(img, M, out, lbl, lout, fill=j.fill, photo=ph))
    plan = ctaug.BatchPlan(jobs, tile=(16, 16, 16), lds_cells=8176)
    plan.launch()
    for (j, M, img, lbl, out, lout), ph in zip(T, phs):
        s_out, s_lout = ctaug.warp_affine(img, M, lbl=lbl, fill=j.fill, photo=ph,
                                          out_dim=j.out_dim)
        assert torch.equal(out, s_out) and torch.equal(lout, s_lout)
        ref, lref = oracle.warp(j.img, M, j.out_dim, lbl=j.lbl, fill=j.fill, photo=ph)
        assert np.array_equal(_np(lout), lref)
        assert_intensity(_np(out), ref, windowed=True)
    plan.close()


def test_photometric_noise_parity():
    rng = np.random.default_rng(5)
    v = rng.uniform(-1200, 1500, (30, 17, 11)).astype(np.float32)
    for window in (True, False):
        ph = PhotoParams(gain=1.07, offset=-13.0, sigma=12.5, win_lo=-900, win_hi=1100,
                         gamma=0.85, window=window, seed=42, volume_id=9)
        t = _t(v)
        ctaug.photometric_noise(t, ph)
        ref = oracle.photometric(v.astype(np.float64), ph)
        assert_intensity(_np(t), ref, windowed=window)


def test_repeat_runs_bit_identical():
    job = configs.c1(dims=(50, 44, 36))[0]
    _, M = ctaug.affine_matrix(job.prm, job.in_dim, job.out_dim)
    a, la = ctaug.warp_affine(_t(job.img), M, lbl=_t(job.lbl), photo=job.photo)
    b, lb = ctaug.warp_affine(_t(job.img), M, lbl=_t(job.lbl), photo=job.photo)
    assert torch.equal(a, b) and torch.equal(la, lb)


# ---------------------------------------------------------------------------
# Displacement warp and B-spline field
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("amp,out_dim,dtype", [(3.0, (38, 34, 24), np.float32),
                                               (80.0, (30, 26, 21), np.int16),
                                               (0.4, (45, 40, 37), np.int16)])
def test_displacement_warp_parity_given_field(amp, out_dim, dtype):
    """Displacement warps: per-tile footprints from the reduced coordinates
    (LDS staging), and a wild field whose tiles exceed the reservation
    (direct gathers)."""
    rng = np.random.default_rng(6 + int(amp))
    in_dim = (40, 36, 28)
    img, lbl = phantom_pair(in_dim, seed=77)
    prm = draw_affine_params(rng, AugmentRanges(), in_dim, out_dim)
    _, M = ctaug.affine_matrix(prm, in_dim, out_dim)
    disp = rng.uniform(-amp, amp, (3,) + out_dim).astype(np.float32)
    ph = draw_photo(rng, AugmentRanges(), seed=99, volume_id=1)
    out, lout = ctaug.warp_displacement(_t(img.astype(dtype)), M, _t(disp), lbl=_t(lbl),
                                        photo=ph)
    ref, lref = oracle.warp(img, M, out_dim, lbl=lbl, disp=disp, photo=ph)
    assert np.array_equal(_np(lout), lref)
    assert_intensity(_np(out), ref, windowed=True)


@pytest.mark.parametrize("out_dim,grid", [((64, 48, 40), (8, 8, 8)), ((33, 17, 9), (6, 5, 7)),
                                          ((1, 12, 16), (4, 4, 4))])
def test_bspline_upsample_parity(out_dim, grid):
    """Equal bit for bit to the oracle's FP32 parity-mode field, and within
    FP32 rounding of the FP64 definition."""
    rng = np.random.default_rng(7)
    C = (4.0 * rng.standard_normal((3,) + grid)).astype(np.float32)
    u = _np(ctaug.bspline_upsample(_t(C), out_dim))
    assert np.array_equal(u.view(np.uint32), oracle.bspline_upsample_f32(C, out_dim).view(np.uint32))
    ref = oracle.bspline_upsample(C, out_dim)
    err = np.abs(u.astype(np.float64) - ref).max()
    assert err <= 1e-5 * np.abs(C).max(), err


@pytest.mark.parametrize("out_dim,grid", [((64, 48, 40), (8, 8, 8)), ((70, 130, 9), (6, 9, 7))])
def test_bspline_adjoint_parity(out_dim, grid):
    rng = np.random.default_rng(8)
    g = rng.standard_normal((3,) + out_dim).astype(np.float32)
    gc = ctaug.bspline_upsample_adjoint(_t(g), grid)
    ref = oracle.bspline_adjoint(g.astype(np.float64), grid)
    assert_grad(_np(gc), ref, "g_ctrl")


@pytest.mark.parametrize("in_dim,out_dim,grid,dtype,amp", [
    ((40, 36, 28), (38, 34, 24), (8, 8, 8), np.float32, 3.0),
    ((40, 36, 28), (30, 26, 21), (6, 5, 7), np.int16, 6.0),      # ragged z, unaligned runs
    ((24, 20, 60), (20, 18, 52), (5, 6, 40), np.float32, 1.5),   # controls < 4 voxels apart
    ((33, 30, 18), (33, 30, 1), (4, 4, 4), np.int16, 2.0),       # single slice
])
def test_warp_bspline_equals_upsample_then_warp(in_dim, out_dim, grid, dtype, amp):
    """The fused nonrigid warp evaluates the B-spline field with the upsampling
    kernel's operations in the same order: bit-identical to upsampling the
    field and warping with it, labels and noise included."""
    rng = np.random.default_rng(sum(out_dim) + grid[2])
    img, lbl = phantom_pair(in_dim, seed=91)
    prm = draw_affine_params(rng, AugmentRanges(), in_dim, out_dim)
    _, M = ctaug.affine_matrix(prm, in_dim, out_dim)
    C = (amp * rng.standard_normal((3,) + grid)).astype(np.float32)
    ph = draw_photo(rng, AugmentRanges(), seed=5, volume_id=2)
    ti, tl, tc = _t(img.astype(dtype)), _t(lbl), _t(C)
    out, lout = ctaug.warp_bspline(ti, M, tc, lbl=tl, photo=ph, out_dim=out_dim)
    u = ctaug.bspline_upsample(tc, out_dim)
    out2, lout2 = ctaug.warp_displacement(ti, M, u, lbl=tl, photo=ph)
    assert np.array_equal(_np(out).view(np.uint32), _np(out2).view(np.uint32))
    assert np.array_equal(_np(lout), _np(lout2))


@pytest.mark.parametrize("out_dim,grid,windowed,dtype", [
    ((44, 40, 36), (8, 8, 8), True, np.int16),
    ((37, 29, 23), (6, 7, 5), False, np.float32),
    ((20, 18, 52), (5, 6, 40), True, np.float32),     # per-voxel profiles
])
def test_warp_bspline_parity_with_oracle(out_dim, grid, windowed, dtype):
    """Fused nonrigid warp against the oracle warp with the oracle's FP32
    parity-mode field: labels bit-exact, intensities within 1e-5."""
    in_dim = (48, 44, 40)
    rng = np.random.default_rng(61 + grid[0])
    img, lbl = phantom_pair(in_dim, seed=8)
    prm = draw_affine_params(rng, AugmentRanges(), in_dim, out_dim)
    _, M = ctaug.affine_matrix(prm, in_dim, out_dim)
    C = (4.0 * rng.standard_normal((3,) + grid)).astype(np.float32)
    ph = draw_photo(rng, AugmentRanges(window=windowed), seed=17, volume_id=4)
    out, lout = ctaug.warp_bspline(_t(img.astype(dtype)), M, _t(C), lbl=_t(lbl), photo=ph,
                                   out_dim=out_dim)
    u = oracle.bspline_upsample_f32(C, out_dim)
    ref, lref = oracle.warp(img, M, out_dim, lbl=lbl, disp=u, photo=ph)
    assert np.array_equal(_np(lout), lref)
    assert_intensity(_np(out), ref, windowed=windowed, what="fused B-spline warp")


@pytest.mark.parametrize("in_dim,out_dim,grid,dtype,fused", [
    ((40, 36, 30), (44, 40, 36), (8, 8, 8), np.float32, True),
    ((40, 36, 30), (37, 29, 23), (6, 7, 5), np.int16, True),      # ragged tiles
    ((24, 20, 60), (20, 18, 52), (5, 6, 40), np.float32, False),  # z controls < 2 voxels apart
    ((40, 36, 30), (48, 40, 44), (10, 10, 10), np.float32, False),  # 3000 control entries
])
def test_warp_bspline_backward_parity(in_dim, out_dim, grid, dtype, fused):
    """Adjoint of the fused nonrigid warp (image, M and control grid) against
    the oracle's warp adjoint, on its FP32 parity-mode field, followed by its
    B-spline adjoint; both the fused control-grid reduction and the dense
    route (grids it does not take) are covered."""
    rng = np.random.default_rng(71 + grid[2])
    img, _ = phantom_pair(in_dim, seed=12)
    img = img.astype(dtype)
    prm = draw_affine_params(rng, AugmentRanges(), in_dim, out_dim)
    _, M = ctaug.affine_matrix(prm, in_dim, out_dim)
    C = (3.0 * rng.standard_normal((3,) + grid)).astype(np.float32)
    u = oracle.bspline_upsample_f32(C, out_dim)
    g = rng.standard_normal(out_dim).astype(np.float32)
    od = (ctypes.c_int64 * 3)(*out_dim)
    G = (ctypes.c_int64 * 3)(*grid)
    L = ctaug._lib.load()
    m_bytes = ctaug.ops.warp_backward_workspace(out_dim)     # rows x 12 doubles
    rows = m_bytes // 96
    ws_fused = -(-m_bytes // 256) * 256 + (rows + min(rows, 64)) * 3 * int(np.prod(grid)) * 8
    assert (int(L.ctaug_warp_bspline_backward_workspace(od, G)) == ws_fused) == fused
    g_img, g_M, g_c = ctaug.warp_bspline_backward(_t(img), M, _t(C), _t(g))
    r_img, r_M, r_u = oracle.warp_backward(img, M, g, disp=u, want_u=True)
    assert_grad(_np(g_img), r_img, "g_img")
    assert_grad(_np(g_M), r_M, "g_M")
    assert_grad(_np(g_c), oracle.bspline_adjoint(r_u, grid), "g_ctrl")
    # deterministic: a second run gives the same bits for M and the control grid
    _, g_M2, g_c2 = ctaug.warp_bspline_backward(_t(img), M, _t(C), _t(g), want_img=False)
    assert np.array_equal(_np(g_M).view(np.uint64), _np(g_M2).view(np.uint64))
    assert np.array_equal(_np(g_c).view(np.uint32), _np(g_c2).view(np.uint32))


def test_warp_bspline_backward_empty_output_zeroes_gradients():
    img = _t(np.zeros((8, 8, 8), np.float32))
    C = _t(np.ones((3, 5, 5, 5), np.float32))
    g = torch.empty((0, 8, 8), dtype=torch.float32, device=DEV)
    _, g_M, g_c = ctaug.warp_bspline_backward(img, np.eye(3, 4).ravel(), C, g, want_img=False)
    assert not _np(g_M).any() and not _np(g_c).any()


def test_autograd_fused_bspline_warp():
    """torch.autograd through the fused nonrigid warp against the oracle."""
    from paper_1811_11226_amd import autograd as ag
    rng = np.random.default_rng(44)
    dims = (26, 22, 30)
    img_np, _ = phantom_pair(dims, seed=14)
    img_np = img_np.astype(np.float32)
    prm = draw_affine_params(rng, AugmentRanges(), dims, dims)
    _, M32 = ctaug.affine_matrix(prm, dims, dims)
    ctrl = rng.normal(0.0, 2.0, (3, 7, 6, 8)).astype(np.float32)
    u = oracle.bspline_upsample_f32(ctrl, dims)
    g = rng.standard_normal(dims).astype(np.float32)
    img = _t(img_np).requires_grad_(True)
    M = torch.tensor(M32.astype(np.float64), requires_grad=True)
    c = _t(ctrl).requires_grad_(True)
    out = ag.warp_bspline(img, M, c)
    (out * _t(g)).sum().backward()
    r_img, r_M, r_u = oracle.warp_backward(img_np, M32, g, disp=u, want_u=True)
    assert_grad(_np(img.grad), r_img, "autograd g_img")
    assert_grad(M.grad.numpy(), r_M, "autograd g_M")
    assert_grad(_np(c.grad), oracle.bspline_adjoint(r_u, (7, 6, 8)), "autograd g_ctrl")


# ---------------------------------------------------------------------------
# Backward
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dims,dtype", [((48, 40, 36), np.float32), ((33, 29, 21), np.int16)])
def test_affine_backward_parity(dims, dtype):
    rng = np.random.default_rng(9)
    img, _ = phantom_pair(dims, seed=5)
    prm = draw_affine_params(rng, AugmentRanges(), dims, dims)
    _, M = ctaug.affine_matrix(prm, dims, dims)
    g = rng.standard_normal(dims).astype(np.float32)
    g_img, g_M = ctaug.warp_affine_backward(_t(img.astype(dtype)), M, _t(g))
    r_img, r_M, _ = oracle.warp_backward(img, M, g)
    assert_grad(_np(g_img), r_img, "g_img")
    assert_grad(_np(g_M), r_M, "g_M")
    # the image adjoint alone (no staged corner values)
    g_img2, none = ctaug.warp_affine_backward(_t(img.astype(dtype)), M, _t(g), want_M=False)
    assert none is None
    assert_grad(_np(g_img2), r_img, "g_img alone")


@pytest.mark.parametrize("gscale,outliers", [(1e30, 0.0), (1e-30, 0.0), (1.0, 1e-12),
                                             (1e-36, 0.0)])
def test_affine_backward_gradient_magnitudes(gscale, outliers):
    """The image adjoint sums a tile in fixed point scaled by the tile's
    largest |g| (32-bit here, as the map bounds a cell's samples; a tile
    maximum below 2^-96 takes per-corner FP32 atomics): huge gradients, tiny
    ones (down to FP32 subnormal products), and a few normal values among
    1e-12 ones (rounded within 2^(b - 30) of the tile maximum), against the
    oracle."""
    rng = np.random.default_rng(int(abs(np.log10(gscale))) + 3)
    dims = (40, 36, 44)
    img, _ = phantom_pair(dims, seed=25)
    img = img.astype(np.float32)
    prm = draw_affine_params(rng, AugmentRanges(), dims, dims)
    _, M = ctaug.affine_matrix(prm, dims, dims)
    g = rng.standard_normal(dims) * gscale
    if outliers:
        g = np.where(rng.random(dims) < 0.01, g, g * outliers)
    g = g.astype(np.float32)
    g_img, g_M = ctaug.warp_affine_backward(_t(img), M, _t(g))
    r_img, r_M, _ = oracle.warp_backward(img, M, g)
    assert_grad(_np(g_img), r_img, "g_img")
    assert_grad(_np(g_M), r_M, "g_M")


@pytest.mark.parametrize("in_dim,out_dim,scale,dtype", [
    ((264, 128, 64), (264, 128, 64), (0.8, 1.2), np.float32),   # > 2048 tiles: strided WGs
    ((120, 100, 80), (30, 25, 20), (3.5, 4.0), np.int16),       # footprints beyond LDS
    ((40, 36, 30), (70, 60, 52), (0.45, 0.55), np.float32),     # upsampling, tiny footprints
    ((30, 28, 24), (96, 90, 80), (0.28, 0.32), np.float32),     # > 2^7 samples per cell: 64-bit sums
])
def test_affine_backward_tiles_and_footprints(in_dim, out_dim, scale, dtype):
    """Image and parameter adjoints across persistent tile striding, tiles
    whose footprint exceeds the LDS reservation (global atomics), and
    crops with out-of-volume tiles."""
    rng = np.random.default_rng(int(in_dim[0]))
    img, _ = phantom_pair(in_dim, seed=8)
    prm = draw_affine_params(rng, AugmentRanges(scale=scale), in_dim, out_dim)
    _, M = ctaug.affine_matrix(prm, in_dim, out_dim)
    g = rng.standard_normal(out_dim).astype(np.float32)
    g_img, g_M = ctaug.warp_affine_backward(_t(img.astype(dtype)), M, _t(g))
    r_img, r_M, _ = oracle.warp_backward(img, M, g)
    assert_grad(_np(g_img), r_img, "g_img")
    assert_grad(_np(g_M), r_M, "g_M")


def test_affine_backward_param_only_and_singular_map():
    """grad_M alone (output-tiled kernel) and a singular A (no inverse map:
    the image adjoint falls back to per-corner atomics) against the oracle."""
    rng = np.random.default_rng(21)
    dims = (40, 36, 44)
    img, _ = phantom_pair(dims, seed=3)
    g = rng.standard_normal(dims).astype(np.float32)
    prm = draw_affine_params(rng, AugmentRanges(), dims, dims)
    _, M = ctaug.affine_matrix(prm, dims, dims)
    _, g_M = ctaug.warp_affine_backward(_t(img), M, _t(g), want_img=False)
    _, r_M, _ = oracle.warp_backward(img, M, g, want_img=False)
    assert_grad(_np(g_M), r_M, "g_M only")
    S = np.array([[0.5, 0.25, 0.0, 12.0], [0.0, 1.0, 0.0, 3.0], [1.0, 0.5, 0.0, 7.5]],
                 dtype=np.float32).ravel()         # rank 2: z does not move the sample
    g_img, g_M = ctaug.warp_affine_backward(_t(img), S, _t(g))
    r_img, r_M, _ = oracle.warp_backward(img, S, g)
    assert_grad(_np(g_img), r_img, "g_img singular")
    assert_grad(_np(g_M), r_M, "g_M singular")


def test_backward_calls_on_two_streams_agree_with_one_stream():
    """Independent backward calls running at once on two streams, each with
    its own workspace, give the parameter gradients bit for bit and the image
    gradients within the bar of the same calls made one after another."""
    rng = np.random.default_rng(61)
    dims = (40, 36, 44)
    cases = []
    for k in range(6):
        img, _ = phantom_pair(dims, seed=400 + k)
        prm = draw_affine_params(rng, AugmentRanges(), dims, dims)
        _, M = ctaug.affine_matrix(prm, dims, dims)
        g = rng.standard_normal(dims).astype(np.float32)
        cases.append((_t(img.astype(np.float32)), M, _t(g)))
    seq = [ctaug.warp_affine_backward(i, M, g) for i, M, g in cases]
    torch.cuda.synchronize()
    side = [torch.cuda.Stream(), torch.cuda.Stream()]
    ready = torch.cuda.Event()
    ready.record()
    for s in side:
        s.wait_event(ready)
    par = []
    for k, (i, M, g) in enumerate(cases):
        with torch.cuda.stream(side[k % 2]):
            par.append(ctaug.warp_affine_backward(i, M, g))
    for s in side:
        s.synchronize()
    for k, ((gi, gM), (pi, pM)) in enumerate(zip(seq, par)):
        assert np.array_equal(_np(gM).view(np.uint64), _np(pM).view(np.uint64)), f"g_M {k}"
        assert_grad(_np(pi), _np(gi).astype(np.float64), f"g_img {k}")


def test_affine_backward_adjoint_identity_gpu():
    rng = np.random.default_rng(10)
    dims = (40, 40, 40)
    x = rng.standard_normal(dims).astype(np.float32)
    y = rng.standard_normal(dims).astype(np.float32)
    prm = draw_affine_params(rng, AugmentRanges(), dims, dims)
    _, M = ctaug.affine_matrix(prm, dims, dims)
    Wx, _ = ctaug.warp_affine(_t(x), M, fill=0.0)
    WTy, _ = ctaug.warp_affine_backward(_t(x), M, _t(y), fill=0.0, want_M=False)
    Wx, WTy = _np(Wx).astype(np.float64), _np(WTy).astype(np.float64)
    lhs, rhs = np.vdot(Wx, y), np.vdot(x, WTy)
    # Higham: |fl(<a,b>) - <a,b>| <= gamma_k |a|^T |b|, k = accumulation chain length
    u = 2.0 ** -24
    k = 64     # upper bound on terms accumulated into one element
    bound = (k * u / (1 - k * u)) * (np.abs(Wx).ravel() @ np.abs(y).ravel() +
                                     np.abs(x).ravel() @ np.abs(WTy).ravel())
    assert abs(lhs - rhs) <= bound


@pytest.mark.parametrize("amp,dims,dtype", [(2.0, (36, 32, 28), np.float32),
                                            (60.0, (40, 36, 33), np.int16),
                                            (0.0, (30, 26, 40), np.float32)])
def test_displacement_backward_parity(amp, dims, dtype):
    """Displacement adjoint: tile footprints from the reduced coordinates
    (small fields: LDS accumulation; a wild field: tiles beyond the LDS
    reservation take per-corner atomics; zero field = affine)."""
    rng = np.random.default_rng(11 + int(amp))
    img, _ = phantom_pair(dims, seed=8)
    img = img.astype(dtype)
    prm = draw_affine_params(rng, AugmentRanges(), dims, dims)
    _, M = ctaug.affine_matrix(prm, dims, dims)
    disp = rng.uniform(-amp, amp, (3,) + dims).astype(np.float32)
    g = rng.standard_normal(dims).astype(np.float32)
    g_img, g_M, g_disp = ctaug.warp_displacement_backward(_t(img), M, _t(disp), _t(g))
    r_img, r_M, r_u = oracle.warp_backward(img, M, g, disp=disp, want_u=True)
    assert_grad(_np(g_img), r_img, "g_img")
    assert_grad(_np(g_M), r_M, "g_M")
    assert_grad(_np(g_disp), r_u, "g_disp")


def test_autograd_affine_with_photometrics():
    """gain, offset, noise and occlusion pass gain * grad_out (zero on the
    occluded slab) to the warp adjoint; the forward output matches the oracle."""
    from paper_1811_11226_amd import autograd as ag
    rng = np.random.default_rng(34)
    dims = (22, 26, 30)
    img_np, _ = phantom_pair(dims, seed=6)
    img_np = img_np.astype(np.float32)
    prm = draw_affine_params(rng, AugmentRanges(), dims, dims)
    _, M32 = ctaug.affine_matrix(prm, dims, dims)
    ph = draw_photo(rng, AugmentRanges(window=False, occlusion=8.0), seed=3, volume_id=1,
                    out_z=dims[2])
    assert ph.occlude
    g = rng.standard_normal(dims).astype(np.float32)
    img = _t(img_np).requires_grad_(True)
    M = torch.tensor(M32.astype(np.float64), requires_grad=True)
    out = ag.warp_affine(img, M, photo=ph)
    ref, _ = oracle.warp(img_np, M32, dims, photo=ph)
    assert_intensity(_np(out), ref, windowed=False, what="autograd forward")
    (out * _t(g)).sum().backward()
    r_img, r_M, _ = oracle.warp_backward(img_np, M32, g, photo=ph)
    assert_grad(_np(img.grad), r_img, "g_img")
    assert_grad(M.grad.numpy(), r_M, "g_M")
    # the windowed chain is refused by the library's adjoint
    out = ag.warp_affine(img, M, photo=draw_photo(rng, AugmentRanges(), seed=1, volume_id=0))
    with pytest.raises(ctaug._lib.CtaugError):
        out.sum().backward()


@pytest.mark.parametrize("kind", ["affine", "displacement", "bspline"])
def test_photometric_adjoint_in_the_kernels(kind):
    """The adjoint calls apply the photometric chain's adjoint (gain, zero on
    the occluded slab) themselves: against the oracle's adjoint of the same
    chain, for the three warps."""
    rng = np.random.default_rng(35)
    dims = (30, 26, 34)
    img_np, _ = phantom_pair(dims, seed=9)
    img_np = img_np.astype(np.float32)
    prm = draw_affine_params(rng, AugmentRanges(), dims, dims)
    _, M = ctaug.affine_matrix(prm, dims, dims)
    ph = draw_photo(rng, AugmentRanges(window=False, gain=(0.8, 0.8)), seed=4, volume_id=2)
    ph.occlude, ph.occ_lo, ph.occ_hi = True, 5.5, 14.0
    g = rng.standard_normal(dims).astype(np.float32)
    if kind == "affine":
        g_img, g_M = ctaug.warp_affine_backward(_t(img_np), M, _t(g), photo=ph)
        r_img, r_M, _ = oracle.warp_backward(img_np, M, g, photo=ph)
    elif kind == "displacement":
        disp = rng.uniform(-2.0, 2.0, (3,) + dims).astype(np.float32)
        g_img, g_M, g_d = ctaug.warp_displacement_backward(_t(img_np), M, _t(disp), _t(g),
                                                            photo=ph)
        r_img, r_M, r_u = oracle.warp_backward(img_np, M, g, disp=disp, photo=ph, want_u=True)
        assert_grad(_np(g_d), r_u, "g_disp")
    else:
        C = (2.0 * rng.standard_normal((3, 6, 6, 6))).astype(np.float32)
        g_img, g_M, g_c = ctaug.warp_bspline_backward(_t(img_np), M, _t(C), _t(g), photo=ph)
        u = oracle.bspline_upsample_f32(C, dims)
        r_img, r_M, r_u = oracle.warp_backward(img_np, M, g, disp=u, photo=ph, want_u=True)
        assert_grad(_np(g_c), oracle.bspline_adjoint(r_u, (6, 6, 6)), "g_ctrl")
    assert_grad(_np(g_img), r_img, f"{kind} g_img")
    assert_grad(_np(g_M), r_M, f"{kind} g_M")


def test_autograd_affine_and_nonrigid_chain():
    """torch.autograd through the library's adjoints: image and M gradients of
    the affine warp, and the control-grid gradient through B-spline
    upsampling and the displacement warp, against the oracle."""
    from paper_1811_11226_amd import autograd as ag
    rng = np.random.default_rng(33)
    dims = (24, 20, 28)
    img_np, _ = phantom_pair(dims, seed=4)
    img_np = img_np.astype(np.float32)
    prm = draw_affine_params(rng, AugmentRanges(), dims, dims)
    _, M32 = ctaug.affine_matrix(prm, dims, dims)
    g = rng.standard_normal(dims).astype(np.float32)

    img = _t(img_np).requires_grad_(True)
    M = torch.tensor(M32.astype(np.float64), requires_grad=True)      # host, FP64
    out = ag.warp_affine(img, M, fill=-1000.0)
    (out * _t(g)).sum().backward()
    r_img, r_M, _ = oracle.warp_backward(img_np, M32, g)
    assert_grad(_np(img.grad), r_img, "autograd g_img")
    assert M.grad.dtype == torch.float64 and M.grad.device.type == "cpu"
    assert_grad(M.grad.numpy(), r_M, "autograd g_M")

    ctrl = rng.normal(0.0, 2.0, (3, 6, 6, 6)).astype(np.float32)
    u_ref = oracle.bspline_upsample_f32(ctrl, dims)        # the oracle's parity-mode field
    c = _t(ctrl).requires_grad_(True)
    u = ag.bspline_upsample(c, dims)
    out2 = ag.warp_displacement(_t(img_np), torch.tensor(M32.astype(np.float64)), u)
    (out2 * _t(g)).sum().backward()
    _, _, r_u = oracle.warp_backward(img_np, M32, g, disp=u_ref, want_img=False, want_M=False,
                                     want_u=True)
    assert_grad(_np(c.grad), oracle.bspline_adjoint(r_u, (6, 6, 6)), "autograd g_ctrl")


@pytest.mark.parametrize("dims,sigma,dtype", [((30, 26, 41), (1.4, 0.0, 2.3), np.float32),
                                              ((17, 33, 20), (0.9, 1.9, 0.6), np.int16),
                                              ((9, 11, 64), (0.0, 0.0, 4.7), np.float32),
                                              ((12, 10, 14), (0.0, 0.0, 0.0), np.int16)])
def test_gaussian_smooth_parity(dims, sigma, dtype):
    rng = np.random.default_rng(int(sum(dims)))
    v = np.round(rng.normal(0, 400, dims)).astype(dtype)
    out = _np(ctaug.gaussian_smooth(_t(v), sigma))
    ref = oracle.gaussian_smooth(v, sigma)
    assert_intensity(out, ref, windowed=False, what=f"smooth {sigma}")


def test_resampling_pipeline_parity():
    """Resample to a coarser target spacing: smooth with the section's widths,
    then trilinear warp with A = diag(target / spacing) about the centres."""
    spacing, target = (0.8, 0.75, 2.0), 3.0
    in_dim = (60, 64, 24)
    img, lbl = phantom_pair(in_dim, seed=41)
    scale = [target / s_ for s_ in spacing]
    out_dim = tuple(int(np.floor(n * s_ / target)) for n, s_ in zip(in_dim, spacing))
    prm = identity_affine_params()
    prm[3:6] = scale
    sig = ctaug.resample_sigma(spacing, target)
    np.testing.assert_allclose(sig, oracle.resample_sigma(spacing, target), rtol=1e-7)
    sm = ctaug.gaussian_smooth(_t(img), sig)
    _, M = ctaug.affine_matrix(prm, in_dim, out_dim)
    out, lout = ctaug.warp_affine(sm, M, lbl=_t(lbl), out_dim=out_dim)
    ref_sm = oracle.gaussian_smooth(img, np.asarray(sig, dtype=np.float64))
    ref, lref = oracle.warp(ref_sm, M, out_dim, lbl=lbl)
    assert_intensity(_np(sm), ref_sm, windowed=False, what="smoothed")
    assert_intensity(_np(out), ref, windowed=False, what="resampled")
    assert np.array_equal(_np(lout), lref)


# ---------------------------------------------------------------------------
# Host-to-device FIFO
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("depth", [2, 3])
def test_pipeline_matches_direct_warps(depth):
    """Volumes streamed from pinned host slots through the FIFO give the same
    bits as ctaug_warp_affine on device copies, with slots reused several times."""
    rng = np.random.default_rng(90 + depth)
    shapes = [(40, 36, 28), (33, 30, 17), (48, 20, 44), (25, 25, 25), (40, 36, 28), (12, 50, 31),
              (37, 29, 40)]
    out_dim = (32, 28, 24)
    cases = []
    for i, shp in enumerate(shapes):
        img, lbl = phantom_pair(shp, seed=300 + i)
        if i % 2:
            img = img.astype(np.float32)
        prm = draw_affine_params(rng, AugmentRanges(), shp, out_dim)
        _, M = ctaug.affine_matrix(prm, shp, out_dim)
        ph = draw_photo(rng, AugmentRanges(), seed=7, volume_id=i) if i % 3 else None
        cases.append((img, lbl if i != 4 else None, M, ph))
    slot = max(ctaug.Pipeline.slot_bytes_for(c[0].shape, c[0].dtype) for c in cases)
    outs = [torch.empty(out_dim, dtype=torch.float32, device=DEV) for _ in cases]
    louts = [torch.empty(out_dim, dtype=torch.int8, device=DEV) for _ in cases]
    with ctaug.Pipeline(depth, slot) as pipe:
        for (img, lbl, M, ph), o, lo in zip(cases, outs, louts):
            pipe.put(img, M, lbl=lbl, photo=ph, out=o, lbl_out=lo if lbl is not None else None)
        pipe.sync()
    for (img, lbl, M, ph), o, lo in zip(cases, outs, louts):
        ref, lref = ctaug.warp_affine(_t(img), M, lbl=_t(lbl) if lbl is not None else None,
                                      photo=ph, out_dim=out_dim)
        assert np.array_equal(_np(o).view(np.uint32), _np(ref).view(np.uint32))
        if lbl is not None:
            assert np.array_equal(_np(lo), _np(lref))


def test_pipeline_rejects_inputs_outside_the_slot():
    L = ctaug._lib.load()
    with ctaug.Pipeline(2, 1 << 16) as pipe:
        img = np.zeros((8, 8, 8), np.int16)
        out = torch.empty((8, 8, 8), dtype=torch.float32, device=DEV)
        vo = ctaug.ops.vol(out)
        M_np = np.eye(3, 4).ravel()
        M = ctaug.ops._M32(M_np)
        vi = ctaug.ops._host_vol(img.ctypes.data, img)       # not a slot address
        assert L.ctaug_pipeline_submit(pipe._h, ctypes.byref(vi), None, M, 0.0, 0, None,
                                       ctypes.byref(vo), None) == 1   # nothing acquired
        addr = pipe.acquire()
        assert L.ctaug_pipeline_submit(pipe._h, ctypes.byref(vi), None, M, 0.0, 0, None,
                                       ctypes.byref(vo), None) == 1   # outside the slot
        big = np.zeros((64, 32, 17), np.int16)                       # 69632 bytes > slot
        vb = ctaug.ops._host_vol(addr, big)
        assert L.ctaug_pipeline_submit(pipe._h, ctypes.byref(vb), None, M, 0.0, 0, None,
                                       ctypes.byref(vo), None) == 1
        ctypes.memmove(addr, img.ctypes.data, img.nbytes)          # the slot stays acquired
        pipe.submit(addr, img, M_np, out=out)
        pipe.sync()
        assert not _np(out).any()


# ---------------------------------------------------------------------------
# Batched persistent launch and HIP graph replay
# ---------------------------------------------------------------------------

def _batch_jobs(n=4, out_dim=(40, 40, 48), size_range=(30, 64)):
    jobs = configs.c3(n=n, size_range=size_range, out_dim=out_dim)
    tensors = []
    for j in jobs:
        _, M = ctaug.affine_matrix(j.prm, j.in_dim, j.out_dim)
        img, lbl = _t(j.img), _t(j.lbl)
        out = torch.empty(out_dim, dtype=torch.float32, device=DEV)
        lout = torch.empty(out_dim, dtype=torch.int8, device=DEV)
        tensors.append((j, M, img, lbl, out, lout))
    return tensors


def test_batch_plan_matches_single_calls_and_oracle():
    T = _batch_jobs()
    jobs = [ctaug.make_job(img, M, out, lbl, lout, fill=j.fill, photo=j.photo)
            for (j, M, img, lbl, out, lout) in T]
    plan = ctaug.BatchPlan(jobs)
    plan.launch()
    for (j, M, img, lbl, out, lout) in T:
        s_out, s_lout = ctaug.warp_affine(img, M, lbl=lbl, fill=j.fill, photo=j.photo,
                                          out_dim=j.out_dim)
        assert torch.equal(out, s_out) and torch.equal(lout, s_lout)
        ref, lref = oracle.warp(j.img, M, j.out_dim, lbl=j.lbl, fill=j.fill, photo=j.photo)
        assert np.array_equal(_np(lout), lref)
        assert_intensity(_np(out), ref, windowed=True)
    plan.close()


def test_batch_plan_bspline_jobs_match_single_calls():
    """B-spline jobs in the batched persistent launch (displacement tiles)
    give the bits of warp_bspline on each volume, across an update and graph
    replays; the plan reports the displacement tile shape."""
    rng = np.random.default_rng(101)
    shapes = [(40, 36, 28), (33, 30, 17), (48, 20, 44), (25, 25, 25)]
    out_dim = (36, 28, 20)
    grids = [(8, 8, 8), (6, 7, 5), (5, 6, 9), (4, 4, 4)]
    items = []
    for i, (shp, grid) in enumerate(zip(shapes, grids)):
        img, lbl = phantom_pair(shp, seed=400 + i)
        prm = draw_affine_params(rng, AugmentRanges(), shp, out_dim)
        _, M = ctaug.affine_matrix(prm, shp, out_dim)
        C = (3.0 * rng.standard_normal((3,) + grid)).astype(np.float32)
        ph = draw_photo(rng, AugmentRanges(), seed=11, volume_id=i)
        items.append([_t(img), _t(lbl), M, _t(C), ph,
                      torch.empty(out_dim, dtype=torch.float32, device=DEV),
                      torch.empty(out_dim, dtype=torch.int8, device=DEV)])

    def jobs():
        return [ctaug.make_job(im, M, o, lb, lo, photo=ph, ctrl=C)
                for im, lb, M, C, ph, o, lo in items]

    def check():
        for im, lb, M, C, ph, o, lo in items:
            ref, lref = ctaug.warp_bspline(im, M, C, lbl=lb, photo=ph, out_dim=out_dim)
            assert np.array_equal(_np(o).view(np.uint32), _np(ref).view(np.uint32))
            assert np.array_equal(_np(lo), _np(lref))

    plan = ctaug.BatchPlan(jobs(), tile=(16, 16, 16))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.launch()
    torch.cuda.synchronize()
    check()
    assert tuple(plan.tuning()[0]) == (8, 8, 16)
    for it in items:                       # new control grids, then graph replays
        it[3] = _t((2.0 * rng.standard_normal(tuple(it[3].shape))).astype(np.float32))
    with torch.cuda.stream(stream):
        plan.capture()
        plan.update(jobs())
        plan.replay()
        plan.replay()
    torch.cuda.synchronize()
    check()
    plan.close()


@pytest.mark.parametrize("tile,wg,lds,fmt", [((4, 8, 32), 0, 0, 0), ((8, 8, 16), 2, 0, 1),
                                             ((2, 4, 64), 1, 2048, 0), ((16, 16, 16), 4, 0, 1),
                                             ((8, 16, 16), 0, -1, 0), ((8, 8, 8), 0, 300, 1),
                                             ((16, 16, 16), 0, 6000, 0), ((16, 16, 16), 2, 8000, 1),
                                             ((32, 16, 16), 0, 3000, 0)])
def test_batch_launch_shapes_bit_identical(tile, wg, lds, fmt):
    """Every launch shape gives the single-call result bit for bit, including
    reservations too small for a whole tile's footprint (tiles staged in
    sub-tiles, or gathered directly)."""
    T = _batch_jobs(n=3, out_dim=(36, 30, 44))
    jobs = [ctaug.make_job(img, M, out, lbl, lout, fill=j.fill, photo=j.photo)
            for (j, M, img, lbl, out, lout) in T]
    plan = ctaug.BatchPlan(jobs, tile=tile, wg_per_cu=wg, lds_cells=lds, lds_format=fmt)
    plan.launch()
    for (j, M, img, lbl, out, lout) in T:
        s_out, s_lout = ctaug.warp_affine(img, M, lbl=lbl, fill=j.fill, photo=j.photo,
                                          out_dim=j.out_dim)
        assert torch.equal(out, s_out) and torch.equal(lout, s_lout)
    plan.close()


@pytest.mark.parametrize("tiles", [(1,), (31, 32), (33, 32), (255, 256), (257, 256),
                                   (64, 64, 64, 64, 64, 64, 64, 65)])
@pytest.mark.parametrize("wg", [0, 1])
def test_batch_tile_counts_around_xcd_chunks(tiles, wg):
    """Batches whose tile totals fall just below and above the XCD chunk (64
    tiles) and a whole round of chunks (512 tiles), one workgroup per tile
    and persistent: every tile is warped exactly once, bit for bit as single
    calls."""
    rng = np.random.default_rng(sum(tiles) + wg)
    items = []
    for k, n in enumerate(tiles):
        out_dim = (4, 4, 4 * n)                # n tiles of 4 x 4 x 4
        in_dim = (9, 7, 4 * n + 3)
        img, lbl = phantom_pair(in_dim, seed=600 + k)
        prm = draw_affine_params(rng, AugmentRanges(), in_dim, out_dim)
        _, M = ctaug.affine_matrix(prm, in_dim, out_dim)
        ph = draw_photo(rng, AugmentRanges(), seed=12, volume_id=k)
        items.append((_t(img), _t(lbl), M, ph, out_dim,
                      torch.full(out_dim, float("nan"), dtype=torch.float32, device=DEV),
                      torch.full(out_dim, 77, dtype=torch.int8, device=DEV)))
    jobs = [ctaug.make_job(im, M, o, lb, lo, photo=ph) for im, lb, M, ph, od, o, lo in items]
    plan = ctaug.BatchPlan(jobs, tile=(4, 4, 4), wg_per_cu=wg)
    plan.launch()
    for im, lb, M, ph, od, o, lo in items:
        ref, lref = ctaug.warp_affine(im, M, lbl=lb, photo=ph, out_dim=od)
        assert np.array_equal(_np(o).view(np.uint32), _np(ref).view(np.uint32))
        assert torch.equal(lo, lref)
    plan.close()


def test_batch_graph_replay_with_updates():
    T = _batch_jobs(n=3)
    jobs = [ctaug.make_job(img, M, out, lbl, lout, fill=j.fill, photo=j.photo)
            for (j, M, img, lbl, out, lout) in T]
    plan = ctaug.BatchPlan(jobs)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.capture()
    rng = np.random.default_rng(12)
    for rep in range(4):
        # new transforms and photometrics each replay, no re-capture
        newT, new_jobs = [], []
        for (j, M, img, lbl, out, lout) in T:
            prm = draw_affine_params(rng, AugmentRanges(), j.in_dim, j.out_dim)
            _, M2 = ctaug.affine_matrix(prm, j.in_dim, j.out_dim)
            ph = draw_photo(rng, AugmentRanges(), seed=1000 + rep, volume_id=j.volume_id)
            newT.append((j, M2, ph, img, lbl, out, lout))
            new_jobs.append(ctaug.make_job(img, M2, out, lbl, lout, fill=j.fill, photo=ph))
        plan.update(new_jobs)
        with torch.cuda.stream(stream):
            plan.replay()
        stream.synchronize()
        for (j, M2, ph, img, lbl, out, lout) in newT:
            s_out, s_lout = ctaug.warp_affine(img, M2, lbl=lbl, fill=j.fill, photo=ph,
                                              out_dim=j.out_dim)
            assert torch.equal(out, s_out) and torch.equal(lout, s_lout), f"replay {rep}"
    plan.close()


def test_autotune_picks_a_candidate_and_results_hold():
    T = _batch_jobs(n=2)
    jobs = [ctaug.make_job(img, M, out, lbl, lout, fill=j.fill, photo=j.photo)
            for (j, M, img, lbl, out, lout) in T]
    plan = ctaug.BatchPlan(jobs)
    cands = [((4, 8, 32), 0, 0, 0), ((8, 8, 16), 0, 4096, 1), ((4, 8, 32), 4, -1, 0)]
    best, times = plan.autotune(cands, reps=2)
    assert best[:2] in [c[:2] for c in cands] and all(t > 0 for t in times)
    assert plan.tuning() == best
    plan.launch()
    for (j, M, img, lbl, out, lout) in T:
        s_out, _ = ctaug.warp_affine(img, M, lbl=lbl, fill=j.fill, photo=j.photo,
                                     out_dim=j.out_dim)
        assert torch.equal(out, s_out)
    plan.close()
    ctaug.autotune_cache_clear()


def test_autotune_then_run_uses_the_winning_tables():
    """After autotuning, run() (no upload) decodes tiles with the winner's
    prefix table and job table, also when the winner was not the last
    candidate timed (here the last one gathers 4^3 tiles directly, far
    slower than the first)."""
    T = _batch_jobs(n=3)
    jobs = [ctaug.make_job(img, M, out, lbl, lout, fill=j.fill, photo=j.photo)
            for (j, M, img, lbl, out, lout) in T]
    plan = ctaug.BatchPlan(jobs)
    cands = [((16, 16, 16), 0, 0, 0), ((4, 4, 4), 0, -1, 0)]
    best, times = plan.autotune(cands, reps=3)
    assert plan.tuning() == best
    for (j, M, img, lbl, out, lout) in T:
        out.zero_()
        lout.zero_()
    plan.run()
    for (j, M, img, lbl, out, lout) in T:
        s_out, s_lout = ctaug.warp_affine(img, M, lbl=lbl, fill=j.fill, photo=j.photo,
                                          out_dim=j.out_dim)
        assert torch.equal(out, s_out) and torch.equal(lout, s_lout)
    plan.close()
    ctaug.autotune_cache_clear()


# ---------------------------------------------------------------------------
# Strided inputs (crop views) and the 24-bit offset limits
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [np.int16, np.float32])
def test_strided_crop_views_match_dense_copies(dtype):
    """A crop passed as a view of the whole scan gives the bits of the same
    crop copied densely: single calls, batch jobs and the adjoint."""
    parent, plbl = phantom_pair((60, 52, 48), seed=33)
    parent = parent.astype(dtype)
    sl = (slice(5, 45), slice(3, 43), slice(7, 39))
    crop, clbl = np.ascontiguousarray(parent[sl]), np.ascontiguousarray(plbl[sl])
    tp, tl = _t(parent), _t(plbl)
    view, lview = tp[sl], tl[sl]
    assert not view.is_contiguous()
    rng = np.random.default_rng(34)
    out_dim = (36, 32, 28)
    prm = draw_affine_params(rng, AugmentRanges(), crop.shape, out_dim)
    _, M = ctaug.affine_matrix(prm, crop.shape, out_dim)
    ph = draw_photo(rng, AugmentRanges(), seed=3, volume_id=1)
    o1, l1 = ctaug.warp_affine(view, M, lbl=lview, photo=ph, out_dim=out_dim)
    o2, l2 = ctaug.warp_affine(_t(crop), M, lbl=_t(clbl), photo=ph, out_dim=out_dim)
    assert torch.equal(o1, o2) and torch.equal(l1, l2)
    ref, lref = oracle.warp(crop, M, out_dim, lbl=clbl, photo=ph)
    assert np.array_equal(_np(l1), lref)
    assert_intensity(_np(o1), ref, windowed=True, what="strided crop")
    # batch job with strided inputs
    o3 = torch.empty(out_dim, dtype=torch.float32, device=DEV)
    l3 = torch.empty(out_dim, dtype=torch.int8, device=DEV)
    plan = ctaug.BatchPlan([ctaug.make_job(view, M, o3, lview, l3, photo=ph)])
    plan.launch()
    assert torch.equal(o3, o1) and torch.equal(l3, l1)
    plan.close()
    # the adjoint reads the view
    g = _t(rng.standard_normal(out_dim).astype(np.float32))
    gi1, gM1 = ctaug.warp_affine_backward(view, M, g)
    gi2, gM2 = ctaug.warp_affine_backward(_t(crop), M, g)
    assert torch.equal(gM1, gM2)
    r_img, r_M, _ = oracle.warp_backward(crop, M, _np(g))
    assert_grad(_np(gi1), r_img, "strided g_img")
    assert_grad(_np(gM1), r_M, "strided g_M")


def test_gather_offsets_at_the_24_bit_limits():
    """Inputs at the largest row count (X*Y = 2^24) and row pitch (2^24 - 1)
    the 24-bit offset arithmetic admits, sampled up to their last voxel."""
    # 2048 x 8192 x 2: X*Y = 2^24 rows
    dims = (2048, 8192, 2)
    rng = np.random.default_rng(35)
    img = rng.integers(-1000, 1500, size=dims, dtype=np.int16)
    lbl = rng.integers(0, 6, size=dims, dtype=np.int8)
    out_dim = (24, 24, 8)
    M = np.array([2047.0 / 23, 0.0, 0.0, 0.0,
                  0.0, 8191.0 / 23, 0.01, 0.0,
                  0.0, 0.0, 1.0 / 7, 0.0], np.float32)
    out, lout = ctaug.warp_affine(_t(img), M, lbl=_t(lbl), out_dim=out_dim)
    ref, lref = oracle.warp(img, M, out_dim, lbl=lbl)
    assert np.array_equal(_np(lout), lref)
    assert_intensity(_np(out), ref, windowed=False, what="X*Y = 2^24")
    # 1 x 1 x (2^24 - 1): the largest row pitch
    n = (1 << 24) - 1
    img2 = rng.integers(-1000, 1500, size=(1, 1, n), dtype=np.int16)
    M2 = np.array([0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1.0, n - 1 - 63], np.float32)
    out2, _ = ctaug.warp_affine(_t(img2), M2, out_dim=(1, 1, 64))
    got = _np(out2)[0, 0]
    assert np.array_equal(got, img2[0, 0, n - 64:].astype(np.float32))


@pytest.mark.parametrize("scale", [1.0, 3.5])
def test_affine_backward_nonfinite_gradients(scale):
    """NaN and infinite upstream gradients propagate to exactly the image
    cells the oracle's FP64 adjoint gives them (every in-volume corner of the
    voxel's cell), on the fixed-point LDS path and on the direct path (large
    footprints); other cells keep the gradient bar."""
    dims = (40, 36, 32)
    img, _ = phantom_pair(dims, seed=21)
    img = img.astype(np.float32)
    rng = np.random.default_rng(22)
    ranges = AugmentRanges(scale=(scale, scale), disp=(0.0, 0.0, 0.0))
    prm = draw_affine_params(rng, ranges, dims, dims)
    _, M = ctaug.affine_matrix(prm, dims, dims)
    g = rng.standard_normal(dims).astype(np.float32)
    flat = g.reshape(-1)
    centre = ((np.indices(dims) - (np.array(dims)[:, None, None, None] - 1) / 2) ** 2).sum(0)
    inner = np.flatnonzero(centre.reshape(-1) < 5.0 ** 2)   # q stays inside
    pick = rng.choice(inner, size=6, replace=False)
    flat[pick[:4]] = np.nan
    flat[pick[4:]] = np.inf
    g_img, g_M = ctaug.warp_affine_backward(_t(img), M, _t(g))
    r_img, r_M, _ = oracle.warp_backward(img, M, g)
    gi = _np(g_img)
    assert np.isnan(r_img).any() and np.array_equal(np.isnan(gi), np.isnan(r_img))
    assert np.array_equal(np.isinf(gi), np.isinf(r_img))
    fin = np.isfinite(r_img)
    assert_grad(gi[fin], r_img[fin], "finite cells")
    assert np.isnan(_np(g_M)).all() and np.isnan(r_M).all()


def test_autotune_cache_feeds_plans_created_without_tuning(tmp_path):
    """The autotuner's choice is cached per device and batch class: a plan
    created later without a tuning takes it, also after a save / clear / load
    round trip; results stay bitwise those of single calls."""
    ctaug.autotune_cache_clear()
    T = _batch_jobs(n=3)
    jobs = [ctaug.make_job(img, M, out, lbl, lout, fill=j.fill, photo=j.photo)
            for (j, M, img, lbl, out, lout) in T]
    assert ctaug.autotune_cache_lookup(jobs) is None
    plan = ctaug.BatchPlan(jobs)
    assert plan.tuning()[0] == (8, 16, 16)                 # the default shape
    cands = [((4, 8, 32), 0, 0, 0), ((16, 16, 16), 0, 6128, 1)]
    best, _ = plan.autotune(cands, reps=2)
    plan.close()
    assert ctaug.autotune_cache_lookup(jobs) == best
    path = tmp_path / "tune.txt"
    ctaug.autotune_cache_save(path)
    ctaug.autotune_cache_clear()
    assert ctaug.autotune_cache_lookup(jobs) is None
    assert ctaug.autotune_cache_load(path) == 1
    plan2 = ctaug.BatchPlan(jobs)
    assert plan2.tuning()[0] == best[0] and plan2.tuning()[3] == best[3]
    plan2.launch()
    for (j, M, img, lbl, out, lout) in T:
        s_out, s_lout = ctaug.warp_affine(img, M, lbl=lbl, fill=j.fill, photo=j.photo,
                                          out_dim=j.out_dim)
        assert torch.equal(out, s_out) and torch.equal(lout, s_lout)
    plan2.close()
    ctaug.autotune_cache_clear()


def test_prepared_updates_equal_updates_and_go_stale_on_retuning():
    """Prepared descriptor sets installed by update_prepared give the outputs
    of plain updates (graph replays); a set prepared before autotuning is
    refused afterwards, and one prepared for another plan is refused."""
    T = _batch_jobs(n=3)
    rng = np.random.default_rng(41)
    draws = []
    for rep in range(3):
        jobs, items = [], []
        for (j, M, img, lbl, out, lout) in T:
            prm = draw_affine_params(rng, AugmentRanges(), j.in_dim, j.out_dim)
            _, M2 = ctaug.affine_matrix(prm, j.in_dim, j.out_dim)
            ph = draw_photo(rng, AugmentRanges(), seed=2000 + rep, volume_id=j.volume_id)
            jobs.append(ctaug.make_job(img, M2, out, lbl, lout, fill=j.fill, photo=ph))
            items.append((j, M2, ph, img, lbl, out, lout))
        draws.append((jobs, items))
    plan = ctaug.BatchPlan(draws[0][0])
    prepared = [plan.prepare(jobs) for jobs, _ in draws]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.capture()
    for rep in (2, 0, 1):
        plan.update_prepared(prepared[rep])
        with torch.cuda.stream(stream):
            plan.replay()
        stream.synchronize()
        for (j, M2, ph, img, lbl, out, lout) in draws[rep][1]:
            s_out, s_lout = ctaug.warp_affine(img, M2, lbl=lbl, fill=j.fill, photo=ph,
                                              out_dim=j.out_dim)
            assert torch.equal(out, s_out) and torch.equal(lout, s_lout), f"draw {rep}"
    other = ctaug.BatchPlan(draws[0][0])
    with pytest.raises(ctaug._lib.CtaugError):
        other.update_prepared(prepared[0])
    other.close()
    plan.autotune([((16, 16, 16), 0, 0, 0)], reps=1)
    with pytest.raises(ctaug._lib.CtaugError):
        plan.update_prepared(prepared[1])
    for p in prepared:
        p.close()
    plan.close()
    ctaug.autotune_cache_clear()


@pytest.mark.parametrize("tiles", [(1,), (63,), (31, 33), (256, 257), (600, 600)])
def test_batched_backward_tile_counts_around_xcd_chunks(tiles):
    """The batched adjoint over tile totals around the XCD chunk (64 tiles),
    a round of chunks (512) and more tiles than resident workgroups (1200):
    grad_img and grad_M of every job against single calls and the oracle.  The
    input tensors are made inline: the job keeps them alive."""
    rng = np.random.default_rng(sum(tiles))
    items = []
    for k, n in enumerate(tiles):
        out_dim = (8, 8, 16 * n)               # n adjoint tiles of 8 x 8 x 16
        in_dim = (12, 11, 16 * n + 5)
        img, _ = phantom_pair(in_dim, seed=700 + k)
        img = img.astype(np.float32)
        prm = draw_affine_params(rng, AugmentRanges(), in_dim, out_dim)
        _, M = ctaug.affine_matrix(prm, in_dim, out_dim)
        g = rng.standard_normal(out_dim).astype(np.float32)
        items.append((img, M, g))
    gis = [torch.zeros(it[0].shape, dtype=torch.float32, device=DEV) for it in items]
    gMs = [torch.empty(12, dtype=torch.float64, device=DEV) for _ in items]
    jobs = [ctaug.ops.make_bwd_job(_t(img), M, _t(g), grad_img=gi, grad_M=gM)
            for (img, M, g), gi, gM in zip(items, gis, gMs)]
    ctaug.ops.warp_affine_backward_batch(jobs)
    for k, (img, M, g) in enumerate(items):
        s_img, s_M = ctaug.warp_affine_backward(_t(img), M, _t(g))
        assert_grad(_np(gis[k]), _np(s_img).astype(np.float64), f"job {k} g_img vs single")
        np.testing.assert_allclose(_np(gMs[k]), _np(s_M), rtol=1e-12,
                                   atol=1e-12 * np.abs(_np(s_M)).max())
        r_img, r_M, _ = oracle.warp_backward(img, M, g)
        assert_grad(_np(gis[k]), r_img, f"job {k} g_img vs oracle")
        assert_grad(_np(gMs[k]), r_M, f"job {k} g_M vs oracle")


@pytest.mark.parametrize("scale", [0.5, 0.3])
def test_affine_backward_same_sign_gradients_fill_the_fixed_point_range(scale):
    """A constant upstream gradient (every contribution of a cell the same
    sign) under upsampling, where the most samples share an input cell: at
    scale 0.5 the bound admits the 32-bit tile sums at their largest count
    (2^7), at 0.3 it does not (64-bit sums).  No rotation, so the samples
    fall on the bound's lattice; single call and batch against the oracle."""
    in_dim, out_dim = (30, 26, 22), (56, 48, 40)
    img, _ = phantom_pair(in_dim, seed=61)
    img = img.astype(np.float32)
    prm = identity_affine_params()
    prm[3:6] = scale
    prm[21:24] = [0.25, -0.5, 0.125]
    _, M = ctaug.affine_matrix(prm, in_dim, out_dim)
    assert abs(M[0] - scale) < 1e-6 and M[1] == 0 and M[2] == 0
    g = np.full(out_dim, 0.99, np.float32)
    r_img, r_M, _ = oracle.warp_backward(img, M, g)
    g_img, g_M = ctaug.warp_affine_backward(_t(img), M, _t(g))
    assert_grad(_np(g_img), r_img, "g_img")
    assert_grad(_np(g_M), r_M, "g_M")
    gi = torch.zeros(in_dim, dtype=torch.float32, device=DEV)
    gM = torch.empty(12, dtype=torch.float64, device=DEV)
    ctaug.ops.warp_affine_backward_batch([ctaug.ops.make_bwd_job(_t(img), M, _t(g), grad_img=gi,
                                                                 grad_M=gM)])
    assert_grad(_np(gi), r_img, "batched g_img")
    assert_grad(_np(gM), r_M, "batched g_M")


def test_batched_backward_mixes_32_and_64_bit_jobs():
    """A batch of jobs whose sample bound admits 32-bit tile sums and one
    strongly upsampling job that does not (the whole launch takes 64-bit
    sums): every job against the oracle and the single call."""
    rng = np.random.default_rng(77)
    items = []
    for k, sc in enumerate([(0.9, 1.1), (0.28, 0.3), (0.8, 1.2)]):
        in_dim = (26, 24, 30)
        out_dim = (40, 36, 48) if sc[0] < 0.5 else (24, 26, 28)
        img, _ = phantom_pair(in_dim, seed=90 + k)
        img = img.astype(np.float32)
        prm = draw_affine_params(rng, AugmentRanges(scale=sc), in_dim, out_dim)
        _, M = ctaug.affine_matrix(prm, in_dim, out_dim)
        g = rng.standard_normal(out_dim).astype(np.float32)
        items.append((img, M, g))
    gis = [torch.zeros(it[0].shape, dtype=torch.float32, device=DEV) for it in items]
    gMs = [torch.empty(12, dtype=torch.float64, device=DEV) for _ in items]
    ctaug.ops.warp_affine_backward_batch([
        ctaug.ops.make_bwd_job(_t(img), M, _t(g), grad_img=gi, grad_M=gM)
        for (img, M, g), gi, gM in zip(items, gis, gMs)])
    for k, (img, M, g) in enumerate(items):
        r_img, r_M, _ = oracle.warp_backward(img, M, g)
        assert_grad(_np(gis[k]), r_img, f"job {k} g_img vs oracle")
        assert_grad(_np(gMs[k]), r_M, f"job {k} g_M vs oracle")
        s_img, s_M = ctaug.warp_affine_backward(_t(img), M, _t(g))
        assert_grad(_np(gis[k]), _np(s_img).astype(np.float64), f"job {k} g_img vs single")


def test_batched_backward_image_only_without_workspace():
    """No job wants grad_M, so the C call takes no workspace (NULL): grad_img
    of every job (ten, two launches) against the oracle."""
    rng = np.random.default_rng(606)
    items, jobs, gis = [], [], []
    for k in range(10):
        in_dim = tuple(int(v) for v in rng.integers(12, 30, 3))
        out_dim = tuple(int(v) for v in rng.integers(10, 34, 3))
        img, _ = phantom_pair(in_dim, seed=620 + k)
        img = img.astype(np.float32)
        prm = draw_affine_params(rng, AugmentRanges(), in_dim, out_dim)
        _, M = ctaug.affine_matrix(prm, in_dim, out_dim)
        g = rng.standard_normal(out_dim).astype(np.float32)
        gi = torch.zeros(in_dim, dtype=torch.float32, device=DEV)
        items.append((img, M, g))
        gis.append(gi)
        jobs.append(ctaug.ops.make_bwd_job(_t(img), M, _t(g), grad_img=gi, grad_M=None))
    arr = (ctaug._lib.BwdJob * len(jobs))(*jobs)
    L = ctaug._lib.load()
    assert L.ctaug_warp_affine_backward_batch(arr, len(jobs), None, 0, ctaug.ops._stream()) == 0
    torch.cuda.synchronize()
    for k, (img, M, g) in enumerate(items):
        r_img, _, _ = oracle.warp_backward(img, M, g)
        assert_grad(_np(gis[k]), r_img, f"job {k} g_img")


def test_batched_backward_writes_every_partial_row():
    """Jobs with no tiles (an empty output) before, between and after jobs
    with tiles, then a batch of empty jobs only, each over a workspace
    filled with NaN bytes first: every grad_M against the oracle (zeros for
    the empty jobs), as every workgroup writes its row of every job."""
    rng = np.random.default_rng(404)
    need = ctaug.ops.warp_affine_backward_batch_workspace(5)
    ws = torch.full((need,), 255, dtype=torch.uint8, device=DEV)
    specs = [((20, 22, 24), (0, 20, 22)), ((20, 22, 24), (18, 20, 22)),
             ((18, 16, 20), (9, 0, 5)), ((16, 18, 20), (17, 15, 33)),
             ((12, 14, 16), (6, 7, 0))]
    items = []
    for k, (in_dim, out_dim) in enumerate(specs):
        img, _ = phantom_pair(in_dim, seed=500 + k)
        img = img.astype(np.float32)
        prm = draw_affine_params(rng, AugmentRanges(), in_dim, out_dim)
        _, M = ctaug.affine_matrix(prm, in_dim, out_dim)
        g = rng.standard_normal(out_dim).astype(np.float32)
        items.append((img, M, g))
    for batch in ([0, 1, 2, 3, 4], [0, 2, 4]):
        ws.fill_(255)
        gis = {k: torch.zeros(items[k][0].shape, dtype=torch.float32, device=DEV) for k in batch}
        gMs = {k: torch.full((12,), np.nan, dtype=torch.float64, device=DEV) for k in batch}
        ctaug.ops.warp_affine_backward_batch(
            [ctaug.ops.make_bwd_job(_t(items[k][0]), items[k][1], _t(items[k][2]),
                                    grad_img=gis[k], grad_M=gMs[k]) for k in batch], ws)
        for k in batch:
            img, M, g = items[k]
            r_img, r_M, _ = oracle.warp_backward(img, M, g)
            if g.size == 0:
                assert np.array_equal(_np(gMs[k]), np.zeros(12)), (batch, k)
                assert not _np(gis[k]).any(), (batch, k)
            else:
                assert_grad(_np(gMs[k]), r_M, f"{batch} job {k} g_M")
                assert_grad(_np(gis[k]), r_img, f"{batch} job {k} g_img")


@pytest.mark.parametrize("dtype,n", [(np.float32, 10), (np.int16, 3)])
def test_batched_backward_matches_single_calls_and_oracle(dtype, n):
    """One batched adjoint launch (two for ten jobs) over volumes of uneven
    sizes, photometrics on some, a strided input on one: grad_img and grad_M
    of every job against the single-call adjoint and the oracle; a second
    batched call gives grad_M bit for bit."""
    rng = np.random.default_rng(51 + n)
    items = []
    for k in range(n):
        dims = tuple(int(v) for v in rng.integers(20, 48, 3))
        out_dim = tuple(int(v) for v in rng.integers(16, 44, 3))
        img, _ = phantom_pair(dims, seed=300 + k)
        img = img.astype(dtype)
        prm = draw_affine_params(rng, AugmentRanges(), dims, out_dim)
        _, M = ctaug.affine_matrix(prm, dims, out_dim)
        ph = None
        if k % 3 == 1:
            ph = draw_photo(rng, AugmentRanges(window=False), seed=k, volume_id=k)
            ph.occlude, ph.occ_lo, ph.occ_hi = True, 3.0, 7.5
        g = rng.standard_normal(out_dim).astype(np.float32)
        if k == 2:                    # a crop view of a larger parent
            parent = np.zeros((dims[0] + 4, dims[1] + 3, dims[2] + 5), dtype)
            parent[2:2 + dims[0], 1:1 + dims[1], 3:3 + dims[2]] = img
            ti = _t(parent)[2:2 + dims[0], 1:1 + dims[1], 3:3 + dims[2]]
        else:
            ti = _t(img)
        items.append((img, ti, M, ph, g, _t(g)))
    gis = [torch.zeros(it[0].shape, dtype=torch.float32, device=DEV) for it in items]
    gMs = [torch.empty(12, dtype=torch.float64, device=DEV) for _ in items]
    jobs = [ctaug.ops.make_bwd_job(ti, M, tg, grad_img=gi, grad_M=gM, photo=ph)
            for (img, ti, M, ph, g, tg), gi, gM in zip(items, gis, gMs)]
    ctaug.ops.warp_affine_backward_batch(jobs)
    first = [_np(gM).copy() for gM in gMs]
    for k, (img, ti, M, ph, g, tg) in enumerate(items):
        s_img, s_M = ctaug.warp_affine_backward(ti, M, tg, photo=ph)
        assert_grad(_np(gis[k]), _np(s_img).astype(np.float64), f"job {k} g_img vs single")
        np.testing.assert_allclose(first[k], _np(s_M), rtol=1e-12,
                                   atol=1e-12 * np.abs(_np(s_M)).max())
        r_img, r_M, _ = oracle.warp_backward(img, M, g, photo=ph)
        assert_grad(_np(gis[k]), r_img, f"job {k} g_img vs oracle")
        assert_grad(first[k], r_M, f"job {k} g_M vs oracle")
    ctaug.ops.warp_affine_backward_batch(jobs)
    for k, gM in enumerate(gMs):
        assert np.array_equal(_np(gM).view(np.uint64), first[k].view(np.uint64)), k
