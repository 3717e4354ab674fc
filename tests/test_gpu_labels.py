"""GPU parity of the labels-only nearest-neighbour warp (the resampling of
predicted label maps back to the original resolution, paper section
"Pre- and post-processing") against the oracle's labels, bit for bit, and
against the labels the fused warp writes for the same matrix."""
import numpy as np
import pytest
import torch

import oracle
import paper_1811_11226_amd as ctaug
from synth import AugmentRanges, draw_affine_params, phantom_pair

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _oracle_labels(lbl, M, out_dim, label_fill):
    _, lref = oracle.warp(np.zeros(lbl.shape, np.float32), M, out_dim, lbl=lbl,
                          label_fill=label_fill, want_img=False, want_lbl=True)
    return lref


def _resample_back(pred_dim, orig_dim):
    # output voxel p of the original grid reads prediction voxel (p + 1/2) r - 1/2
    # per axis, r = pred / orig (the inverse of the down-sampling by r)
    r = [pred_dim[i] / orig_dim[i] for i in range(3)]
    M = np.zeros(12, np.float32)
    for i in range(3):
        M[4 * i + i] = r[i]
        M[4 * i + 3] = 0.5 * r[i] - 0.5
    return M


@pytest.mark.parametrize("pred_dim,orig_dim", [
    ((24, 20, 17), (61, 50, 43)),        # up-sampling back, ragged z (43 % 4 = 3)
    ((33, 31, 29), (33, 31, 29)),        # identity size
    ((40, 36, 12), (80, 72, 96)),        # anisotropic, z aligned to 4
])
def test_labels_resampled_back_match_oracle(pred_dim, orig_dim):
    _, lbl = phantom_pair(pred_dim, seed=sum(pred_dim))
    M = _resample_back(pred_dim, orig_dim)
    got = _np(ctaug.warp_labels(_t(lbl), M, out_dim=orig_dim, label_fill=0))
    assert np.array_equal(got, _oracle_labels(lbl, M, orig_dim, 0))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_labels_only_equal_fused_warp_labels_and_oracle(seed):
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    in_dim, out_dim = (45, 38, 51), (40, 41, 37)
    img, lbl = phantom_pair(in_dim, seed=seed)
    prm = draw_affine_params(rng, AugmentRanges(), in_dim, out_dim)
    _, M = ctaug.affine_matrix(prm, in_dim, out_dim)
    got = _np(ctaug.warp_labels(_t(lbl), M, out_dim=out_dim, label_fill=-3))
    _, fused = ctaug.warp_affine(_t(img), M, lbl=_t(lbl), label_fill=-3, out_dim=out_dim)
    assert np.array_equal(got, _np(fused))
    assert np.array_equal(got, _oracle_labels(lbl, M, out_dim, -3))


def test_labels_only_from_a_strided_crop_view():
    _, lbl = phantom_pair((48, 44, 40), seed=7)
    parent = _t(lbl)
    view = parent[5:37, 3:41, 6:34]          # non-contiguous crop
    crop = np.ascontiguousarray(lbl[5:37, 3:41, 6:34])
    M = np.array([0.9, 0.1, 0.0, 1.5, -0.1, 0.95, 0.05, -2.0, 0.0, 0.0, 1.1, 0.25], np.float32)
    out_dim = (30, 33, 26)
    got = _np(ctaug.warp_labels(view, M, out_dim=out_dim, label_fill=5))
    assert np.array_equal(got, _oracle_labels(crop, M, out_dim, 5))
    assert np.array_equal(got, _np(ctaug.warp_labels(_t(crop), M, out_dim=out_dim,
                                                     label_fill=5)))


def test_labels_only_edge_cases():
    _, lbl = phantom_pair((9, 8, 7), seed=3)
    # every sample outside: label_fill everywhere
    M = np.array([1, 0, 0, 500, 0, 1, 0, 0, 0, 0, 1, 0], np.float32)
    got = _np(ctaug.warp_labels(_t(lbl), M, out_dim=(5, 6, 7), label_fill=-128))
    assert (got == -128).all()
    # half-voxel ties round up, and the last voxel of every axis is reached
    M = np.array([0.5, 0, 0, 0, 0, 0.5, 0, 0, 0, 0, 0.5, 0], np.float32)
    out_dim = (17, 15, 13)
    got = _np(ctaug.warp_labels(_t(lbl), M, out_dim=out_dim, label_fill=0))
    assert np.array_equal(got, _oracle_labels(lbl, M, out_dim, 0))
    # a 1-voxel input and an empty output
    one = np.full((1, 1, 1), 9, np.int8)
    got = _np(ctaug.warp_labels(_t(one), np.eye(3, 4, dtype=np.float32).ravel(),
                                out_dim=(2, 2, 2), label_fill=1))
    assert np.array_equal(got, _oracle_labels(one, np.eye(3, 4, dtype=np.float32).ravel(),
                                              (2, 2, 2), 1))
    empty = ctaug.warp_labels(_t(lbl), M, out_dim=(3, 0, 4))
    assert empty.numel() == 0


def test_labels_only_more_x_slabs_than_one_launch_row():
    """An output with more x slabs (70000) than one launch's second grid axis
    holds (65535): the slabs past it go to a second launch."""
    rng = np.random.default_rng(9)
    lbl = rng.integers(-5, 6, size=(1200, 2, 5)).astype(np.int8)
    M = np.array([1200 / 70000, 0, 0, 0.1, 0, 1, 0, 0, 0, 0, 1.1, -0.2], np.float32)
    out_dim = (70000, 1, 4)
    got = _np(ctaug.warp_labels(_t(lbl), M, out_dim=out_dim, label_fill=3))
    assert np.array_equal(got, _oracle_labels(lbl, M, out_dim, 3))
