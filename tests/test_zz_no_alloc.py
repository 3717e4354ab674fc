"""The allocation-free affine adjoint (static device scratch) against the
workspace entry point, through the C ABI: two calls in a row, the second on a
smaller input, each compared with the workspace call (grad_M bit for bit,
grad_img within the gradient bar) and with the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_1811_11226_amd as ctaug
from synth import AugmentRanges, PhotoParams, draw_affine_params, phantom_pair

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _grad_bar(got, ref, what):
    got, ref = got.astype(np.float64), np.asarray(ref, np.float64)
    nref = np.linalg.norm(ref)
    assert np.linalg.norm(got - ref) <= 1e-4 * max(nref, 1e-30), what
    floor = 1e-2 * np.abs(ref).max()
    assert (np.abs(got - ref) <= 1e-4 * np.maximum(np.abs(ref), floor)).all(), what


@pytest.mark.parametrize("dtype", [np.float32, np.int16])
def test_noalloc_backward_matches_workspace_call(dtype):
    rng = np.random.default_rng(77)
    ph = PhotoParams(gain=0.95, offset=3.0, sigma=10.0, window=False, seed=9, volume_id=1,
                     occlude=True, occ_lo=6.0, occ_hi=11.5)
    for dims, out_dim in [((72, 64, 56), (80, 72, 60)), ((30, 26, 34), (20, 22, 18))]:
        img_np, _ = phantom_pair(dims, seed=int(sum(dims)))
        img_np = img_np.astype(dtype)
        prm = draw_affine_params(rng, AugmentRanges(), dims, out_dim)
        _, M = ctaug.affine_matrix(prm, dims, out_dim)
        g_np = rng.standard_normal(out_dim).astype(np.float32)
        img = torch.from_numpy(img_np).to(DEV)
        g = torch.from_numpy(g_np).to(DEV)
        gi = torch.zeros(dims, dtype=torch.float32, device=DEV)
        gM = torch.full((12,), np.nan, dtype=torch.float64, device=DEV)
        ctaug.ops.warp_affine_backward_noalloc(img, M, g, photo=ph, grad_img=gi, grad_M=gM)
        ref_img, ref_M = ctaug.warp_affine_backward(img, M, g, photo=ph)
        assert np.array_equal(_np(gM).view(np.uint64), _np(ref_M).view(np.uint64)), out_dim
        _grad_bar(_np(gi), _np(ref_img), f"grad_img {out_dim}")
        r_img, r_M, _ = oracle.warp_backward(img_np, M, g_np, photo=ph)
        _grad_bar(_np(gi), r_img, f"grad_img vs oracle {out_dim}")
        _grad_bar(_np(gM), r_M, f"grad_M vs oracle {out_dim}")
