"""The counting argument behind the 32-bit tile sums of the affine image
adjoint: for q = A p + t, the samples p of one 8 x 8 x 16 output tile whose
trilinear corners include a given input cell all lie in A^-1 of that cell's
2-cube, so along output axis i at most floor((2 + 2 delta) sum_j |A^-1_ij|)
+ 1 of them share a coordinate range, capped by the tile's extent; the
product bounds how many samples can add into one cell, which keeps the sums
within 2^30.  Checked by brute force (every corner of every sample counted,
FP32 coordinates) over random affine maps with rotation, shear, and
scalings from strong upsampling to downsampling."""
import numpy as np
import pytest

EXT = np.array([8, 8, 16])


def sample_bound(A, delta):
    Ai = np.linalg.inv(A)
    K = 1
    for i in range(3):
        w = (2.0 + 2.0 * delta) * np.abs(Ai[i]).sum()
        K *= min(EXT[i], int(np.floor(w)) + 1) if w < EXT[i] else EXT[i]
    return K


def max_samples_per_cell(A, t, origin):
    p = np.stack(np.meshgrid(np.arange(8), np.arange(8), np.arange(16), indexing="ij"),
                 -1).reshape(-1, 3) + origin
    q = (p @ A.T + t).astype(np.float32).astype(np.float64)
    f = np.floor(q).astype(np.int64)
    keys = []
    for d in np.ndindex(2, 2, 2):
        c = f + np.array(d)
        keys.append((c[:, 0] * 1_000_003 + c[:, 1]) * 1_000_033 + c[:, 2])
    _, counts = np.unique(np.concatenate(keys), return_counts=True)
    return counts.max()


@pytest.mark.parametrize("seed", range(4))
def test_samples_per_cell_within_the_bound(seed):
    rng = np.random.default_rng(seed)
    tight = 0
    for _ in range(100):
        A = np.eye(3) + rng.uniform(-1, 1, (3, 3)) * rng.uniform(0.0, 1.2)
        A *= rng.uniform(0.25, 2.0)
        if abs(np.linalg.det(A)) < 1e-3:
            continue
        t = rng.uniform(-50, 50, 3)
        m = max_samples_per_cell(A, t, rng.integers(0, 100, 3))
        K = sample_bound(A, 1e-4)
        assert m <= K, (m, K, A)
        tight += m == K
    assert tight > 0                   # the bound is reached, not just safe


def test_identity_and_half_scale():
    """Identity: each cell collects at most the 8 samples around it (2 per
    axis); scale 0.5: 5 per axis (125 <= 2^7, the largest count the 32-bit
    sums take)."""
    assert sample_bound(np.eye(3), 1e-4) == 27
    assert max_samples_per_cell(np.eye(3), np.array([0.25, 0.5, 0.75]), np.zeros(3, int)) == 8
    assert sample_bound(0.5 * np.eye(3), 1e-4) == 125
    assert max_samples_per_cell(0.5 * np.eye(3), np.zeros(3), np.zeros(3, int)) <= 125
