"""The five seeded synthetic workloads of the augmentation path.

  c1  one 128x128x64 float32 phantom + int8 labels, random affine, full
      photometrics (gain, offset, noise sigma = 10 HU, window [-1000, 1000],
      gamma), output 128x128x64.
  c2  one 512x512x320 int16 phantom + labels -> float32 + int8, same ranges.
  c3  16 int16 phantoms with per-axis sizes U{96..256}, each with its own
      affine, crop shift and photometrics, cropped to a common 120x120x160
      float32 + int8 output (the paper's network input size).
  c4  8 float32 128^3 phantoms, affine warp without labels or photometrics,
      upstream gradient ~ N(0, 1), for the differentiable warp.
  c5  4 float32 256^3 phantoms, affine composed with a cubic B-spline
      displacement from an 8^3 control grid ~ N(0, 4^2 voxel^2), additive
      noise sigma ~ U(0, 25) HU, upstream gradient ~ N(0, 1).

Seeds: phantom = 20181127 + 1000 * config + volume index; transform draws =
phantom + 1; noise key = phantom + 2; volume id = index in the batch.  Every
generator takes optional reduced dimensions so that parity tests can run the
same recipe at sizes the oracle finishes in seconds.
"""
from dataclasses import dataclass
from typing import Optional

import numpy as np

from .draws import AugmentRanges, PhotoParams, draw_affine_params, draw_photo
from .phantom import phantom_pair

SEED_BASE = 20181127
FILL_HU = -1000.0
LABEL_FILL = 0


def seeds(config, index):
    p = SEED_BASE + 1000 * config + index
    return p, p + 1, p + 2


@dataclass
class Job:
    img: np.ndarray                  # int16 or float32 [X][Y][Z]
    lbl: Optional[np.ndarray]        # int8 [X][Y][Z] or None
    out_dim: tuple
    prm: np.ndarray                  # 27 raw affine draws (see draws.py)
    photo: Optional[PhotoParams]     # None = no photometric transform
    fill: float = FILL_HU
    label_fill: int = LABEL_FILL
    volume_id: int = 0

    @property
    def in_dim(self):
        return tuple(self.img.shape)


def _job(config, index, in_dim, out_dim, dtype, ranges, with_labels=True, with_photo=True):
    ps, ts, ns = seeds(config, index)
    img, lbl = phantom_pair(in_dim, ps)
    rng = np.random.Generator(np.random.PCG64(ts))
    prm = draw_affine_params(rng, ranges, in_dim, out_dim)
    photo = draw_photo(rng, ranges, seed=ns, volume_id=index) if with_photo else None
    return Job(img=img.astype(dtype), lbl=lbl if with_labels else None, out_dim=tuple(out_dim),
               prm=prm, photo=photo, volume_id=index)


def c1(dims=(128, 128, 64)):
    return [_job(1, 0, dims, dims, np.float32, AugmentRanges())]


def c2(dims=(512, 512, 320)):
    return [_job(2, 0, dims, dims, np.int16, AugmentRanges())]


def c3(n=16, size_range=(96, 256), out_dim=(120, 120, 160), batch=0):
    """Batch `batch` of the c3 dataset: volumes batch*n .. batch*n + n - 1."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 3000 - 1))
    sizes = rng.integers(size_range[0], size_range[1] + 1, size=((batch + 1) * n, 3))
    return [_job(3, i, tuple(int(s) for s in sizes[i]), out_dim, np.int16, AugmentRanges())
            for i in range(batch * n, (batch + 1) * n)]


def c4(n=8, dim=128):
    ranges = AugmentRanges()
    jobs = [_job(4, i, (dim,) * 3, (dim,) * 3, np.float32, ranges, with_labels=False,
                 with_photo=False) for i in range(n)]
    grads = [np.random.Generator(np.random.PCG64(seeds(4, i)[2] + 7)).standard_normal(
        (dim,) * 3).astype(np.float32) for i in range(n)]
    return jobs, grads


def c5(n=4, dim=256, grid=8, ctrl_std=4.0):
    ranges = AugmentRanges(sigma=(0.0, 25.0), window=False, gain=(1.0, 1.0), offset=(0.0, 0.0),
                           gamma=(1.0, 1.0))
    jobs = [_job(5, i, (dim,) * 3, (dim,) * 3, np.float32, ranges, with_labels=False)
            for i in range(n)]
    ctrls, grads = [], []
    for i in range(n):
        r = np.random.Generator(np.random.PCG64(seeds(5, i)[2] + 11))
        ctrls.append((ctrl_std * r.standard_normal((3, grid, grid, grid))).astype(np.float32))
        grads.append(r.standard_normal((dim,) * 3).astype(np.float32))
    return jobs, ctrls, grads
