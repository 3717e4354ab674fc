"""Random draws of augmentation parameters from user ranges.

The paper draws every geometric and photometric parameter uniformly from
user-specified ranges (rotation, scaling, shearing, per-axis reflection
probability, generic affine, centre displacement, noise sigma, window limits),
and the training crop location uniformly at random.  This module performs only
those draws.  Turning them into the matrix [A|b] is the library's job (and,
independently, the oracle's); the layout of the 27-value parameter vector is
shared so that both sides receive the same numbers.

Parameter vector (float64, N_AFFINE_PARAMS = 27):
  [0:3]   rotation angles about x, y, z (radians)
  [3:6]   scale factors along x, y, z
  [6:9]   shears h_xy, h_xz, h_yz
  [9:12]  reflection flags for x, y, z (0.0 or 1.0)
  [12:21] generic 3x3 matrix, row-major (identity when unused)
  [21:24] displacement of the volume centre d (input voxels)
  [24:27] crop shift k (input voxels)
"""
from dataclasses import dataclass, field

import numpy as np

N_AFFINE_PARAMS = 27


@dataclass
class AugmentRanges:
    rot_deg: tuple = (30.0, 30.0, 30.0)        # |theta_i| <= rot_deg[i]
    scale: tuple = (0.8, 1.2)                   # s ~ U(scale)
    isotropic: bool = True                      # one s for all axes
    shear: tuple = (0.0, 0.0, 0.0)              # |h| <= shear[i]
    reflect_prob: tuple = (0.0, 0.0, 0.0)       # P(reflect about axis i)
    generic: float = 0.0                        # G = I + E, E_ij ~ U(+-generic)
    disp: tuple = (10.0, 10.0, 10.0)            # |d_i| <= disp[i]
    crop: bool = True                           # uniform crop shift when out < in
    gain: tuple = (0.9, 1.1)
    offset: tuple = (-20.0, 20.0)
    gamma: tuple = (0.8, 1.25)
    win_lo: tuple = (-1000.0, -1000.0)
    win_hi: tuple = (1000.0, 1000.0)
    sigma: tuple = (10.0, 10.0)
    window: bool = True
    occlusion: float = 0.0                      # delta_max of the occluded slab (0 = none)


@dataclass
class PhotoParams:
    gain: float = 1.0
    offset: float = 0.0
    sigma: float = 0.0
    win_lo: float = -1000.0
    win_hi: float = 1000.0
    gamma: float = 1.0
    window: bool = False
    seed: int = 0
    volume_id: int = 0
    occlude: bool = False
    occ_lo: float = 0.0                         # occluded output slab occ_lo <= z <= occ_hi
    occ_hi: float = -1.0

    def occ_pair(self):
        """(occ_lo, occ_hi) rounded to FP32, or None without occlusion."""
        if not self.occlude:
            return None
        return float(np.float32(self.occ_lo)), float(np.float32(self.occ_hi))

    def as_tuple6(self):
        """(gain, offset, sigma, win_lo, win_hi, gamma) rounded to FP32, the
        precision in which both the library and the oracle receive them."""
        return tuple(float(np.float32(v)) for v in
                     (self.gain, self.offset, self.sigma, self.win_lo, self.win_hi, self.gamma))


def identity_affine_params():
    p = np.zeros(N_AFFINE_PARAMS, dtype=np.float64)
    p[3:6] = 1.0
    p[12:21] = np.eye(3).ravel()
    return p


def _u(rng, lo, hi):
    return float(lo + (hi - lo) * rng.random())


def draw_affine_params(rng, ranges, in_dim, out_dim):
    p = identity_affine_params()
    for i in range(3):
        r = np.deg2rad(ranges.rot_deg[i])
        p[i] = _u(rng, -r, r)
    if ranges.isotropic:
        p[3:6] = _u(rng, *ranges.scale)
    else:
        p[3:6] = [_u(rng, *ranges.scale) for _ in range(3)]
    p[6:9] = [_u(rng, -h, h) for h in ranges.shear]
    p[9:12] = [1.0 if rng.random() < pr else 0.0 for pr in ranges.reflect_prob]
    if ranges.generic > 0:
        e = ranges.generic
        p[12:21] = (np.eye(3) + rng.uniform(-e, e, size=(3, 3))).ravel()
    p[21:24] = [_u(rng, -d, d) for d in ranges.disp]
    if ranges.crop:
        for i in range(3):
            m = max(0.0, 0.5 * (in_dim[i] - out_dim[i]))
            p[24 + i] = _u(rng, -m, m)
    return p


def draw_occlusion(rng, delta_max, z_max):
    """Occluded slab of the output's z axis: height delta ~ U[0, delta_max]
    and start z ~ U[-delta_max, z_max], so that every z in [0, z_max] has the
    same chance of being occluded (the paper's occlusion paragraph)."""
    delta = _u(rng, 0.0, delta_max)
    start = _u(rng, -delta_max, z_max)
    return start, start + delta


def draw_photo(rng, ranges, seed, volume_id, out_z=None):
    ph = PhotoParams(
        gain=_u(rng, *ranges.gain), offset=_u(rng, *ranges.offset),
        sigma=_u(rng, *ranges.sigma), win_lo=_u(rng, *ranges.win_lo),
        win_hi=_u(rng, *ranges.win_hi), gamma=_u(rng, *ranges.gamma),
        window=ranges.window, seed=int(seed), volume_id=int(volume_id))
    if ranges.occlusion > 0 and out_z is not None:
        ph.occlude = True
        ph.occ_lo, ph.occ_hi = draw_occlusion(rng, ranges.occlusion, out_z - 1)
    return ph
