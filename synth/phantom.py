"""CT-like ellipsoid phantoms.

Stand-in for the paper's 130-scan CT organ dataset (3 mm^3 abdominal CT with
lung, liver, bone, kidney, bladder labels), which is not available.  Values are
integer Hounsfield units so that int16 and float32 copies hold identical values;
labels use the paper's six classes (0 = background/other, 1..5 organs, 3 = bone).

Recipe: background -1000 HU; 6-12 soft-tissue ellipsoids with intensity
U(0, 400) HU and label 1 + (k mod 5); then 2 dense ellipsoids U(1150, 1250) HU
with label 3 painted last (later ellipsoids overwrite earlier ones).  Centres
are uniform over the central 80% box, semi-axes U(0.05, 0.25) * dim per axis,
orientation a uniformly random rotation (normalised Gaussian quaternion).
"""
import numpy as np

BACKGROUND_HU = -1000


def _rotation_from_quaternion(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _paint(img, lbl, center, semi, rot, value, label):
    dims = np.array(img.shape)
    r = float(np.max(semi))
    lo = np.maximum(np.floor(center - r).astype(np.int64), 0)
    hi = np.minimum(np.ceil(center + r).astype(np.int64) + 1, dims)
    if np.any(hi <= lo):
        return
    gx = np.arange(lo[0], hi[0], dtype=np.float64)[:, None, None] - center[0]
    gy = np.arange(lo[1], hi[1], dtype=np.float64)[None, :, None] - center[1]
    gz = np.arange(lo[2], hi[2], dtype=np.float64)[None, None, :] - center[2]
    # coordinates in the ellipsoid's own frame: rot^T (p - c)
    ex = rot[0, 0] * gx + rot[1, 0] * gy + rot[2, 0] * gz
    ey = rot[0, 1] * gx + rot[1, 1] * gy + rot[2, 1] * gz
    ez = rot[0, 2] * gx + rot[1, 2] * gy + rot[2, 2] * gz
    inside = (ex / semi[0]) ** 2 + (ey / semi[1]) ** 2 + (ez / semi[2]) ** 2 <= 1.0
    sl = (slice(lo[0], hi[0]), slice(lo[1], hi[1]), slice(lo[2], hi[2]))
    img[sl][inside] = value
    if lbl is not None:
        lbl[sl][inside] = label


def phantom_pair(dims, seed):
    """Return (image int16 [X][Y][Z] HU, labels int8 [X][Y][Z]) for `seed`."""
    dims = tuple(int(d) for d in dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    img = np.full(dims, BACKGROUND_HU, dtype=np.int16)
    lbl = np.zeros(dims, dtype=np.int8)
    d = np.array(dims, dtype=np.float64)
    n_soft = int(rng.integers(6, 13))
    specs = []
    for k in range(n_soft):
        specs.append((int(rng.integers(0, 401)), 1 + (k % 5)))
    for _ in range(2):
        specs.append((int(rng.integers(1150, 1251)), 3))
    for value, label in specs:
        center = 0.1 * d + 0.8 * d * rng.random(3) - 0.5 * (d > 0)
        center = np.maximum(center, 0.0)
        semi = np.maximum((0.05 + 0.20 * rng.random(3)) * d, 0.5)
        rot = _rotation_from_quaternion(rng.standard_normal(4))
        _paint(img, lbl, center, semi, rot, value, label)
    return img, lbl


def phantom(dims, seed, dtype=np.float32):
    """Image only, converted (exactly) to `dtype`."""
    img, _ = phantom_pair(dims, seed)
    return img.astype(dtype)
