"""Comparison of the nonrigid GPU path with the plain FP64 B-spline definition.

The warp with a B-spline displacement evaluates the field in FP32, so its
coordinate q differs from the one built on the FP64 field (rounded once to
FP32) by at most delta per axis: the FP32 field's rounding bound plus the
rounding of the coordinate sums.  Against the FP64-field oracle that leaves
exactly three effects, each bounded here rather than masked wholesale:

  * labels j = floor(q + 0.5) may differ only where q lies within delta of a
    half-integer tie, and then only between the candidate voxels on either
    side of the tie;
  * the trilinear value moves by at most 3 delta times the spread of the
    corner values around q (the interpolant's Lipschitz constant per axis is
    at most that spread);
  * dV/dq jumps across cell planes, so gradients that carry dV/dq (M,
    displacement, control grid) are compared with the upstream gradient
    zeroed where q lies within delta of an integer plane; inside a cell dV/dq
    moves by at most 4 delta times the corner spread, and the image adjoint's
    weights by at most 3 delta per contribution.  These elementwise
    allowances are bounds, loose for large sums; the normwise 1e-4 bar is
    applied without any allowance.

The FP32 field bound is the one pinned against the FP64 definition for the
oracle's own FP32 evaluation (each of the 64 terms carries about 20 u
relative rounding error and the weights sum to one; the cell coordinate
s = p / h is off by at most 2 u s per axis, |du/ds| <= 2 max|C|), doubled to
cover any FP32 evaluation order.
"""
import numpy as np

U = 2.0 ** -24


def fp32_field_bound(C):
    """Bound on |u_fp32 - u_fp64| for an FP32 evaluation of the cubic B-spline
    field of control grid C [3][Gx][Gy][Gz]."""
    G = C.shape[1:]
    return 2.0 * U * (20 + 12 * (max(G) - 3)) * float(np.abs(C).max())


def coords(M, out_dim, u):
    """q = A p + b + u in FP64 from the FP32 matrix M and field u [3][...]."""
    A = np.asarray(M, np.float32).astype(np.float64).reshape(3, 4)
    P = np.indices(out_dim).astype(np.float64)
    q = np.empty((3,) + tuple(out_dim))
    for i in range(3):
        q[i] = A[i, 0] * P[0] + A[i, 1] * P[1] + A[i, 2] * P[2] + A[i, 3] + u[i]
    return q


def delta(M, out_dim, C, u):
    """Per-axis bound on |q_gpu - q_ref| (FP32-field coordinate against the
    FP64-field one): the field bound plus a few ulps of the coordinate sums on
    both sides."""
    A = np.asarray(M, np.float32).astype(np.float64).reshape(3, 4)
    last = np.maximum(np.asarray(out_dim, np.float64) - 1.0, 0.0)
    d = np.empty(3)
    for i in range(3):
        S = np.abs(A[i, :3]) @ last + abs(A[i, 3]) + float(np.abs(u[i]).max())
        d[i] = fp32_field_bound(C) + 8.0 * U * S
    return d


def near_ties(q, d):
    """Per voxel: True on axes where q is within d of a half-integer."""
    return np.abs(q - (np.floor(q) + 0.5)) <= d[:, None, None, None]


def near_planes(q, d):
    """True where q is within d of an integer plane on some axis."""
    return (np.abs(q - np.round(q)) <= d[:, None, None, None]).any(axis=0)


def _padded(vol, fill, pad=3):
    return np.pad(np.asarray(vol, np.float64), pad, constant_values=fill)


def assert_labels_up_to_ties(got, ref, q, d, lbl, label_fill, max_frac=1e-3, what=""):
    """Labels equal except within d of a .5 tie, where the GPU label must be
    one of the labels on either side of the tie; such voxels are rare."""
    bad = np.argwhere(got != ref)
    assert len(bad) <= max_frac * got.size, \
        f"{what}: {len(bad)} label differences of {got.size}"
    ties = near_ties(q, d)
    n = lbl.shape
    for p in map(tuple, bad):
        qp = q[(slice(None),) + p]
        tp = ties[(slice(None),) + p]
        assert tp.any(), f"{what}: label differs at {p}, q={qp}, no axis near a tie"
        cand = []
        for i in range(3):
            j = np.floor(qp[i] + 0.5)
            cand.append({int(j), int(j) - 1, int(j) + 1} if tp[i] else {int(j)})
        labels = set()
        for jx in cand[0]:
            for jy in cand[1]:
                for jz in cand[2]:
                    inside = 0 <= jx < n[0] and 0 <= jy < n[1] and 0 <= jz < n[2]
                    labels.add(int(lbl[jx, jy, jz]) if inside else int(label_fill))
        assert int(got[p]) in labels, f"{what}: label {got[p]} at {p} is no candidate {labels}"


def corner_spread(img, q, d, fill):
    """max - min of the corner values (fill outside the volume) of every cell
    within d of the points q [3][...]: bounds the interpolant's change per
    unit move per axis there.  The cells floor(q - d) .. floor(q + d) <=
    floor(q - d) + 1 have their corners in the 3^3 block centred on
    floor(q - d) + 1, whose extremes come from 3^3 max / min filters."""
    from scipy import ndimage
    pad = 3
    P = _padded(img, fill, pad)
    hi = ndimage.maximum_filter(P, size=3, mode="nearest")
    lo = ndimage.minimum_filter(P, size=3, mode="nearest")
    n = np.asarray(img.shape)
    idx = tuple(np.clip(np.floor(q[i] - d[i]).astype(np.int64) + 1, 1 - pad, n[i] + pad - 2) + pad
                for i in range(3))
    return hi[idx] - lo[idx]


def dvdq_slack(img, q, d, fill, g):
    """Per output voxel, a bound on how far g(p) dV/dq_i(p) can move when q
    moves by at most d inside its cell: dV/dq_i is bilinear in the other two
    fractions with slopes at most twice the corner spread, so
    |delta(g dV/dq_i)| <= 4 max(d) spread |g|."""
    return 4.0 * float(d.max()) * corner_spread(img, q, d, fill) * np.abs(np.asarray(g, np.float64))


def grad_M_slack(a):
    """Allowance of the 12 parameter gradients from per-voxel allowances a of
    g dV/dq (the same for the three components): sum_p a(p) |[x, y, z, 1]_j|."""
    P = np.indices(a.shape).astype(np.float64)
    s = np.array([(a * P[0]).sum(), (a * P[1]).sum(), (a * P[2]).sum(), a.sum()])
    return np.tile(s, 3)


def assert_values_within_field_slack(got, ref, img, q, d, fill, R, what="", strict_frac=0.99,
                                     gain=1.0):
    """|V_gpu - V_ref| <= 1e-5 max(|ref|, R) + 3 d |gain| spread(q); and most
    voxels meet the plain 1e-5 bar.  (The spread is evaluated only where the
    plain bar is exceeded.)"""
    got = got.astype(np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    tol = 1e-5 * np.maximum(np.abs(ref), R)
    err = np.abs(got - ref)
    over = np.flatnonzero(~(err <= tol))
    assert over.size <= (1.0 - strict_frac) * err.size, \
        f"{what}: {over.size / err.size:.3%} beyond 1e-5"
    if over.size:
        qo = q.reshape(3, -1)[:, over]
        slack = float(d.max()) * 3.0 * abs(gain) * corner_spread(img, qo, d, fill)
        bad = ~(err[over] <= tol[over] + slack)
        i = int(np.argmax(bad)) if bad.any() else 0
        assert not bad.any(), \
            f"{what}: error {err[over][i]:.3e} beyond {tol[over][i]:.3e} + {slack[i]:.3e}"


def corner_abs_sums(q, absg, in_dim):
    """For every input voxel c, the sum of |g(p)| over output voxels p whose
    cells within reach (floor(q) - 1 .. floor(q) + 2 per axis) include c: the
    image adjoint's change from weights that move by 3 d is at most
    3 d times this sum."""
    n = np.asarray(in_dim)
    acc = np.zeros(tuple(int(v) + 8 for v in n))
    base = [np.floor(q[i]).astype(np.int64) - 1 for i in range(3)]
    inside = np.ones(q.shape[1:], bool)
    for i in range(3):
        inside &= (base[i] > -4) & (base[i] < n[i] + 2)
    b = [np.clip(base[i], -3, n[i] + 1)[inside] + 3 for i in range(3)]
    w = absg[inside]
    for a in range(4):
        for bb in range(4):
            for c in range(4):
                np.add.at(acc, (b[0] + a, b[1] + bb, b[2] + c), w)
    return acc[3:3 + n[0], 3:3 + n[1], 3:3 + n[2]]


def assert_grad_masked(got, ref, what="", slack=None):
    """Gradient bar (normwise 1e-4, elementwise 1e-4 max(|ref|, 1e-2 ||ref||_inf)),
    with an optional elementwise allowance."""
    got = got.astype(np.float64)
    nref = np.linalg.norm(ref)
    assert np.linalg.norm(got - ref) <= 1e-4 * max(nref, 1e-30), \
        f"{what}: normwise {np.linalg.norm(got - ref) / max(nref, 1e-30):.3e}"
    floor = 1e-2 * np.abs(ref).max() if ref.size else 0.0
    tol = 1e-4 * np.maximum(np.abs(ref), floor)
    if slack is not None:
        tol = tol + slack
    err = np.abs(got - ref)
    assert err.size == 0 or (err <= tol).all(), \
        f"{what}: elementwise {(err / np.maximum(tol, 1e-300)).max():.3e} of the allowance"
