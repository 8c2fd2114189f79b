"""The collision-free deterministic batch check of the update (Alg. 1's stress
step with the clamped update), shared by the CPU test that measures what the
check can resolve and the GPU tests that apply it to the HIP kernels.

A batch is the first K sampled terms of an iteration, greedily thinned so that
no two kept terms share a coordinate slot; applied in any order it gives one
result, which the oracle computes in FP64 from the same FP32 start.  The check
bounds, per coordinate the batch moves, the difference between a result and
the FP64 result by

    1e-5 * |displacement of the FP64 result|
    + one FP32 ulp of the coordinate (the rounding of the stored result)
    + mu * |delta_axis| * (4 * eps32 + |fl32(d) - d| / mag)

The last term is what an FP32 evaluation of the step cannot avoid: the FP32
distance mag carries a relative error of about eps32, which (mag - d) passes
on to r = mu (mag - d) / (2 mag) as an absolute error of about mu * eps32, and
the displacement r * delta_axis multiplies it by |delta_axis|; a reference
distance d above 2^24 nt is itself rounded to FP32.  It matters only for terms
whose points are already within about 10% of their reference distance.
"""
import numpy as np

import oracle as O

EPS32 = 2.0 ** -23
REL_BAR = 1e-5
K_TERMS = 65536


def slots(og, i, j, f):
    """Coordinate slots a = 2 node(i) + e_i and b = 2 node(j) + e_j of each term."""
    sn = og.step_node
    a = 2 * (sn[np.asarray(i, np.int64)] & 0x7FFFFFFF).astype(np.int64) + (f & 1)
    b = 2 * (sn[np.asarray(j, np.int64)] & 0x7FFFFFFF).astype(np.int64) + ((f >> 1) & 1)
    return a, b


def collision_free(og, i, j, f, limit=K_TERMS):
    """Indices of the terms kept: in order, a term is kept when it is not
    skipped and neither of its slots was seen before."""
    a, b = slots(og, i, j, f)
    seen = set()
    keep = []
    for k in range(len(i)):
        if f[k] & 8 or a[k] in seen or b[k] in seen:
            continue
        seen.add(int(a[k]))
        seen.add(int(b[k]))
        keep.append(k)
        if len(keep) >= limit:
            break
    return np.array(keep, np.int64)


def start_coords(og, it):
    """Start coordinates near the origin (normal, sd 100 nt), so that FP32
    storage resolves the displacements of the batch finely."""
    rng = np.random.default_rng(1000 + it)
    return rng.normal(scale=100.0, size=4 * og.n_nodes).astype(np.float32)


def _distances(og, pos, i, j, f):
    nl = og.node_len.astype(np.int64)
    sn = og.step_node

    def endpoint(s, e):
        s = np.asarray(s, np.int64)
        rev = (sn[s] >> 31).astype(np.int64)
        return pos[s] + nl[sn[s] & 0x7FFFFFFF] * (e.astype(np.int64) ^ rev)

    return np.abs(endpoint(i, f & 1) - endpoint(j, (f >> 1) & 1))


def check(og, pos, i, j, f, eta, start, got, ref):
    """Worst ratio of |got - ref| to the bound over the moved coordinates (the
    batch passes when it is <= 1), and whether the untouched coordinates kept
    their start values exactly.  i, j, f: the kept terms; start: FP32 start;
    got: a result (FP64 array of FP32 values); ref: the oracle's FP64 result."""
    n2 = 2 * og.n_nodes
    a, b = slots(og, i, j, f)
    d = _distances(og, pos, i, j, f).astype(np.float64)
    s64 = start.astype(np.float64)
    dx = s64[a] - s64[b]
    dy = s64[n2 + a] - s64[n2 + b]
    mag = np.sqrt(dx * dx + dy * dy)
    mu = np.minimum(eta / (d * d), 1.0)
    d_round = np.abs(d.astype(np.float32).astype(np.float64) - d)
    with np.errstate(divide="ignore", invalid="ignore"):
        lost = np.where(mag > 0, 4 * EPS32 + d_round / mag, 0.0)
    worst = 0.0
    touched = np.zeros(2 * n2, bool)
    for plane, delta in ((0, dx), (n2, dy)):
        kappa = mu * np.abs(delta) * lost
        for slot in (a, b):
            c = plane + slot
            touched[c] = True
            disp = ref[c] - s64[c]
            ulp = np.spacing(np.maximum(np.abs(s64[c]), np.abs(ref[c])).astype(np.float32)).astype(np.float64)
            bound = REL_BAR * np.abs(disp) + ulp + kappa
            worst = max(worst, float(np.max(np.abs(got[c] - ref[c]) / bound)))
    untouched_ok = bool(np.array_equal(got[~touched], s64[~touched]))
    return worst, untouched_ok


def fp64_result(og, eta, i, j, f, start, r_scale=1.0):
    """The oracle's FP64 result of the batch (r scaled by r_scale: a planted
    error, for the resolution measurement only)."""
    ref = start.astype(np.float64)
    if r_scale == 1.0:
        applied = O.apply_terms_f64(og, eta, i, j, f, ref)
    else:
        applied = O.apply_terms_f64_scaled(og, eta, r_scale, i, j, f, ref)
    return ref, applied


def resolution(og, pos, i, j, f, eta, start, grid=None):
    """The smallest relative error eps of the update's r, on a grid of quarter
    decades from 1e-7 to 1, that the check rejects when the batch is applied
    with r * (1 + eps) and stored in FP32; None if it rejects none."""
    if grid is None:
        grid = [10.0 ** (e / 4.0) for e in range(-28, 1)]
    ref, _ = fp64_result(og, eta, i, j, f, start)
    for eps in grid:
        pert, _ = fp64_result(og, eta, i, j, f, start, 1.0 + eps)
        got = pert.astype(np.float32).astype(np.float64)
        worst, _ = check(og, pos, i, j, f, eta, start, got, ref)
        if worst > 1.0:
            return eps
    return None
