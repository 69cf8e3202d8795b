"""Pins of the oracle's crop geometry (steps O1-O8) against things other than itself.

* rotation: scipy's quaternion routine and a hand-worked 90 degree case;
* relative pose: the composition law of rigid motions;
* crop box and membership: exact rational arithmetic with a different
  formulation (cross-product matrix form of the rotation, hull of the 8
  transformed box corners instead of centre/extent);
* closed intervals: dyadic points placed exactly on box faces;
* the paper's margin guarantee (no false negatives, Sec. III);
* the b-side identity with the paper's own selection rule (points of one
  object inside the other's padded box, appendix "Architecture Details");
* rigid-motion equivariance (the augmentation argument of Sec. III-A);
* closed-form sphere-sphere boxes.
"""

from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

from oracle import locc_oracle as O
from paper_2304_09439_amd import inputs as I

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ------------------------------------------------------------------ rotation

def test_rotation_matches_scipy_for_unit_quaternions():
    rng = np.random.default_rng(11)
    q = I.uniform_quaternions(rng, 500)
    R = O.rotation(q)
    ref = Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], axis=1)).as_matrix()
    assert np.max(np.abs(R - ref)) < 2e-15


def test_rotation_hand_example_quarter_turn_about_z():
    s = np.sqrt(0.5)
    R = O.rotation([s, 0.0, 0.0, s])
    np.testing.assert_allclose(R, [[0, -1, 0], [1, 0, 0], [0, 0, 1]], atol=5e-16)
    # the x axis turns into the y axis: an active rotation
    np.testing.assert_allclose(R @ [1.0, 0, 0], [0, 1.0, 0], atol=5e-16)


def _exact_rotation(q):
    """R = I + 2 w [v]x + 2 [v]x^2 with exact rationals (equals the quaternion
    rotation for unit q, and is the same polynomial for any q)."""
    w, x, y, z = (Fraction(float(c)) for c in q)
    V = [[0, -z, y], [z, 0, -x], [-y, x, 0]]
    V2 = [[sum(V[i][k] * V[k][j] for k in range(3)) for j in range(3)] for i in range(3)]
    return [[(1 if i == j else 0) + 2 * w * V[i][j] + 2 * V2[i][j] for j in range(3)] for i in range(3)]


def test_rotation_is_the_quaternion_polynomial_even_when_not_unit():
    rng = np.random.default_rng(12)
    q = (I.uniform_quaternions(rng, 50) * rng.uniform(0.8, 1.2, (50, 1))).astype(np.float32)
    for k in range(50):
        R = O.rotation(q[k])
        E = _exact_rotation(q[k])
        for i in range(3):
            for j in range(3):
                assert abs(Fraction(float(R[i, j])) - E[i][j]) <= Fraction(1, 2 ** 51)


def test_relative_pose_composes_back_to_the_world():
    rng = np.random.default_rng(13)
    for _ in range(200):
        qa, qb = I.uniform_quaternions(rng, 2)
        ta, tb = rng.uniform(-1, 1, (2, 3))
        Ra, Rb = O.rotation(qa), O.rotation(qb)
        Rab, tab = O.relative_pose(Ra, ta, Rb, tb)
        p = rng.uniform(-0.1, 0.1, 3)
        # b's point seen from the world two ways: directly, and through a's frame
        np.testing.assert_allclose(Ra @ (Rab @ p + tab) + ta, Rb @ p + tb, atol=1e-15)


# -------------------------------------------------------- exact crop geometry

def _tiny_scene(seed, n_shapes=12, n_points=32, n_pairs=200, non_unit=False):
    rng = np.random.default_rng(seed)
    lib = I.shape_library(rng, n_shapes, n_points, (3, 5), 0.5)
    sa = rng.integers(0, n_shapes, n_pairs)
    sb = rng.integers(0, n_shapes, n_pairs)
    ta, qa, tb, qb = I.overlapping_pair_poses(rng, lib, sa, sb)
    if non_unit:
        qa = (qa * rng.uniform(0.9, 1.1, (n_pairs, 1))).astype(np.float32)
        qb = (qb * rng.uniform(0.9, 1.1, (n_pairs, 1))).astype(np.float32)
    return lib, sa, sb, ta, qa, tb, qb


def _exact_box_and_members(pa, pb, qa, ta, qb, tb, pad):
    F = Fraction
    Ra, Rb = _exact_rotation(qa), _exact_rotation(qb)
    Rab = [[sum(Ra[k][i] * Rb[k][j] for k in range(3)) for j in range(3)] for i in range(3)]
    d = [F(float(tb[k])) - F(float(ta[k])) for k in range(3)]
    tab = [sum(Ra[k][i] * d[k] for k in range(3)) for i in range(3)]

    def xf(p):
        return [sum(Rab[i][j] * F(float(p[j])) for j in range(3)) + tab[i] for i in range(3)]

    lo_a = [F(float(v)) for v in pa[:, :3].min(axis=0)]
    hi_a = [F(float(v)) for v in pa[:, :3].max(axis=0)]
    lo_b = pb[:, :3].min(axis=0)
    hi_b = pb[:, :3].max(axis=0)
    corners = [xf([(lo_b if (c >> k) & 1 == 0 else hi_b)[k] for k in range(3)]) for c in range(8)]
    P = F(pad)
    lo = [max(lo_a[i], min(c[i] for c in corners)) - P for i in range(3)]
    hi = [min(hi_a[i], max(c[i] for c in corners)) + P for i in range(3)]

    def classify(q):
        near = min(min(abs(q[i] - lo[i]), abs(q[i] - hi[i])) for i in range(3)) < F(1, 10 ** 9)
        return all(lo[i] <= q[i] <= hi[i] for i in range(3)), near

    a = [classify([F(float(v)) for v in p[:3]]) for p in pa]
    b = [classify(xf(p[:3])) for p in pb]
    return lo, hi, a, b


@pytest.mark.parametrize("non_unit", [False, True])
def test_crop_membership_matches_exact_rational_geometry(non_unit):
    lib, sa, sb, ta, qa, tb, qb = _tiny_scene(21 + non_unit, non_unit=non_unit)
    checked = skipped = 0
    for k in range(len(sa)):
        pa, pb = lib.shape_points(sa[k]), lib.shape_points(sb[k])
        g = O.pair_geometry(pa, pb, qa[k], ta[k], qb[k], tb[k], K=32)
        lo, hi, ea, eb = _exact_box_and_members(pa, pb, qa[k], ta[k], qb[k], tb[k], O.PAD_M)
        for i in range(3):
            assert abs(Fraction(float(g.lo[i])) - lo[i]) < Fraction(1, 10 ** 14)
            assert abs(Fraction(float(g.hi[i])) - hi[i]) < Fraction(1, 10 ** 14)
        for mask, exact in ((g.in_a, ea), (g.in_b, eb)):
            for m, (inside, near) in zip(mask, exact):
                if near:
                    skipped += 1
                    continue
                checked += 1
                assert bool(m) == inside
    assert checked > 10000 and skipped < checked // 1000


def _on_face_shapes():
    """A: box [-1/4, 1/4]^3 (corners stored) plus probe points; B: box [-1/8, 1/8]^3."""
    f32 = np.float32
    lo_probe = f32(0.28125)                   # frame-a face value hit by b's probe
    above = np.nextafter(f32(0.03125), f32(1))
    a_pts = [[0.25, 0.25, 0.25], [-0.25, -0.25, -0.25],
             [0.09375, 0.0, 0.0],                                   # on the lower x face
             [np.nextafter(f32(0.09375), f32(0)), 0.0, 0.0],        # just outside it
             [0.1, 0.15625, -0.15625],                              # on both y and z faces
             [0.1, np.nextafter(f32(0.15625), f32(1)), 0.0]]        # just outside y
    b_pts = [[0.125, 0.125, 0.125], [-0.125, -0.125, -0.125],
             [0.03125, 0.0, 0.0],                                   # lands on the upper x face
             [above, 0.0, 0.0]]                                     # lands just outside it
    def cloud(p):
        p = np.asarray(p, np.float32)
        return np.concatenate([p, np.tile(np.float32([1, 0, 0]), (len(p), 1))], axis=1)
    assert lo_probe == f32(0.25) + f32(0.03125)
    return cloud(a_pts), cloud(b_pts)


def test_points_exactly_on_the_box_faces_are_members():
    # identity orientations, b at (1/4, 0, 0), pad 1/32: every number is dyadic
    # and exact, so the box is x in [3/32, 9/32], y and z in [-5/32, 5/32].
    pa, pb = _on_face_shapes()
    g = O.pair_geometry(pa, pb, [1, 0, 0, 0], [0, 0, 0], [1, 0, 0, 0], [0.25, 0, 0], K=8, pad=0.03125)
    np.testing.assert_array_equal(g.lo, [0.09375, -0.15625, -0.15625])
    np.testing.assert_array_equal(g.hi, [0.28125, 0.15625, 0.15625])
    assert list(g.in_a) == [False, False, True, False, True, False]
    # b's corners land at x = 3/8 (outside) and x = 1/8 (inside)
    assert list(g.in_b) == [False, True, True, False]
    assert list(g.idx_a[:2]) == [2, 4] and g.n_a == 2
    assert list(g.idx_b[:2]) == [1, 2] and g.n_b == 2


def test_first_k_keeps_stored_order_and_counts_before_the_cap():
    m = np.zeros(100, bool)
    m[[3, 7, 8, 50, 99]] = True
    idx, n = O.first_k(m, 3)
    assert list(idx) == [3, 7, 8] and n == 5
    idx, n = O.first_k(m, 8)
    assert list(idx) == [3, 7, 8, 50, 99, -1, -1, -1] and n == 5
    idx, n = O.first_k(np.zeros(10, bool), 4)
    assert list(idx) == [-1] * 4 and n == 0


def test_nan_coordinates_are_never_members():
    pa, pb = _on_face_shapes()
    g = O.pair_geometry(pa, pb, [1, 0, 0, 0], [0, 0, 0], [1, 0, 0, 0], [np.nan, 0, 0], K=8, pad=0.03125)
    assert not g.in_a.any() and not g.in_b.any() and g.n_a == 0 and g.n_b == 0


# ---------------------------------------------------------------- invariants

def test_no_false_negatives_within_the_margin(small_scene):
    """Sec. III: the padded selection never misses a part of one object that is
    within the margin of the other (here: Euclidean distance <= pad)."""
    sc = small_scene
    geoms, _, _ = O.crop(sc.lib.pts, sc.lib.offsets, sc.pos, sc.quat, sc.shape, sc.pairs, K=64)
    close_pairs = 0
    r = O.PAD_M * (1 - 1e-9)
    for g in geoms:
        pa = sc.lib.shape_points(sc.shape[g.a])
        pb = sc.lib.shape_points(sc.shape[g.b])
        qa = pa[:, :3].astype(np.float64)
        qb = O.transform_points(g.Rab, g.tab, pb[:, :3])
        ta, tb = cKDTree(qa), cKDTree(qb)
        need_a = np.array([len(x) > 0 for x in tb.query_ball_point(qa, r)])
        need_b = np.array([len(x) > 0 for x in ta.query_ball_point(qb, r)])
        assert not (need_a & ~g.in_a).any()
        assert not (need_b & ~g.in_b).any()
        close_pairs += need_a.any()
    assert close_pairs >= 20  # the check is not vacuous


def test_b_side_matches_the_papers_counter_box_rule(small_scene):
    """b's members are exactly b's points inside a's AABB widened by the margin
    (the paper's rule: keep one object's parts inside the other's padded box)."""
    sc = small_scene
    geoms, _, _ = O.crop(sc.lib.pts, sc.lib.offsets, sc.pos, sc.quat, sc.shape, sc.pairs, K=64)
    for g in geoms:
        pa = sc.lib.shape_points(sc.shape[g.a])
        pb = sc.lib.shape_points(sc.shape[g.b])
        lo_a = pa[:, :3].min(axis=0).astype(np.float64) - O.PAD_M
        hi_a = pa[:, :3].max(axis=0).astype(np.float64) + O.PAD_M
        q = O.transform_points(g.Rab, g.tab, pb[:, :3])
        np.testing.assert_array_equal(g.in_b, np.all((lo_a <= q) & (q <= hi_a), axis=1))


def _compose(qg, tg, q, t):
    rg = Rotation.from_quat([qg[1], qg[2], qg[3], qg[0]])
    r = Rotation.from_quat([q[1], q[2], q[3], q[0]])
    x, y, z, w = (rg * r).as_quat()
    return np.array([w, x, y, z]), rg.apply(np.asarray(t, np.float64)) + tg


def test_crop_sets_are_invariant_under_a_rigid_motion_of_the_world(small_scene):
    """Sec. III-A: moving both objects by the same rigid motion leaves the
    occupied volume, and hence the crop, unchanged (FP64 poses, points within
    1e-9 of a face excluded)."""
    sc = small_scene
    rng = np.random.default_rng(31)
    same = 0
    for p in range(sc.n_pairs):
        a, b, _ = O.canonical(*sc.pairs[p])
        pa = sc.lib.shape_points(sc.shape[a])
        pb = sc.lib.shape_points(sc.shape[b])
        qa = np.asarray(sc.quat[a], np.float64)
        qb = np.asarray(sc.quat[b], np.float64)
        qa, qb = qa / np.linalg.norm(qa), qb / np.linalg.norm(qb)
        g0 = O.pair_geometry(pa, pb, qa, sc.pos[a], qb, sc.pos[b], K=64)
        qg = I.uniform_quaternions(rng, 1)[0]
        tg = rng.uniform(-2, 2, 3)
        qa1, ta1 = _compose(qg, tg, qa, sc.pos[a])
        qb1, tb1 = _compose(qg, tg, qb, sc.pos[b])
        g1 = O.pair_geometry(pa, pb, qa1, ta1, qb1, tb1, K=64)
        np.testing.assert_allclose(g1.lo, g0.lo, atol=1e-13)
        np.testing.assert_allclose(g1.hi, g0.hi, atol=1e-13)
        qb_pts = O.transform_points(g0.Rab, g0.tab, pb[:, :3])
        for mask0, mask1, pts in ((g0.in_a, g1.in_a, pa[:, :3]), (g0.in_b, g1.in_b, qb_pts)):
            d = np.minimum(np.abs(pts - g0.lo), np.abs(pts - g0.hi)).min(axis=1)
            far = d > 1e-9
            np.testing.assert_array_equal(mask0[far], mask1[far])
        same += 1
    assert same == sc.n_pairs


# --------------------------------------------------------------- sphere boxes

def test_sphere_crop_box_closed_form():
    """Spheres with identity orientation and centres on the x axis: the box is
    [max(-ra, d - rb) - pad, min(ra, d + rb) + pad] in x and
    [max(-ra, -rb) - pad, min(ra, rb) + pad] in y and z."""
    rng = np.random.default_rng(41)
    for _ in range(50):
        ra, rb = (float(np.float32(v)) for v in rng.uniform(0.02, 0.08, 2))
        d = float(np.float32(rng.uniform(0.5, 1.2) * (ra + rb)))
        lib = I.sphere_library(rng, 2, 256, [ra, rb])
        pa, pb = lib.shape_points(0), lib.shape_points(1)
        g = O.pair_geometry(pa, pb, [1, 0, 0, 0], [0, 0, 0], [1, 0, 0, 0], [d, 0, 0], K=256)
        lo = np.array([max(-ra, d - rb), max(-ra, -rb), max(-ra, -rb)]) - O.PAD_M
        hi = np.array([min(ra, d + rb), min(ra, rb), min(ra, rb)]) + O.PAD_M
        np.testing.assert_allclose(g.lo, lo, atol=1e-16)
        np.testing.assert_allclose(g.hi, hi, atol=1e-16)
        xb = pb[:, :3].astype(np.float64) + [d, 0, 0]
        for pts, mask in ((pa[:, :3].astype(np.float64), g.in_a), (xb, g.in_b)):
            far = np.minimum(np.abs(pts - lo), np.abs(pts - hi)).min(axis=1) > 1e-12
            expect = np.all((pts >= lo) & (pts <= hi), axis=1)
            np.testing.assert_array_equal(mask[far], expect[far])


def test_b_side_rows_are_radial_for_spheres(small_scene):
    """Encoder rows of a sphere b, in a's frame: normal = (point - centre_b) / r_b.
    The centre of b in a's frame comes from scipy, not from the oracle."""
    sc = small_scene
    geoms, _, _ = O.crop(sc.lib.pts, sc.lib.offsets, sc.pos, sc.quat, sc.shape, sc.pairs, K=64)
    checked = 0
    for g in geoms:
        rb = sc.lib.radius[sc.shape[g.b]]
        if np.isnan(rb) or len(g.rows_b) == 0:
            continue
        qa = sc.quat[g.a].astype(np.float64)
        ra = Rotation.from_quat([qa[1], qa[2], qa[3], qa[0]])
        cb = ra.inv().apply(sc.pos[g.b].astype(np.float64) - sc.pos[g.a])
        np.testing.assert_allclose(g.rows_b[:, 3:6], (g.rows_b[:, :3] - cb) / rb, atol=2e-5)
        checked += 1
    assert checked >= 8
