"""Pins of the voxel-embedding oracle (oracle.voxel_locc), each against
something other than the oracle itself: scipy's N-d correlation for the
convolution; adjointness (a property of the mathematics) for the transposed
convolution; cell boundaries enumerated one by one for the grid assignment;
a per-point loop for the cell max; constructed weights that turn the whole
encoder and the predictor into closed forms (which fixes the U-Net's wiring,
its skip order and its index conventions); dense sampling of each cell for
the no-false-negative guarantee of the margin; world-frame invariance."""

import numpy as np
import pytest
from scipy import signal
from scipy.spatial.transform import Rotation

from oracle import locc_oracle as O
from oracle import voxel_locc as V
from paper_2304_09439_amd import inputs as I


def test_weight_layout_matches_the_generator():
    assert [tuple(w.shape) for w in I.voxel_weights()] == [tuple(s) for s in V.layer_shapes()]
    assert V.n_weights() == sum(w.size for w in I.voxel_weights())


@pytest.mark.parametrize("pad", [0, 1])
def test_conv_is_scipy_correlation(pad):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 4, 4, 4))
    W = rng.standard_normal((3, 5, 3, 3, 3))
    b = rng.standard_normal(3)
    y = V.conv3d(x, W, b, pad)
    xp = np.pad(x, ((0, 0),) + ((pad, pad),) * 3)
    ref = np.stack([sum(signal.correlate(xp[c], W[o, c], mode="valid") for c in range(5)) + b[o] for o in range(3)])
    assert y.shape == (3, 4 + 2 * pad - 2) + (4 + 2 * pad - 2,) * 2
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("pad", [0, 1])
def test_transposed_conv_is_the_adjoint_of_conv(pad):
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4, 4, 4, 4)) if pad else rng.standard_normal((4, 6, 6, 6))
    W = rng.standard_normal((3, 4, 3, 3, 3))
    y = rng.standard_normal((3,) + V.conv3d(x, W, np.zeros(3), pad).shape[1:])
    lhs = np.sum(V.conv3d(x, W, np.zeros(3), pad) * y)
    xt = V.conv3d_transpose(y, W.transpose(1, 0, 2, 3, 4), np.zeros(4), pad)
    assert xt.shape == x.shape
    assert np.isclose(lhs, np.sum(x * xt), rtol=1e-12)
    # 4^3 -> 6^3 without padding, 4^3 -> 4^3 with
    assert V.conv3d_transpose(np.ones((1, 4, 4, 4)), np.ones((1, 1, 3, 3, 3)), np.zeros(1), pad).shape[1] == 6 - 2 * pad


def test_voxel_index_against_enumerated_boundaries():
    rng = np.random.default_rng(3)
    lo, hi = np.array([-0.07, -0.031, 0.012]), np.array([0.05, 0.044, 0.09])
    p = lo + rng.random((4000, 3)) * (hi - lo)
    p = np.concatenate([p, [lo, hi, [hi[0], lo[1], (lo[2] + hi[2]) / 2]]])
    edges = [lo[k] + np.arange(1, V.M) * (hi[k] - lo[k]) / V.M for k in range(3)]
    ok = np.all([np.min(np.abs(p[:, k, None] - edges[k][None]), axis=1) > 1e-12 for k in range(3)], axis=0)
    cell = np.stack([np.sum(p[:, k, None] >= edges[k][None], axis=1) for k in range(3)], axis=1)
    ref = (cell[:, 0] * V.M + cell[:, 1]) * V.M + cell[:, 2]
    got = V.voxel_index(p, lo, hi)
    np.testing.assert_array_equal(got[ok], ref[ok])
    assert got[-3] == 0 and got[-2] == V.M ** 3 - 1           # lo in the first cell, hi in the last
    # an axis of zero extent puts every point in its first layer
    flat = V.voxel_index(np.array([[0.1, 0.2, 0.5]]), np.array([0.0, 0.2, 0.0]), np.array([1.0, 0.2, 1.0]))
    assert flat[0] == (0 * V.M + 0) * V.M + 3


def test_cell_max_against_a_point_loop():
    rng = np.random.default_rng(4)
    idx = rng.integers(0, V.M ** 3, 300)
    idx[idx == 17] = 18                       # cell 17 stays empty
    feat = np.maximum(rng.standard_normal((300, 7)), 0)
    ref = np.zeros((V.M ** 3, 7))
    for r in range(300):
        ref[idx[r]] = np.maximum(ref[idx[r]], feat[r])
    np.testing.assert_array_equal(V.voxel_max(feat, idx), ref)
    assert not V.voxel_max(feat, idx)[17].any()


def _constructed_encoder():
    """Weights under which E[cell][0] = 107 * max over the cell's points of (x + 1) for interior cells (0 on
    the border shell), E[:, 1] = 30 * the largest interior cell value, E[:, 2] = 30 * their mean."""
    w = [np.zeros(s) for s in V.layer_shapes()]
    w[0][0, 0], w[1][0] = 1.0, 1.0            # h0 = x + 1
    w[2][0, 0] = w[4][0, 0] = 1.0             # passed through layers 2 and 3
    c = (1, 1, 1)
    w[6][(0, 0) + c] = 1.0                    # c1 = g shifted by one cell (no padding)
    w[8][(0, 0) + c] = 2.0                    # c2 = 2 c1
    w[10][(0, 0) + c] = 3.0                   # c3 = 6 c1
    w[12][(0, 0) + c] = 5.0                   # c4 = 30 c1
    w[14][(0, 0) + c] = 1.0                   # d1 = c4 = 30 c1
    w[16][(0, 0) + c], w[16][(0, 128) + c] = 1.0, 7.0     # d2 = d1 + 7 c3 = 72 c1
    w[18][(0, 0) + c], w[18][(0, 128) + c] = 1.0, 11.0    # d3 = d2 + 11 c2 = 94 c1
    w[20][(0, 0) + c], w[20][(0, 128) + c] = 1.0, 13.0    # d4 = shift(d3 + 13 c1) = 107 g
    w[22][0, 0] = 1.0                         # E0 = d4 channel 0
    w[22][1, 128] = 1.0                       # E1 = global max of c4 channel 0
    w[22][2, 256] = 1.0                       # E2 = global mean of c4 channel 0
    return w


def test_constructed_encoder_gives_the_closed_form():
    lib = I.scale_library(n_shapes=2, n_points=2048)
    xyz = lib.shape_points(1)[:, :3].astype(np.float64)
    lo, hi = O.aabb(xyz)
    E = V.shape_embedding(xyz, _constructed_encoder())
    cell = V.voxel_index(xyz, lo, hi)
    g = np.zeros(V.M ** 3)
    np.maximum.at(g, cell, xyz[:, 0] + 1.0)
    i0, i1, i2 = np.unravel_index(np.arange(V.M ** 3), (V.M,) * 3)
    interior = (i0 > 0) & (i0 < V.M - 1) & (i1 > 0) & (i1 < V.M - 1) & (i2 > 0) & (i2 < V.M - 1)
    np.testing.assert_allclose(E[:, 0], np.where(interior, 107.0 * g, 0.0), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(E[:, 1], 30.0 * g[interior].max(), rtol=1e-13)
    np.testing.assert_allclose(E[:, 2], 30.0 * g[interior].mean(), rtol=1e-13)
    assert not E[:, 3:].any()
    assert (g[interior] > 0).sum() > 10      # the shape reaches into the interior


def _pose(rng, spread=0.06):
    q = I.uniform_quaternions(rng, 1)[0]
    return rng.standard_normal(3) * spread, q


def test_margin_leaves_no_false_negative():
    """Every cell of a that has a point inside b's box is selected (and vice versa)."""
    lib = I.scale_library(n_shapes=4, n_points=2048)
    boxes = [O.aabb(lib.shape_points(s)[:, :3]) for s in range(4)]
    rng = np.random.default_rng(5)
    u = rng.random((40, 3))
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], np.float64)
    frac = np.concatenate([corners, u])      # sample positions inside a cell, in cell units
    n_sel = 0
    for trial in range(30):
        sa, sb = rng.integers(0, 4, 2)
        ta, qa = _pose(rng)
        tb, qb = _pose(rng)
        Ra = Rotation.from_quat(np.r_[qa[1:], qa[:1]]).as_matrix()
        Rb = Rotation.from_quat(np.r_[qb[1:], qb[:1]]).as_matrix()
        Rab, tab = O.relative_pose(O.rotation(qa), ta, O.rotation(qb), tb)
        sel_a, sel_b = V.select_cells(Rab, tab, boxes[sa], boxes[sb])
        n_sel += sel_a.sum() + sel_b.sum()
        for (s_self, s_other, R_self, t_self, R_other, t_other, sel) in (
                (sa, sb, Ra, ta, Rb, tb, sel_a), (sb, sa, Rb, tb, Ra, ta, sel_b)):
            lo, hi = boxes[s_self]
            size = (hi - lo) / V.M
            i0, i1, i2 = np.unravel_index(np.arange(V.M ** 3), (V.M,) * 3)
            base = lo + np.stack([i0, i1, i2], axis=1) * size            # cell min corners
            pts = base[:, None, :] + frac[None] * size                   # [cells, samples, 3]
            world = pts @ R_self.T + t_self
            other = (world - t_other) @ R_other                         # into the other object's frame
            lo_o, hi_o = boxes[s_other]
            hit = np.all((other >= lo_o - 1e-12) & (other <= hi_o + 1e-12), axis=2).any(axis=1)
            assert not np.any(hit & ~sel), (trial, np.flatnonzero(hit & ~sel))
    assert n_sel > 100


def test_predictor_closed_forms_and_empty_crops():
    lib = I.scale_library(n_shapes=2, n_points=2048)
    wv = [np.zeros(s) for s in V.layer_shapes()]
    rng = np.random.default_rng(6)
    emb = rng.standard_normal((2, V.M ** 3, V.F_EMB))
    # logit = max(ReLU(mean_a[0]), ReLU(mean_b[0]))
    wv[24][0, 0] = 1.0
    wv[26][0, 0] = wv[28][0, 0] = wv[30][0, 0] = wv[32][0, 0] = wv[34][0, 0] = wv[36][0, 0] = 1.0
    pos = np.array([[0.0, 0.0, 0.0], [0.02, -0.01, 0.005], [5.0, 0.0, 0.0]], np.float32)
    quat = np.array([[1, 0, 0, 0], [0.9, 0.1, -0.3, 0.2], [1, 0, 0, 0]], np.float32)
    shape = np.array([0, 1, 1], np.int32)
    pairs = np.array([[0, 1], [1, 0], [0, 2], [0, 0], [0, 7]], np.int32)
    flat = I.flatten_weights(wv)
    r = V.detect(lib.pts, lib.offsets, pos, quat, shape, pairs, flat, emb=emb)
    boxes = [O.aabb(lib.shape_points(s)[:, :3]) for s in range(2)]
    Rab, tab = O.relative_pose(O.rotation(quat[0]), pos[0], O.rotation(quat[1]), pos[1])
    sa, sb = V.select_cells(Rab, tab, boxes[0], boxes[1])
    ma, mb = emb[0][sa].mean(axis=0), emb[1][sb].mean(axis=0)
    want = max(max(np.float32(ma[0]), 0.0), max(np.float32(mb[0]), 0.0))
    assert sa.any() and sb.any()
    assert r["logit"][0] == pytest.approx(want, rel=1e-12) and r["logit"][1] == r["logit"][0]
    np.testing.assert_array_equal(r["counts"][0], [sa.sum(), sb.sum()])
    np.testing.assert_array_equal(r["counts"][1], [sb.sum(), sa.sum()])         # caller order
    np.testing.assert_array_equal(r["counts"][2], [0, 0])                       # far apart: nothing selected
    assert not r["pooled"][2].any() and r["logit"][2] == 0.0
    assert np.isnan(r["logit"][3:]).all() and (r["counts"][3:] == -1).all()
    # logit = max(ReLU(t_ba.x), ReLU(t_ab.x)) = |x_b - x_a| for unrotated objects
    wv = [np.zeros(s) for s in V.layer_shapes()]
    wv[24][0, V.F_EMB + 0] = 1.0
    wv[26][0, 0] = wv[28][0, 0] = wv[30][0, 0] = wv[32][0, 0] = wv[34][0, 0] = wv[36][0, 0] = 1.0
    quat[1] = [1, 0, 0, 0]
    r = V.detect(lib.pts, lib.offsets, pos, quat, shape, pairs[:2], I.flatten_weights(wv), emb=emb)
    assert r["logit"][0] == pytest.approx(0.02, rel=1e-6) and r["logit"][1] == r["logit"][0]


def test_world_frame_invariance():
    lib = I.scale_library(n_shapes=3, n_points=2048)
    rng = np.random.default_rng(7)
    w = I.flatten_weights(I.voxel_weights(seed=1, bias_std=0.1))
    emb = V.library_embeddings(lib.pts, lib.offsets, w)
    n = 8
    pos = (rng.standard_normal((n, 3)) * 0.04).astype(np.float32)
    quat = I.uniform_quaternions(rng, n).astype(np.float32)
    shape = rng.integers(0, 3, n).astype(np.int32)
    pairs = np.array([(i, j) for i in range(n) for j in range(i + 1, n)], np.int32)
    r0 = V.detect(lib.pts, lib.offsets, pos, quat, shape, pairs, w, emb=emb)
    # a common rigid motion of every object: quarter turn about z and a shift
    qz = np.array([np.cos(np.pi / 4), 0, 0, np.sin(np.pi / 4)])
    R = Rotation.from_quat(np.r_[qz[1:], qz[:1]])
    pos2 = R.apply(pos.astype(np.float64)) + [0.3, -0.2, 0.1]
    quat2 = (R * Rotation.from_quat(np.c_[quat[:, 1:], quat[:, :1]].astype(np.float64))).as_quat()
    quat2 = np.c_[quat2[:, 3:], quat2[:, :3]]
    r1 = V.detect(lib.pts, lib.offsets, pos2.astype(np.float32), quat2.astype(np.float32), shape, pairs, w, emb=emb)
    assert (r0["counts"] > 0).sum() > 10
    frac_same = np.mean(np.all(r0["counts"] == r1["counts"], axis=1))
    assert frac_same >= 0.95                     # a cell exactly on a widened face may flip with float32 poses
    same = np.all(r0["counts"] == r1["counts"], axis=1)
    np.testing.assert_allclose(r1["logit"][same], r0["logit"][same], rtol=1e-4, atol=1e-4)


def test_pose_inputs_are_each_object_in_the_others_frame():
    """V7 against the relative pose computed the other way round (b's frame from scratch)."""
    rng = np.random.default_rng(8)
    for _ in range(20):
        ta, qa = _pose(rng)
        tb, qb = _pose(rng)
        Ra, Rb = O.rotation(qa), O.rotation(qb)
        Rab, tab = O.relative_pose(Ra, ta, Rb, tb)
        Rba, tba = O.relative_pose(Rb, tb, Ra, ta)
        pose_a, pose_b = V.pose_inputs(Rab, tab)
        np.testing.assert_allclose(pose_a, np.concatenate([tba, Rba.ravel()]), rtol=0, atol=1e-14)
        np.testing.assert_array_equal(pose_b, np.concatenate([tab, Rab.ravel()]))
