"""Pins of the pose-gradient oracle (oracle.pose_grad): central finite
differences of a forward pass written independently (rows rebuilt through the
world frame with the polynomial rotation of the unnormalised quaternion, the
crop selection frozen), wherever the argmax rows and every ReLU pattern do
not change across the step; zero gradient for crops that select nothing of
the second object; the caller's order."""

import numpy as np
import pytest

from oracle import locc_oracle as O
from oracle import pose_grad as PG
from paper_2304_09439_amd import inputs as I

LW = I.SCALE_WIDTHS
WIDTHS = (LW.h1, LW.h2, LW.hh)
K = 128


@pytest.fixture(scope="module")
def scene():
    return I.scale_workload(n_pairs=24)


@pytest.fixture(scope="module")
def weights():
    return I.flatten_weights(I.gaussian_weights(LW, seed=0, bias_std=0.1))


def _rot(q):
    """R(q) = I + 2 w [v]x + 2 [v]x^2 for q = (w, v) as given (equal to O3's polynomial)."""
    w, v = float(q[0]), np.asarray(q[1:], np.float64)
    V = np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]])
    return np.eye(3) + 2 * w * V + 2 * V @ V


def _frozen_logit(g, pts_a, pts_b, pa, qa, pb, qb, wts):
    """Logit with g's selection frozen, rows rebuilt through the world frame; also a signature of the
    piecewise-smooth region (argmax rows of b, the ReLU patterns of the encoder on b and of the head)."""
    W1, b1, W2, b2, H1, c1, H2, c2, H3, c3 = wts
    Ra, Rb = _rot(qa), _rot(qb)
    sa, sb = g.idx_a[g.idx_a >= 0], g.idx_b[g.idx_b >= 0]
    rows_a = np.asarray(pts_a[sa], np.float64)
    world = np.asarray(pts_b[sb, :3], np.float64) @ Rb.T + pb
    rows_b = np.concatenate([(world - pa) @ Ra, np.asarray(pts_b[sb, 3:], np.float64) @ Rb.T @ Ra], axis=1)
    z = np.concatenate([O.encode(rows_a, W1, b1, W2, b2), O.encode(rows_b, W1, b1, W2, b2)])
    u1 = z @ H1.T + c1
    u2 = O.relu(u1) @ H2.T + c2
    pre1 = rows_b @ W1.T + b1
    s = O.relu(pre1) @ W2.T
    arg = np.argmax(s, axis=0) if len(rows_b) else np.zeros(0)
    sig = (tuple(arg), tuple(u1 > 0), tuple(u2 > 0), (pre1 > 0).tobytes(), tuple(z > 0))
    return float(O.relu(u2) @ H3[0] + c3[0]), sig


def test_gradient_matches_central_differences(scene, weights):
    r = PG.pose_gradients(scene.lib.pts, scene.lib.offsets, scene.pos, scene.quat, scene.shape, scene.pairs,
                          weights, WIDTHS, K)
    wts = O.unpack_weights(weights, *WIDTHS)
    h = 1e-6
    checked = skipped = 0
    worst = 0.0
    for p, g in enumerate(r["geoms"]):
        pts_a = scene.lib.shape_points(int(scene.shape[g.a]))
        pts_b = scene.lib.shape_points(int(scene.shape[g.b]))
        x = np.concatenate([scene.pos[g.a], scene.quat[g.a], scene.pos[g.b], scene.quat[g.b]]).astype(np.float64)
        parts = lambda v: (v[0:3], v[3:7], v[7:10], v[10:14])
        pa, qa, pb, qb = parts(x)
        base, sig = _frozen_logit(g, pts_a, pts_b, pa, qa, pb, qb, wts)
        assert abs(base - r["logit"][p]) <= 1e-9 * max(1.0, abs(base))
        an = r["grad"][p] if g.sgn > 0 else np.concatenate([r["grad"][p][7:], r["grad"][p][:7]])
        scale = np.abs(an).max()
        if scale == 0:
            continue
        for k in range(14):
            e = np.zeros(14)
            e[k] = h
            lp, sp = _frozen_logit(g, pts_a, pts_b, *parts(x + e), wts)
            lm, sm = _frozen_logit(g, pts_a, pts_b, *parts(x - e), wts)
            if sp != sig or sm != sig:
                skipped += 1
                continue
            fd = (lp - lm) / (2 * h)
            worst = max(worst, abs(fd - an[k]) / scale)
            checked += 1
    assert checked > 0.9 * (checked + skipped) and checked > 200
    assert worst < 1e-6, worst


def test_empty_second_crop_gives_zero_and_caller_order(scene, weights):
    i, j = (int(v) for v in scene.pairs[0])  # a pair with a non-zero gradient
    k, l = (int(v) for v in scene.pairs[3])
    pos = scene.pos.copy()
    pos[l] = pos[k] + [3.0, 0.0, 0.0]        # pair (k, l) far apart: nothing selected
    pairs = np.array([[k, l], [l, k], [i, j], [j, i], [4, 4]], np.int32)
    r = PG.pose_gradients(scene.lib.pts, scene.lib.offsets, pos, scene.quat, scene.shape, pairs, weights,
                          WIDTHS, K)
    assert np.all(r["grad"][0] == 0) and np.all(r["grad"][1] == 0)
    np.testing.assert_array_equal(r["grad"][3], np.concatenate([r["grad"][2][7:], r["grad"][2][:7]]))
    assert np.isnan(r["grad"][4]).all() and np.isnan(r["logit"][4])
    assert np.abs(r["grad"][2]).max() > 0
    # a common translation of both objects leaves the logit unchanged
    np.testing.assert_allclose(r["grad"][2][0:3], -r["grad"][2][7:10], rtol=1e-12, atol=1e-15)
