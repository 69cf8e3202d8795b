"""Pins of the broad-phase oracle (oracle.broad_phase).

Against the input generator's own broad phase (scipy rotations, vectorised
einsum: a different formulation and evaluation order), the corner hull of
each rotated shape box, containment of every transformed point, and the
listing order.
"""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import broad_phase as BP
from paper_2304_09439_amd import inputs as I


@pytest.fixture(scope="module")
def envs():
    return I.env_workload(n_envs=192, steps=2, target_pairs=2e5 * 192 / 4096)


def _boxes(envs, step):
    return BP.world_boxes(envs.lib.pts, envs.lib.offsets, envs.pos[step], envs.quat[step], envs.shape)


def test_pairs_equal_the_generator_broad_phase(envs):
    for step in range(envs.n_steps):
        lo, hi = _boxes(envs, step)
        got = BP.broad_phase(lo, hi, envs.env_offsets)
        ref = envs.pairs[step]
        assert len(got) > 100
        key = lambda a: a[np.lexsort((a[:, 1], a[:, 0]))]
        np.testing.assert_array_equal(key(got), key(ref))


def test_listing_order_and_environments(envs):
    lo, hi = _boxes(envs, 0)
    pairs = BP.broad_phase(lo, hi, envs.env_offsets)
    assert np.all(pairs[:, 0] < pairs[:, 1])
    assert np.all(envs.env[pairs[:, 0]] == envs.env[pairs[:, 1]])
    env = envs.env[pairs[:, 0]]
    order = np.lexsort((pairs[:, 1], pairs[:, 0], env))
    np.testing.assert_array_equal(order, np.arange(len(pairs)))


def test_world_box_is_the_hull_of_the_rotated_corners(envs):
    lo, hi = _boxes(envs, 1)
    c, e = BP.shape_boxes(envs.lib.pts, envs.lib.offsets)
    signs = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], np.float64)
    # the quaternion as given (float32, not renormalised): R = I + 2 w [v]x + 2 [v]x^2
    q = envs.quat[1].astype(np.float64)
    w_, v = q[:, 0], q[:, 1:]
    Vx = np.zeros((len(q), 3, 3))
    Vx[:, 0, 1], Vx[:, 0, 2], Vx[:, 1, 2] = -v[:, 2], v[:, 1], -v[:, 0]
    Vx -= Vx.transpose(0, 2, 1)
    R = np.eye(3)[None] + 2 * w_[:, None, None] * Vx + 2 * Vx @ Vx
    corners = c[envs.shape][:, None, :] + signs[None] * e[envs.shape][:, None, :]
    w = np.einsum("nij,nkj->nki", R, corners) + envs.pos[1].astype(np.float64)[:, None, :]
    np.testing.assert_allclose(lo, w.min(axis=1), rtol=0, atol=1e-12)
    np.testing.assert_allclose(hi, w.max(axis=1), rtol=0, atol=1e-12)


def test_every_transformed_point_lies_in_its_world_box(envs):
    lo, hi = _boxes(envs, 0)
    q = envs.quat[0].astype(np.float64)
    R = Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], axis=1)).as_matrix()
    for k in range(0, len(envs.shape), 97):
        s = envs.shape[k]
        pts = envs.lib.pts[envs.lib.offsets[s]:envs.lib.offsets[s + 1], :3].astype(np.float64)
        w = pts @ R[k].T + envs.pos[0, k]
        assert np.all(w >= lo[k] - 1e-12) and np.all(w <= hi[k] + 1e-12)


def test_empty_and_single_object_environments():
    lo = np.array([[0.0, 0, 0], [0.5, 0, 0], [2.0, 0, 0]])
    hi = lo + 1.0
    # environments: {}, {0}, {1, 2}: 1 and 2 do not touch (1.5 < 2.0); then one where 0 and 1 touch on a face
    pairs = BP.broad_phase(lo, hi, np.array([0, 0, 1, 3]))
    assert pairs.shape == (0, 2)
    pairs = BP.broad_phase(lo, hi, np.array([0, 2]))
    np.testing.assert_array_equal(pairs, [[0, 1]])
    lo2 = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    np.testing.assert_array_equal(BP.broad_phase(lo2, lo2 + 1.0, np.array([0, 2])), [[0, 1]])   # closed intervals


def test_invalid_shapes_and_clamped_environments(envs):
    """Readings for input outside the paper's setting: an out-of-range shape id
    gives a NaN box (in no pair); environment bounds are clamped to [0, n]."""
    shape = envs.shape.copy()
    shape[[3, 10]] = [-1, envs.lib.n_shapes]
    lo, hi = BP.world_boxes(envs.lib.pts, envs.lib.offsets, envs.pos[0], envs.quat[0], shape)
    assert np.isnan(lo[[3, 10]]).all() and np.isfinite(np.delete(lo, [3, 10], axis=0)).all()
    pairs = BP.broad_phase(lo, hi, envs.env_offsets)
    assert not np.isin(pairs, [3, 10]).any()
    lo0, hi0 = _boxes(envs, 0)
    full = BP.broad_phase(lo0, hi0, envs.env_offsets)
    keep = ~np.isin(full, [3, 10]).any(axis=1)
    np.testing.assert_array_equal(pairs, full[keep])
    # bounds past either end clamp; a reversed range is empty
    n = len(lo0)
    got = np.concatenate([BP.broad_phase(lo0, hi0, np.array([-5, 4, 2, 60])),
                          BP.broad_phase(lo0, hi0, np.array([n - 30, n + 7]))])
    ref = np.concatenate([BP.broad_phase(lo0[:4], hi0[:4], np.array([0, 4])),
                          BP.broad_phase(lo0, hi0, np.array([2, 60])),
                          BP.broad_phase(lo0, hi0, np.array([n - 30, n]))])
    assert len(ref) > 0
    np.testing.assert_array_equal(got, ref)
