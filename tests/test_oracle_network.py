"""Pins of the oracle's network and outputs (steps O2, O8-O11).

* constructed weights turn the network into the closed-form sphere-sphere
  contact, checked against hand-derived fixtures (tests/golden);
* swapping a pair negates the normal and leaves everything else bitwise equal;
* outputs move with a rigid motion of the world (Sec. III-A argument);
* the max-pool is order-free and the batched formulation agrees;
* the empty crop pools to zero; invalid pairs give NaN and -1.
"""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import locc_oracle as O
from paper_2304_09439_amd import inputs as I

from helpers import FIELDS, sphere_case_scene, sphere_cases, sphere_probe_weights

SW = I.SMALL_WIDTHS
WID = (SW.h1, SW.h2, SW.hh)


def test_constructed_weights_reproduce_closed_form_sphere_contact():
    cases = sphere_cases()
    sc = sphere_case_scene(cases)
    r = O.detect_scene(sc, sphere_probe_weights(SW, beta=4.0), WID, K=64)
    for k, c in enumerate(cases):
        out = r["contacts"][k]
        swapped = sc.pairs[k, 0] > sc.pairs[k, 1]
        tol = 1e-12 if c["exact"] else 1e-8       # inexact cases: radii and d rounded to float32
        assert out[7] == pytest.approx(c["depth"], abs=tol)
        assert out[0] == pytest.approx(4.0 * c["depth"], abs=4 * tol)
        assert (out[0] > 0) == c["flag"]
        np.testing.assert_allclose(out[1:4], [c["point_x"], 0, 0], atol=tol)
        # the normal points from the caller's first object to its second
        np.testing.assert_array_equal(out[4:7], [-1.0, 0, 0] if swapped else [1.0, 0, 0])
        if c["exact"]:
            assert out[7] == c["depth"] and out[1] == c["point_x"]


def test_constructed_weights_agree_with_generated_sphere_labels():
    """Randomised version: radii, separations and twists drawn at random."""
    rng = np.random.default_rng(3)
    cases = []
    for _ in range(40):
        ra, rb = (float(np.float32(v)) for v in rng.uniform(0.02, 0.08, 2))
        d = float(np.float32(ra + rb + rng.uniform(-0.5 * min(ra, rb), 0.009)))
        cases.append(dict(ra=ra, rb=rb, d=d, theta=float(rng.uniform(-3, 3))))
    sc = sphere_case_scene(cases, swap_every_other=True)
    r = O.detect_scene(sc, sphere_probe_weights(SW), WID, K=64)
    lab = I.sphere_labels(sc)
    np.testing.assert_allclose(r["contacts"][:, 7], lab["depth"], atol=1e-12)
    np.testing.assert_allclose(r["contacts"][:, 1:4], lab["point"], atol=1e-12)
    np.testing.assert_allclose(r["contacts"][:, 4:7], lab["normal"], atol=1e-12)
    np.testing.assert_array_equal(r["contacts"][:, 0] > 0, lab["flag"])


def _scene_weights(bias=0.1):
    return I.flatten_weights(I.gaussian_weights(SW, seed=0, bias_std=bias))


def test_swapping_a_pair_negates_only_the_normal(small_scene):
    sc = small_scene
    w = _scene_weights()
    r1 = O.detect_scene(sc, w, WID, K=64)
    sw = I.Scene(sc.lib, sc.pos, sc.quat, sc.shape, np.ascontiguousarray(sc.pairs[:, ::-1]))
    r2 = O.detect_scene(sw, w, WID, K=64)
    c1, c2 = r1["contacts"], r2["contacts"]
    for sl in (FIELDS["logit"], FIELDS["point"], FIELDS["depth"]):
        np.testing.assert_array_equal(c1[:, sl], c2[:, sl])
    np.testing.assert_array_equal(c1[:, 4:7], -c2[:, 4:7])
    np.testing.assert_array_equal(r1["counts"], r2["counts"][:, ::-1])
    np.testing.assert_array_equal(r1["idx"], r2["idx"][:, ::-1])


def test_outputs_follow_a_rigid_motion_of_the_world(small_scene):
    sc = small_scene
    w = _scene_weights()
    rng = np.random.default_rng(8)
    q = sc.quat.astype(np.float64)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    pos = sc.pos.astype(np.float64)
    r0 = O.detect(sc.lib.pts, sc.lib.offsets, pos, q, sc.shape, sc.pairs, w, WID, K=64)
    qg = I.uniform_quaternions(rng, 1)[0]
    rg = Rotation.from_quat([qg[1], qg[2], qg[3], qg[0]])
    tg = rng.uniform(-2, 2, 3)
    r = rg * Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], axis=1))
    xyzw = r.as_quat()
    q1 = np.concatenate([xyzw[:, 3:], xyzw[:, :3]], axis=1)
    pos1 = rg.apply(pos) + tg
    r1 = O.detect(sc.lib.pts, sc.lib.offsets, pos1, q1, sc.shape, sc.pairs, w, WID, K=64)
    same = np.all(r0["idx"] == r1["idx"], axis=(1, 2))
    assert same.mean() > 0.95
    c0, c1 = r0["contacts"][same], r1["contacts"][same]
    scale = np.abs(c0).max()
    np.testing.assert_allclose(c1[:, 0], c0[:, 0], atol=1e-10 * scale)
    np.testing.assert_allclose(c1[:, 7], c0[:, 7], atol=1e-10 * scale)
    np.testing.assert_allclose(c1[:, 1:4], rg.apply(c0[:, 1:4]) + tg, atol=1e-10 * scale)
    np.testing.assert_allclose(c1[:, 4:7], rg.apply(c0[:, 4:7]), atol=1e-10 * scale)


def test_max_pool_is_independent_of_member_order(small_scene):
    sc = small_scene
    Wl = O.unpack_weights(_scene_weights(), *WID)
    geoms, _, _ = O.crop(sc.lib.pts, sc.lib.offsets, sc.pos, sc.quat, sc.shape, sc.pairs, K=64)
    rng = np.random.default_rng(4)
    for g in geoms:
        for rows in (g.rows_a, g.rows_b):
            f = O.encode(rows, *Wl[:4])
            f2 = O.encode(rows[rng.permutation(len(rows))], *Wl[:4])
            np.testing.assert_array_equal(f, f2)


def test_batched_einsum_formulation_agrees(small_scene):
    """All pairs at once: padded row tensors, masked max, einsum products."""
    sc = small_scene
    w = _scene_weights()
    K = 64
    r = O.detect_scene(sc, w, WID, K=K)
    W1, b1, W2, b2, H1, c1, H2, c2, H3, c3 = O.unpack_weights(w, *WID)
    P = sc.n_pairs
    X = np.zeros((P, 2, K, 6))
    M = np.zeros((P, 2, K), bool)
    for p, g in enumerate(r["geoms"]):
        X[p, 0, :len(g.rows_a)] = g.rows_a
        X[p, 1, :len(g.rows_b)] = g.rows_b
        M[p, 0, :len(g.rows_a)] = True
        M[p, 1, :len(g.rows_b)] = True
    h1 = np.maximum(np.einsum("pskc,hc->pskh", X, W1) + b1, 0)
    h2 = np.maximum(np.einsum("pskh,oh->psko", h1, W2) + b2, 0)
    f = np.where(M[..., None], h2, -np.inf).max(axis=2)
    f = np.where(np.isfinite(f), f, 0.0).reshape(P, -1)
    np.testing.assert_allclose(f, r["z"], rtol=1e-13, atol=1e-13)
    g1 = np.maximum(np.einsum("pi,oi->po", f, H1) + c1, 0)
    g2 = np.maximum(np.einsum("pi,oi->po", g1, H2) + c2, 0)
    y = np.einsum("pi,oi->po", g2, H3) + c3
    np.testing.assert_allclose(y, r["y"], rtol=1e-12, atol=1e-12)


def test_empty_crop_pools_to_zero():
    rng = np.random.default_rng(9)
    lib = I.shape_library(rng, 2, 128, (3, 3), 0.0)
    pos = np.array([[0, 0, 0], [5, 0, 0]], np.float32)     # far apart: empty crop box
    quat = np.tile(np.float32([1, 0, 0, 0]), (2, 1))
    sc = I.Scene(lib, pos, quat, np.array([0, 1], np.int32), np.array([[0, 1]], np.int32))
    w = _scene_weights()
    r = O.detect_scene(sc, w, WID, K=64)
    assert list(r["counts"][0]) == [0, 0]
    np.testing.assert_array_equal(r["z"][0], 0.0)
    np.testing.assert_array_equal(r["idx"][0], -1)
    W = O.unpack_weights(w, *WID)
    np.testing.assert_allclose(r["y"][0], O.head(np.zeros(2 * SW.h2), *W[4:]), rtol=0, atol=0)


def test_invalid_pairs_give_nan_and_minus_one(small_scene):
    sc = small_scene
    bad = np.array([[0, 0], [-1, 3], [3, sc.n_objects], [1, 0]], np.int32)
    shape = sc.shape.copy()
    shape[5] = sc.lib.n_shapes           # shape id out of range
    bad = np.concatenate([bad, [[4, 5]]]).astype(np.int32)
    r = O.detect(sc.lib.pts, sc.lib.offsets, sc.pos, sc.quat, shape, bad, _scene_weights(), WID, K=64)
    for p in (0, 1, 2, 4):
        assert np.isnan(r["contacts"][p]).all() and list(r["counts"][p]) == [-1, -1]
    assert np.isfinite(r["contacts"][3]).all() and (r["counts"][3] >= 0).all()
