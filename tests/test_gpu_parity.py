"""GPU parity: the HIP path through the C-ABI against the CPU FP64 oracle.

Crop index sets and counts must match bit for bit; FP32 network outputs must
match within 1e-5 relative (per field, relative to max(|ref|, RMS |ref|)).
"""

import sys

import numpy as np
import pytest

from oracle import locc_oracle as O
from paper_2304_09439_amd import binding as B
from paper_2304_09439_amd import inputs as I

from helpers import (field_errors, flag_agreement, oracle_crop_all, sphere_case_scene, sphere_cases,
                     sphere_probe_weights)

pytestmark = pytest.mark.gpu

SW, LW = I.SMALL_WIDTHS, I.SCALE_WIDTHS
SMALL = (SW.h1, SW.h2, SW.hh)
SCALE = (LW.h1, LW.h2, LW.hh)
FP32_TOL = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    B.load()
    return t


@pytest.fixture(scope="module")
def scale_scene():
    return I.scale_workload()


def _weights(widths, bias=0.1):
    return I.flatten_weights(I.gaussian_weights(widths, seed=0, bias_std=bias))


def _run_crop(torch, scene, K, widths, pad=0.01):
    ctx = B.Context(K, widths, pad)
    ctx.upload_shapes(scene.lib.offsets, scene.lib.pts)
    objs, pairs = B.scene_tensors(scene)
    idx, counts = ctx.debug_crop(objs, pairs)
    torch.cuda.synchronize()
    ctx.close()
    return idx.cpu().numpy(), counts.cpu().numpy()


def _run_forward(torch, scene, K, widths, w, pad=0.01):
    ctx = B.context_for_scene(scene, K, widths, w, pad)
    objs, pairs = B.scene_tensors(scene)
    out, counts, z, y = ctx.debug_forward(objs, pairs)
    torch.cuda.synchronize()
    ctx.close()
    return out.cpu().numpy(), counts.cpu().numpy(), z.cpu().numpy(), y.cpu().numpy()


# --------------------------------------------------------------------- crop

def test_crop_matches_oracle_bit_exactly_small(torch, small_scene):
    say("crop parity: small workload, K=64")
    idx, counts = _run_crop(torch, small_scene, 64, SMALL)
    _, ridx, rcounts = O.crop(small_scene.lib.pts, small_scene.lib.offsets, small_scene.pos, small_scene.quat,
                              small_scene.shape, small_scene.pairs, 64)
    np.testing.assert_array_equal(counts, rcounts)
    np.testing.assert_array_equal(idx, ridx)


@pytest.mark.parametrize("K", [32, 64, 256])
def test_crop_matches_oracle_on_tiny_shapes_and_non_unit_quaternions(torch, K):
    rng = np.random.default_rng(77)
    lib = I.shape_library(rng, 12, 40, (3, 5), 0.5)
    n = 200
    sa, sb = rng.integers(0, 12, n), rng.integers(0, 12, n)
    ta, qa, tb, qb = I.overlapping_pair_poses(rng, lib, sa, sb)
    qa = (qa * rng.uniform(0.9, 1.1, (n, 1))).astype(np.float32)
    sc = I._pack_pair_scene(lib, ta, qa, tb, qb, sa.astype(np.int32), sb.astype(np.int32),
                            I._interleave_pairs(rng, n))
    say(f"crop parity: tiny shapes, K={K}")
    idx, counts = _run_crop(torch, sc, K, SMALL)
    _, ridx, rcounts = O.crop(sc.lib.pts, sc.lib.offsets, sc.pos, sc.quat, sc.shape, sc.pairs, K)
    np.testing.assert_array_equal(counts, rcounts)
    np.testing.assert_array_equal(idx, ridx)


@pytest.mark.parametrize("K", [32, 64])
def test_crop_matches_oracle_on_ragged_shape_sizes(torch, K):
    """Shape sizes that end inside a lane's group of four points and inside a
    256-point block, on both objects of a pair."""
    rng = np.random.default_rng(41)
    sizes = [1, 2, 3, 5, 6, 7, 63, 65, 255, 257, 258, 259, 513, 1023]
    half = rng.uniform(0.05, 0.3, (len(sizes), 3))
    pts = [np.concatenate([rng.uniform(-h, h, (m, 3)), rng.normal(size=(m, 3))], 1) for h, m in zip(half, sizes)]
    lib = I.ShapeLibrary(np.concatenate(pts).astype(np.float32), np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64),
                         np.full(len(sizes), np.nan, np.float32))
    n = 300
    sa, sb = rng.integers(0, len(sizes), n), rng.integers(0, len(sizes), n)
    ta, qa, tb, qb = I.overlapping_pair_poses(rng, lib, sa, sb)
    sc = I._pack_pair_scene(lib, ta, qa, tb, qb, sa.astype(np.int32), sb.astype(np.int32),
                            I._interleave_pairs(rng, n))
    say(f"crop parity: ragged shape sizes, K={K}")
    idx, counts = _run_crop(torch, sc, K, SMALL)
    _, ridx, rcounts = O.crop(sc.lib.pts, sc.lib.offsets, sc.pos, sc.quat, sc.shape, sc.pairs, K)
    assert (rcounts % 4 != 0).sum() > 50 and (rcounts > K).sum() > 20
    np.testing.assert_array_equal(counts, rcounts)
    np.testing.assert_array_equal(idx, ridx)


def test_points_on_box_faces_are_members_on_the_gpu(torch):
    import test_oracle_geometry as TG
    pa, pb = TG._on_face_shapes()
    lib = I.ShapeLibrary(np.concatenate([pa, pb]), np.array([0, len(pa), len(pa) + len(pb)], np.int64),
                         np.full(2, np.nan, np.float32))
    sc = I.Scene(lib, np.array([[0, 0, 0], [0.25, 0, 0]], np.float32), np.tile(np.float32([1, 0, 0, 0]), (2, 1)),
                 np.array([0, 1], np.int32), np.array([[0, 1], [1, 0]], np.int32))
    say("crop parity: dyadic on-face points, pad 1/32")
    idx, counts = _run_crop(torch, sc, 32, SMALL, pad=0.03125)
    assert list(counts[0]) == [2, 2] and list(counts[1]) == [2, 2]
    assert list(idx[0, 0, :3]) == [2, 4, -1] and list(idx[0, 1, :3]) == [1, 2, -1]
    np.testing.assert_array_equal(idx[1], idx[0][::-1])


def _near_face_scene(seed=5, n_pairs=32):
    """Pairs whose b points land within float32 rounding of the crop-box faces
    in a's frame, so that the b-side float32 screen leaves many of them to the
    exact float64 test.  b's stored box is set by 8 far corners (the crop box is
    then a's box widened by the pad) and b's frame origin lies up to 60 units
    away, which widens the screen's undecided band."""
    rng = np.random.default_rng(seed)
    half = rng.uniform(0.3, 1.5, 3)
    pts_a = np.concatenate([rng.uniform(-half, half, (64, 3)), rng.normal(size=(64, 3))], 1).astype(np.float32)
    lo_a, hi_a = O.aabb(pts_a)
    quat = rng.normal(size=(2 * n_pairs, 4)).astype(np.float32)
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    pos = np.empty((2 * n_pairs, 3), np.float32)
    pos[0::2] = rng.uniform(-20, 20, (n_pairs, 3))
    pos[1::2] = pos[0::2] + rng.uniform(-60, 60, (n_pairs, 3))
    shapes, offsets = [pts_a], [0, len(pts_a)]
    for p in range(n_pairs):
        Rab, tab = O.relative_pose(O.rotation(quat[2 * p]), pos[2 * p].astype(np.float64),
                                   O.rotation(quat[2 * p + 1]), pos[2 * p + 1].astype(np.float64))
        L = np.ceil(np.abs(tab).max()) + 4.0
        corners = np.array([[sx, sy, sz] for sx in (-L, L) for sy in (-L, L) for sz in (-L, L)])
        lo, hi = lo_a - O.PAD_M, hi_a + O.PAD_M
        q = rng.uniform(lo, hi, (248, 3))
        ax = rng.integers(0, 3, 248)
        side = rng.integers(0, 2, 248)
        q[np.arange(248), ax] = np.where(side == 1, hi[ax], lo[ax])
        q[:8] = np.array([[(lo, hi)[(c >> k) & 1][k] for k in range(3)] for c in range(8)])  # box corners
        pb = ((q - tab) @ Rab).astype(np.float32)  # Rab^T (q - tab), rounded
        xyz = np.concatenate([corners.astype(np.float32), pb])
        shapes.append(np.concatenate([xyz, rng.normal(size=(len(xyz), 3))], 1).astype(np.float32))
        offsets.append(offsets[-1] + len(xyz))
    lib = I.ShapeLibrary(np.concatenate(shapes), np.array(offsets, np.int64), np.full(len(shapes), np.nan, np.float32))
    shape = np.zeros(2 * n_pairs, np.int32)
    shape[1::2] = np.arange(1, n_pairs + 1)
    pairs = np.stack([np.arange(0, 2 * n_pairs, 2), np.arange(1, 2 * n_pairs, 2)], 1).astype(np.int32)
    return I.Scene(lib, pos, quat, shape, pairs)


def test_b_points_on_rotated_box_faces_match_oracle(torch):
    sc = _near_face_scene()
    say("crop parity: b points within rounding of rotated crop-box faces, K=256")
    idx, counts = _run_crop(torch, sc, 256, SMALL)
    _, ridx, rcounts = O.crop(sc.lib.pts, sc.lib.offsets, sc.pos, sc.quat, sc.shape, sc.pairs, 256)
    nb = rcounts[:, 1]
    assert nb.min() >= 8 and (nb < 256).all() and (nb > 8 + 40).all()  # near-face points fall on both sides
    np.testing.assert_array_equal(counts, rcounts)
    np.testing.assert_array_equal(idx, ridx)   # every b member, in order


def test_flat_and_separated_boxes_match_oracle(torch):
    """A zero-width crop box (coplanar flat shapes, no pad) takes every b point
    to the exact test; a pair whose boxes do not overlap has an empty box."""
    rng = np.random.default_rng(9)
    flat = np.concatenate([rng.uniform(-1, 1, (100, 2)), np.zeros((100, 1)), rng.normal(size=(100, 3))], 1)
    flat = flat.astype(np.float32)
    lib = I.ShapeLibrary(flat, np.array([0, 100], np.int64), np.full(1, np.nan, np.float32))
    pos = np.array([[0, 0, 0], [0.5, 0.25, 0], [0, 0, 0], [40, 0, 0]], np.float32)
    quat = np.tile(np.float32([1, 0, 0, 0]), (4, 1))
    sc = I.Scene(lib, pos, quat, np.zeros(4, np.int32), np.array([[0, 1], [2, 3]], np.int32))
    say("crop parity: coplanar flat shapes with pad 0, and a separated pair")
    idx, counts = _run_crop(torch, sc, 128, SMALL, pad=0.0)
    _, ridx, rcounts = O.crop(sc.lib.pts, sc.lib.offsets, sc.pos, sc.quat, sc.shape, sc.pairs, 128, pad=0.0)
    assert rcounts[0, 1] > 20 and list(rcounts[1]) == [0, 0]
    np.testing.assert_array_equal(counts, rcounts)
    np.testing.assert_array_equal(idx, ridx)


# ------------------------------------------------------------------ forward

@pytest.mark.parametrize("bias", [0.0, 0.1])
def test_fp32_forward_matches_oracle_small(torch, small_scene, bias):
    w = _weights(SW, bias)
    say(f"forward parity: small workload, fp32, bias_std={bias}")
    out, counts, z, y = _run_forward(torch, small_scene, 64, SMALL, w)
    ref = O.detect_scene(small_scene, w, SMALL, 64)
    np.testing.assert_array_equal(counts, ref["counts"])
    zs = np.abs(ref["z"]).max()
    assert np.max(np.abs(z - ref["z"])) <= FP32_TOL * zs
    ey = field_errors(y, ref["y"])
    ec = field_errors(out, ref["contacts"])
    say(f"  raw y errors {ey}\n  world errors {ec}")
    assert max(ey.values()) < FP32_TOL and max(ec.values()) < FP32_TOL
    assert flag_agreement(out[:, 0], ref["contacts"][:, 0]) == 1.0


def test_constructed_weights_give_closed_form_sphere_contact_on_the_gpu(torch):
    cases = sphere_cases()
    sc = sphere_case_scene(cases)
    say("forward: constructed sphere weights")
    out, counts, _, _ = _run_forward(torch, sc, 64, SMALL, sphere_probe_weights(SW, beta=4.0))
    for k, c in enumerate(cases):
        swapped = sc.pairs[k, 0] > sc.pairs[k, 1]
        assert out[k, 7] == pytest.approx(c["depth"], abs=2e-7)
        assert out[k, 1] == pytest.approx(c["point_x"], abs=2e-7)
        assert out[k, 2] == 0 and out[k, 3] == 0
        np.testing.assert_array_equal(out[k, 4:7], [-1.0, 0, 0] if swapped else [1.0, 0, 0])
        assert (out[k, 0] > 0) == c["flag"] or abs(c["depth"]) < 1e-7


def test_swapping_pairs_negates_only_the_normal_on_the_gpu(torch, small_scene):
    w = _weights(SW)
    say("forward: swap invariance")
    ctx = B.context_for_scene(small_scene, 64, SMALL, w)
    objs, pairs = B.scene_tensors(small_scene)
    o1, c1 = ctx.detect(objs, pairs)
    o2, c2 = ctx.detect(objs, pairs.flip(1).contiguous())
    torch.cuda.synchronize()
    o1, o2, c1, c2 = o1.cpu().numpy(), o2.cpu().numpy(), c1.cpu().numpy(), c2.cpu().numpy()
    np.testing.assert_array_equal(o1[:, [0, 1, 2, 3, 7]], o2[:, [0, 1, 2, 3, 7]])
    np.testing.assert_array_equal(o1[:, 4:7], -o2[:, 4:7])
    np.testing.assert_array_equal(c1, c2[:, ::-1])
    ctx.close()


def test_invalid_pairs_give_nan_and_count_as_device_errors(torch, small_scene):
    w = _weights(SW)
    bad = np.array([[0, 0], [-1, 3], [3, small_scene.n_objects], [1, 0], [2, 3]], np.int32)
    say("forward: invalid pairs")
    ctx = B.context_for_scene(small_scene, 64, SMALL, w)
    objs, _ = B.scene_tensors(small_scene)
    pairs = torch.from_numpy(bad).cuda()
    assert ctx.device_errors(reset=True) == 0
    out, counts = ctx.detect(objs, pairs)
    n_bad = ctx.device_errors()
    out, counts = out.cpu().numpy(), counts.cpu().numpy()
    assert n_bad == 3
    for p in range(3):
        assert np.isnan(out[p]).all() and list(counts[p]) == [-1, -1]
    assert np.isfinite(out[3:]).all() and (counts[3:] >= 0).all()
    ctx.close()


@pytest.mark.parametrize("n", [0, 1, 31, 33])
def test_empty_and_ragged_batches(torch, small_scene, n):
    w = _weights(SW)
    sub = small_scene.subset(np.arange(n))
    say(f"forward: ragged batch of {n} pairs")
    ctx = B.context_for_scene(sub, 64, SMALL, w)
    objs, pairs = B.scene_tensors(sub)
    out, counts = ctx.detect(objs, pairs)
    torch.cuda.synchronize()
    assert out.shape == (n, 8)
    if n:
        ref = O.detect_scene(sub, w, SMALL, 64)
        np.testing.assert_array_equal(counts.cpu().numpy(), ref["counts"])
        assert max(field_errors(out.cpu().numpy(), ref["contacts"]).values()) < FP32_TOL
    ctx.close()


def test_uploads_validate_and_detect_needs_them(torch):
    ctx = B.Context(64, SMALL)
    objs = torch.zeros((2, 8), dtype=torch.float32, device="cuda")
    pairs = torch.zeros((1, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(B.LoccError) as e:
        ctx.detect(objs, pairs)
    assert e.value.status == B.ERR_NOT_READY
    with pytest.raises(B.LoccError) as e:
        ctx.upload_shapes(np.array([0, 4, 4], np.int64), np.zeros((4, 6), np.float32))   # empty shape
    assert e.value.status == B.ERR_INVALID_ARG
    with pytest.raises(B.LoccError) as e:
        ctx.upload_shapes(np.array([1, 4], np.int64), np.zeros((4, 6), np.float32))      # offsets[0] != 0
    assert e.value.status == B.ERR_INVALID_ARG
    pts = np.zeros((4, 6), np.float32)
    pts[2, 1] = np.nan
    with pytest.raises(B.LoccError) as e:
        ctx.upload_shapes(np.array([0, 4], np.int64), pts)
    assert e.value.status == B.ERR_INVALID_ARG
    with pytest.raises(B.LoccError) as e:
        ctx.upload_weights(np.zeros(10, np.float32))
    assert e.value.status == B.ERR_INVALID_ARG
    with pytest.raises(B.LoccError) as e:
        ctx.upload_shapes(np.array([0, 20000], np.int64), np.zeros((20000, 6), np.float32))
    assert e.value.status == B.ERR_RANGE
    ctx.close()


# -------------------------------------------------------------------- scale

def test_fp32_at_scale_matches_oracle_on_sampled_pairs(torch, scale_scene):
    """16,384 pairs, N=2048, K=128, widths 128/256/512, same launch as the
    benchmark; the oracle checks a seeded sample of 192 pairs."""
    sc = scale_scene
    w = _weights(LW, bias=0.0)
    say("scale parity: 16384 pairs fp32")
    ctx = B.context_for_scene(sc, 128, SCALE, w)
    objs, pairs = B.scene_tensors(sc)
    out, counts = ctx.detect(objs, pairs)
    idx, counts2 = ctx.debug_crop(objs, pairs)
    out2, _ = ctx.detect(objs, pairs)
    torch.cuda.synchronize()
    out, counts, idx, out2 = out.cpu().numpy(), counts.cpu().numpy(), idx.cpu().numpy(), out2.cpu().numpy()
    ctx.close()
    np.testing.assert_array_equal(out, out2)            # deterministic
    np.testing.assert_array_equal(counts, counts2.cpu().numpy())
    rows = np.sort(np.random.default_rng(123).choice(sc.n_pairs, 192, replace=False))
    ref = O.detect_scene(sc, w, SCALE, 128, rows=rows)
    np.testing.assert_array_equal(counts[rows], ref["counts"])
    np.testing.assert_array_equal(idx[rows], ref["idx"])
    e = field_errors(out[rows], ref["contacts"])
    say(f"  world errors {e}")
    assert max(e.values()) < FP32_TOL
    assert flag_agreement(out[rows, 0], ref["contacts"][:, 0], band=1e-3) >= 0.999


def test_crop_matches_oracle_on_every_pair_at_scale(torch, scale_scene):
    """Every one of the 16,384 pairs: index sets and member counts of the crop (the oracle's O1-O7, run
    over worker processes without the network) bit for bit."""
    sc = scale_scene
    say("scale crop: 16384 pairs, every pair against the oracle")
    idx, counts = _run_crop(torch, sc, 128, SCALE)
    ridx, rcounts = oracle_crop_all(sc, 128, workers=8)
    np.testing.assert_array_equal(counts, rcounts)
    np.testing.assert_array_equal(idx, ridx)
    say(f"  objects with more than K members {np.mean(rcounts > 128):.3f}, empty {np.mean(rcounts == 0):.3f}")
