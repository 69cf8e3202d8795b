"""GPU pose gradients (locc_pose_gradients, FP32 contexts) against the float64
oracle of oracle.pose_grad.

The gradient is piecewise smooth: it jumps where an argmax row of the second
object changes or a ReLU changes sign, and the kernel takes those decisions
in float32.  Argmax rows: where two raw sums of a channel lie within the
float32 error of each other either row is a correct argmax, so the kernel's
rows (returned by the parity hook) are checked to attain the float64 maximum
within 1e-5 of the layer's largest magnitude (sums of 128 products), and the
oracle then differentiates with those rows.  ReLU decisions: a pair whose
float64 pre-activation at an argmax row (6 terms and a bias on rows rounded
to float32: margin 1e-6), pooled maximum plus bias or head pre-activation
(sums of up to 512 terms: margin 1e-5) is that close to zero may take the
other branch and is counted and left out.  The rest must agree normwise
within 1e-4 overall and 1e-3 per pair (float32 arithmetic through the same
chain).
Swapping a pair reorders its gradient exactly; a pair whose crops select
nothing has zero gradient; invalid pairs give NaN."""

import sys

import numpy as np
import pytest

from oracle import locc_oracle as O
from oracle import pose_grad as PG
from paper_2304_09439_amd import binding as B
from paper_2304_09439_amd import inputs as I

from helpers import normwise_errors

pytestmark = pytest.mark.gpu

LW = I.SCALE_WIDTHS
WIDTHS = (LW.h1, LW.h2, LW.hh)
K = 128
PRE_MARGIN = 1e-6
SUM_MARGIN = 1e-5


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
def setup():
    sc = I.scale_workload(n_pairs=600)
    w = I.flatten_weights(I.gaussian_weights(LW, seed=0, bias_std=0.1))
    return sc, w


def _check_argmax_and_relu(g, wts, h2, arg_gpu):
    """Asserts the kernel's argmax rows of the second object attain the float64 maxima within the
    margin; returns True when a ReLU decision the gradient depends on is within its margin of zero."""
    W1, b1, W2, b2, H1, c1, H2, c2, H3, c3 = wts
    z = []
    near = False
    for side, rows in enumerate((g.rows_a, g.rows_b)):
        rows = np.asarray(rows, np.float64).reshape(-1, 6)
        if len(rows) == 0:
            z.append(np.zeros(h2))
            if side == 1:
                assert np.all(arg_gpu == 255)
            continue
        pre = rows @ W1.T + b1
        s = O.relu(pre) @ W2.T
        m = s.max(axis=0)
        z.append(O.relu(m + b2))
        if side == 0:
            continue
        scale = np.abs(s).max()
        r = arg_gpu.astype(np.int64)
        assert np.all(r < len(rows))
        assert np.all(s[r, np.arange(h2)] >= m - SUM_MARGIN * scale)
        near |= bool(np.min(np.abs(m + b2)) < SUM_MARGIN * scale)
        near |= bool(np.min(np.abs(pre[r])) < PRE_MARGIN * np.abs(pre).max())
    u1 = np.concatenate(z) @ H1.T + c1
    u2 = O.relu(u1) @ H2.T + c2
    near |= bool(np.min(np.abs(u1)) < SUM_MARGIN * np.abs(u1).max())
    near |= bool(np.min(np.abs(u2)) < SUM_MARGIN * np.abs(u2).max())
    return near


def test_gradients_match_the_oracle(torch, setup):
    sc, w = setup
    rows = np.arange(0, 600, 3)
    pairs = sc.pairs[rows].copy()
    pairs[7] = [5, 5]                     # invalid
    ctx = B.context_for_scene(sc, K, WIDTHS, w, precision="fp32")
    objs = torch.from_numpy(B.pack_objects(sc.pos, sc.quat, sc.shape)).cuda()
    pr = torch.from_numpy(pairs).cuda()
    grad, out, arg = ctx.pose_gradients(objs, pr, want_contacts=True, want_argmax=True)
    ref_out, _ = ctx.detect(objs, pr)
    torch.cuda.synchronize()
    assert torch.equal(out.isnan(), ref_out.isnan()) and torch.equal(out[~out.isnan()], ref_out[~ref_out.isnan()])
    grad, arg = grad.cpu().numpy(), arg.cpu().numpy()
    ref = PG.pose_gradients(sc.lib.pts, sc.lib.offsets, sc.pos, sc.quat, sc.shape, pairs, w, WIDTHS, K,
                            argmax_b=arg)
    wts = O.unpack_weights(w, *WIDTHS)
    assert np.all(arg[7] == 255)
    assert np.isnan(grad[7]).all() and np.isnan(ref["grad"][7]).all()
    keep, amb, zero = [], 0, 0
    for p, g in enumerate(ref["geoms"]):
        if g is None:
            continue
        if _check_argmax_and_relu(g, wts, LW.h2, arg[p]):
            amb += 1
            continue
        if not np.any(ref["grad"][p]):
            zero += 1
            assert not np.any(grad[p]), p
            continue
        keep.append(p)
    keep = np.array(keep)
    e_pair = np.linalg.norm(grad[keep] - ref["grad"][keep], axis=1) / np.linalg.norm(ref["grad"][keep], axis=1)
    e_all = np.linalg.norm(grad[keep] - ref["grad"][keep]) / np.linalg.norm(ref["grad"][keep])
    ties = sum(int(np.any(arg[p] != ref["first_argmax_b"][p])) for p in keep) if len(keep) else 0
    say(f"pose gradients: {len(keep)} pairs compared ({ties} with an argmax tie taken the other way), "
        f"{amb} near a ReLU kink, {zero} with zero gradient; "
        f"normwise {e_all:.2e}, worst pair {e_pair.max():.2e}")
    assert len(keep) > 0.6 * len(pairs)
    assert e_all < 1e-4 and e_pair.max() < 1e-3
    ctx.close()


def test_swapped_and_empty_pairs(torch, setup):
    sc, w = setup
    ref = PG.pose_gradients(sc.lib.pts, sc.lib.offsets, sc.pos, sc.quat, sc.shape, sc.pairs[:20], w, WIDTHS, K)
    q = int(np.flatnonzero(np.any(ref["grad"] != 0, axis=1))[0])   # a pair with a non-zero gradient
    i, j = (int(v) for v in sc.pairs[q])
    k, l = (int(v) for v in sc.pairs[q + 1])
    pos = sc.pos.copy()
    pos[l] = pos[k] + np.float32([3.0, 0.0, 0.0])   # far apart: nothing selected
    pairs = np.array([[i, j], [j, i], [k, l], [l, k]], np.int32)
    ctx = B.context_for_scene(sc, K, WIDTHS, w, precision="fp32")
    objs = torch.from_numpy(B.pack_objects(pos, sc.quat, sc.shape)).cuda()
    grad, _ = ctx.pose_gradients(objs, torch.from_numpy(pairs).cuda())
    torch.cuda.synchronize()
    g = grad.cpu().numpy()
    np.testing.assert_array_equal(g[1], np.concatenate([g[0][7:], g[0][:7]]))
    assert np.any(g[0]) and not np.any(g[2]) and not np.any(g[3])
    ctx.close()


# BF16 contexts: the encoder's raw sums come from bf16 rows, weights and layer-1 outputs with float32
# accumulation, a relative error of a few 2^-8 of the layer's magnitude, so an argmax row must attain the
# float64 maximum within 1e-2 of that magnitude.  The gradient then differs from the float64 one, taken at the
# same argmax rows, by more than the pooled features' bf16 error: every pooled feature whose pre-activation
# lies within that error of zero may take the other ReLU branch, which adds or drops that channel's whole
# term.  With 2 x 256 channels per pair nearly every pair has such a channel (on this workload all but one
# of 155 pairs at 1e-3 of the scale), so no pair can be left out as in the FP32 test.  The bars are the
# measured size of that effect with room: normwise 0.1 over the pairs (measured 0.058) and a median per-pair
# error of 3e-2 (measured 0.015); the contacts of this path (an FP32 head on the BF16 pooled features) meet
# the BF16 bar of 2e-2.
BF16_ARG_MARGIN = 1e-2
BF16_TOL = 2e-2
BF16_GRAD_TOL = 1e-1
BF16_GRAD_MEDIAN_TOL = 3e-2


def _bf16_margins(g, wts, h2, arg_gpu):
    """Asserts the kernel's argmax rows of the second object attain the float64 maxima within the BF16
    margin; returns (smallest |pooled pre-activation| / scale over both objects, smallest |head
    pre-activation| / scale)."""
    W1, b1, W2, b2, H1, c1, H2, c2, H3, c3 = wts
    z, zmin = [], np.inf
    for side, rows in enumerate((g.rows_a, g.rows_b)):
        rows = np.asarray(rows, np.float64).reshape(-1, 6)
        if len(rows) == 0:
            z.append(np.zeros(h2))
            if side == 1:
                assert np.all(arg_gpu == 255)
            continue
        pre = rows @ W1.T + b1
        s = O.relu(pre) @ W2.T
        m = s.max(axis=0)
        z.append(O.relu(m + b2))
        scale = np.abs(s).max()
        zmin = min(zmin, float(np.min(np.abs(m + b2)) / scale))
        if side == 1:
            r = arg_gpu.astype(np.int64)
            assert np.all(r < len(rows))
            assert np.all(s[r, np.arange(h2)] >= m - BF16_ARG_MARGIN * scale)
    u1 = np.concatenate(z) @ H1.T + c1
    u2 = O.relu(u1) @ H2.T + c2
    umin = min(float(np.min(np.abs(u1)) / np.abs(u1).max()), float(np.min(np.abs(u2)) / np.abs(u2).max()))
    return zmin, umin


def test_bf16_gradients_match_the_oracle(torch, setup):
    """A BF16 context: its split-schedule encoder records the argmax rows; the gradient kernels are the FP32
    path's.  Checked against the float64 oracle at the kernel's argmax rows."""
    sc, w = setup
    rows = np.arange(0, 600, 3)
    pairs = sc.pairs[rows].copy()
    pairs[7] = [5, 5]                     # invalid
    ctx = B.context_for_scene(sc, K, WIDTHS, w, precision="bf16")
    objs = torch.from_numpy(B.pack_objects(sc.pos, sc.quat, sc.shape)).cuda()
    pr = torch.from_numpy(pairs).cuda()
    grad, out, arg = ctx.pose_gradients(objs, pr, want_contacts=True, want_argmax=True)
    torch.cuda.synchronize()
    grad, arg, out = grad.cpu().numpy(), arg.cpu().numpy(), out.cpu().numpy()
    ref = PG.pose_gradients(sc.lib.pts, sc.lib.offsets, sc.pos, sc.quat, sc.shape, pairs, w, WIDTHS, K,
                            argmax_b=arg)
    wts = O.unpack_weights(w, *WIDTHS)
    assert np.all(arg[7] == 255)
    assert np.isnan(grad[7]).all() and np.isnan(ref["grad"][7]).all() and np.isnan(out[7]).all()
    # contacts (the FP32 head on the BF16 encoder's pooled features) against the oracle's
    scene = I.Scene(sc.lib, sc.pos, sc.quat, sc.shape, pairs)
    ref_c = O.detect_scene(scene, w, WIDTHS, K)["contacts"]
    ok = ~np.isnan(ref_c[:, 0])
    ec = normwise_errors(out[ok], ref_c[ok])
    say(f"BF16 pose path contacts vs oracle normwise {ec}")
    assert max(ec.values()) < BF16_TOL
    valid, zm, um = [], [], []
    for p, g in enumerate(ref["geoms"]):
        if g is None or not np.any(ref["grad"][p]):
            continue
        a, b = _bf16_margins(g, wts, LW.h2, arg[p])
        valid.append(p)
        zm.append(a)
        um.append(b)
    valid, zm, um = np.array(valid), np.array(zm), np.array(um)
    err = np.linalg.norm(grad[valid] - ref["grad"][valid], axis=1) / np.linalg.norm(ref["grad"][valid], axis=1)
    e_all = np.linalg.norm(grad[valid] - ref["grad"][valid]) / np.linalg.norm(ref["grad"][valid])
    say(f"BF16 pose gradients on {len(valid)} pairs: normwise {e_all:.2e}; per pair median {np.median(err):.2e}, "
        f"90% {np.percentile(err, 90):.2e}, max {err.max():.2e}")
    k = (zm > 1e-3) & (um > 1e-3)
    say(f"  {int(k.sum())} of {len(valid)} pairs have every pooled and head pre-activation beyond 1e-3 of the "
        f"scale from zero")
    assert len(valid) > 0.5 * len(pairs)
    assert e_all < BF16_GRAD_TOL and np.median(err) < BF16_GRAD_MEDIAN_TOL
    ctx.close()


def test_bf16_swapped_pair_reorders_the_gradient(torch, setup):
    sc, w = setup
    pairs = np.array([sc.pairs[0], sc.pairs[0][::-1], sc.pairs[1], sc.pairs[1][::-1]], np.int32)
    ctx = B.context_for_scene(sc, K, WIDTHS, w, precision="bf16")
    objs = torch.from_numpy(B.pack_objects(sc.pos, sc.quat, sc.shape)).cuda()
    for sched in (dict(wg_per_cu=2, claim=4, dynamic=True), dict(wg_per_cu=1, claim=16, dynamic=False)):
        ctx.set_schedule(**sched)
        grad, _ = ctx.pose_gradients(objs, torch.from_numpy(pairs).cuda())
        torch.cuda.synchronize()
        g = grad.cpu().numpy()
        np.testing.assert_array_equal(g[1], np.concatenate([g[0][7:], g[0][:7]]))
        np.testing.assert_array_equal(g[3], np.concatenate([g[2][7:], g[2][:7]]))
    ctx.close()


def test_bf16_gradients_do_not_depend_on_the_encoder_kernel(torch, setup):
    """The argmax encoder of either split-schedule kernel (W2 slices in registers, two workgroups per CU; W2 in
    LDS, one workgroup of eight waves per CU): the same argmax rows, contacts and gradients, bit for bit."""
    sc, w = setup
    pairs = torch.from_numpy(sc.pairs[:700].copy()).cuda()
    ctx = B.context_for_scene(sc, K, WIDTHS, w, precision="bf16")
    objs = torch.from_numpy(B.pack_objects(sc.pos, sc.quat, sc.shape)).cuda()
    res = []
    for wg in (2, 1):
        ctx.set_schedule(wg_per_cu=wg, claim=16, dynamic=False, split=True)
        grad, out, arg = ctx.pose_gradients(objs, pairs, want_contacts=True, want_argmax=True)
        torch.cuda.synchronize()
        res.append([t.cpu().numpy() for t in (grad, out, arg)])
    for x, y in zip(*res):
        np.testing.assert_array_equal(x, y)
    ctx.close()


def test_unsupported_precision(torch, setup):
    sc, w = setup
    ctx = B.context_for_scene(sc, K, WIDTHS, w, precision="fp8")
    objs = torch.from_numpy(B.pack_objects(sc.pos, sc.quat, sc.shape)).cuda()
    with pytest.raises(B.LoccError):
        ctx.pose_gradients(objs, torch.from_numpy(sc.pairs[:4]).cuda())
    ctx.close()
