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


def test_unsupported_precision(torch, setup):
    sc, w = setup
    ctx = B.context_for_scene(sc, K, WIDTHS, w, precision="bf16")
    objs = torch.from_numpy(B.pack_objects(sc.pos, sc.quat, sc.shape)).cuda()
    with pytest.raises(B.LoccError):
        ctx.pose_gradients(objs, torch.from_numpy(sc.pairs[:4]).cuda())
    ctx.close()
