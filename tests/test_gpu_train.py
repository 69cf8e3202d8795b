"""GPU training step (locc_train_step, FP32 contexts) against the float64
oracle of oracle.train, on labelled sphere pairs placed by distance
manipulation.

Branches are float32 decisions on the GPU: argmax rows within the float32
error of each other are both correct, so the kernel's rows (returned by the
parity hook) are checked to attain the float64 maxima within 1e-5 of the
layer's scale and the oracle differentiates with them; the batch is made of
pairs whose float64 ReLU decisions (layer-1 pre-activations at argmax rows:
margin 1e-6; pooled maxima plus bias, head pre-activations: 1e-5) are not
within their float32 error of zero.  Gradients then agree per weight array
normwise within 1e-4 (float32 sums of up to 512 terms and a batch sum of 96
pairs); the untrained outputs get exactly zero.  Adam (float32) moves every
weight whose gradient is clearly non-zero as the float64 step does within
1e-4 relative (plus two float32 spacings of the weights), and no weight by
more than lr.  Fitting: held-out accuracy
rises above 0.8."""

import sys

import numpy as np
import pytest

from oracle import locc_oracle as O
from oracle import train as T
from paper_2304_09439_amd import binding as B
from paper_2304_09439_amd import inputs as I

pytestmark = pytest.mark.gpu

W = I.Widths(64, 128, 256)
WIDTHS = (W.h1, W.h2, W.hh)
K = 64
PRE_MARGIN, SUM_MARGIN = 1e-6, 1e-5
NAMES = ("W1", "b1", "W2", "b2", "H1", "c1", "H2", "c2", "H3", "c3")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    B.load()
    return t


def _weights(seed=0):
    return I.flatten_weights(I.gaussian_weights(W, seed=seed, bias_std=0.1))


def _near_kink(g, wts):
    """A float64 ReLU decision of the pair within its float32 error of zero (both objects)."""
    W1, b1, W2, b2, H1, c1, H2, c2, H3, c3 = wts
    z = []
    for rows in (g.rows_a, g.rows_b):
        rows = np.asarray(rows, np.float64).reshape(-1, 6)
        if len(rows) == 0:
            z.append(np.zeros(W.h2))
            continue
        pre = rows @ W1.T + b1
        s = O.relu(pre) @ W2.T
        m = s.max(axis=0)
        z.append(O.relu(m + b2))
        if np.min(np.abs(m + b2)) < SUM_MARGIN * np.abs(s).max():
            return True
        if np.min(np.abs(pre[np.argmax(s, axis=0)])) < PRE_MARGIN * np.abs(pre).max():
            return True
    u1 = np.concatenate(z) @ H1.T + c1
    u2 = O.relu(u1) @ H2.T + c2
    return (np.min(np.abs(u1)) < SUM_MARGIN * np.abs(u1).max()
            or np.min(np.abs(u2)) < SUM_MARGIN * np.abs(u2).max())


def _check_argmax(g, wts, arg):
    W1, b1, W2 = wts[0], wts[1], wts[2]
    for side, rows in enumerate((g.rows_a, g.rows_b)):
        rows = np.asarray(rows, np.float64).reshape(-1, 6)
        if len(rows) == 0:
            continue
        s = O.relu(rows @ W1.T + b1) @ W2.T
        r = arg[side].astype(np.int64)
        assert np.all(r < len(rows))
        assert np.all(s[r, np.arange(W.h2)] >= s.max(axis=0) - SUM_MARGIN * np.abs(s).max())


@pytest.fixture(scope="module")
def batch():
    sc, y = I.sphere_training_set(n_pairs=400)
    w = _weights()
    wts = O.unpack_weights(w, *WIDTHS)
    geoms, _, _ = O.crop(sc.lib.pts, sc.lib.offsets, sc.pos, sc.quat, sc.shape, sc.pairs, K)
    rows = [p for p, g in enumerate(geoms) if not _near_kink(g, wts)][:96]
    assert len(rows) == 96
    return sc.subset(rows), y[rows], [geoms[p] for p in rows], w


def test_one_step_matches_the_oracle(torch, batch):
    sc, y, geoms, w = batch
    ctx = B.context_for_scene(sc, K, WIDTHS, w, precision="fp32")
    objs, pairs = B.scene_tensors(sc)
    loss, arg = ctx.train_step(objs, pairs, torch.from_numpy(y).cuda(), want_argmax=True)
    torch.cuda.synchronize()
    loss, arg = loss.cpu().numpy(), arg.cpu().numpy()
    grad = ctx.get_weights(1)
    w_after = ctx.get_weights(0)
    wts = O.unpack_weights(w, *WIDTHS)
    for p, g in enumerate(geoms):
        _check_argmax(g, wts, arg[p])
    bce, reg, grads, _ = T.loss_and_grads(geoms, y, [a.copy() for a in wts], T.ALPHA, argmax=arg)
    say(f"train step: loss {loss} vs oracle {bce:.6f} {reg:.6f}")
    assert loss[0] == pytest.approx(bce, rel=1e-5) and loss[1] == pytest.approx(reg, rel=1e-5)
    g_gpu = O.unpack_weights(grad, *WIDTHS)
    errs = {}
    for name, a, b in zip(NAMES, g_gpu, grads):
        if name in ("H3", "c3"):
            assert not np.any(a[1:]) and not np.any(b[1:])
            a, b = a[:1], b[:1]
        errs[name] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    say("  gradient normwise errors " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))
    assert max(errs.values()) < 1e-4
    # Adam: the float64 step from the float32 weights with the oracle's gradient
    ref = [a.copy() for a in wts]
    T.adam_step(ref, grads, {})
    lr = T.ADAM["lr"]
    moved = O.unpack_weights(w_after, *WIDTHS)
    for name, a_after, a_ref, a0, g in zip(NAMES, moved, ref, wts, grads):
        d_gpu, d_ref = a_after - a0, a_ref - a0
        clear = np.abs(g) > 1e-3 * max(np.abs(g).max(), 1e-30)
        ulp = float(np.spacing(np.float32(np.abs(a0).max())))   # the new weights are rounded to float32
        np.testing.assert_allclose(d_gpu[clear], d_ref[clear], rtol=1e-4, atol=2 * ulp, err_msg=name)
        assert np.all(np.abs(d_gpu) <= lr * 1.0001), name
    ctx.close()


def test_steps_are_reproducible(torch, batch):
    sc, y, _, w = batch
    objs, pairs = B.scene_tensors(sc)
    lab = torch.from_numpy(y).cuda()
    out = []
    for _ in range(2):
        ctx = B.context_for_scene(sc, K, WIDTHS, w, precision="fp32")
        for _ in range(3):
            ctx.train_step(objs, pairs, lab)
        out.append(ctx.get_weights(0))
        ctx.close()
    np.testing.assert_array_equal(out[0], out[1])


def test_fitting_raises_held_out_accuracy(torch):
    full, yy = I.sphere_training_set(n_pairs=5120)
    sc, y = full.subset(np.arange(4096)), yy[:4096]        # training pairs
    hsc, hy = full.subset(np.arange(4096, 5120)), yy[4096:]  # held out
    ctx = B.context_for_scene(sc, K, WIDTHS, _weights(seed=1), precision="fp32")
    objs, pairs = B.scene_tensors(sc)
    hobjs, hpairs = B.scene_tensors(hsc)
    lab = torch.from_numpy(y).cuda()

    def accuracy():
        out, _ = ctx.detect(hobjs, hpairs)
        torch.cuda.synchronize()
        return float(np.mean((out[:, 0].cpu().numpy() > 0) == (hy > 0.5)))

    acc0 = accuracy()
    rng = np.random.default_rng(0)
    losses = []
    for step in range(200):
        rows = torch.from_numpy(np.sort(rng.choice(4096, 512, replace=False))).cuda()
        loss = ctx.train_step(objs, pairs[rows].contiguous(), lab[rows].contiguous())
        if step % 50 == 0 or step == 199:
            losses.append(loss.cpu().numpy().tolist())
    acc1 = accuracy()
    say(f"fitting: held-out accuracy {acc0:.3f} -> {acc1:.3f}; loss (cross-entropy, feature term) {losses}")
    assert acc1 > 0.8 and acc1 > acc0 + 0.1
    assert ctx.device_errors() == 0
    ctx.close()


def test_argument_errors(torch, batch):
    sc, y, _, w = batch
    objs, pairs = B.scene_tensors(sc)
    lab = torch.from_numpy(y).cuda()
    ctx = B.context_for_scene(sc, K, WIDTHS, w, precision="fp32")
    with pytest.raises(B.LoccError):
        ctx.train_step(objs, pairs, lab, lr=0.0)
    with pytest.raises(B.LoccError):
        ctx.train_step(objs, pairs, lab, beta1=1.0)
    with pytest.raises(B.LoccError):
        ctx.get_weights(1)                                 # no step yet
    ctx.close()
    ctx = B.context_for_scene(sc, K, WIDTHS, w, precision="bf16")
    with pytest.raises(B.LoccError):
        ctx.train_step(objs, pairs, lab)
    ctx.close()
