"""Pins of the training-step oracle (oracle.train): central finite differences
of the loss written independently (the pinned O9-O10 forward, cross-entropy
in its log-sigmoid form, the squared norm of the pooled features) for entries
of every weight array, wherever no argmax or ReLU pattern changes across the
step; Adam against torch.optim.Adam (float64, the paper's hyperparameters)."""

import numpy as np
import pytest
import torch

from oracle import locc_oracle as O
from oracle import train as T
from paper_2304_09439_amd import inputs as I

W = I.Widths(64, 128, 256)
WIDTHS = (W.h1, W.h2, W.hh)
K = 64


@pytest.fixture(scope="module")
def batch():
    sc, y = I.sphere_training_set(n_pairs=12)
    geoms, _, _ = O.crop(sc.lib.pts, sc.lib.offsets, sc.pos, sc.quat, sc.shape, sc.pairs, K)
    return geoms, y


def _weights(seed=0):
    return [a.copy() for a in O.unpack_weights(I.flatten_weights(I.gaussian_weights(W, seed=seed, bias_std=0.1)),
                                               *WIDTHS)]


def _loss(geoms, y, w, alpha):
    """Independent loss: mean of -y log s(x) - (1 - y) log(1 - s(x)) plus alpha mean ||z||^2, and a
    signature of the piecewise-smooth region (argmax rows, every ReLU pattern)."""
    W1, b1, W2, b2, H1, c1, H2, c2, H3, c3 = w
    tot, sig = 0.0, []
    for g, lab in zip(geoms, y):
        z = np.concatenate([O.encode(g.rows_a, W1, b1, W2, b2), O.encode(g.rows_b, W1, b1, W2, b2)])
        x = O.head(z, H1, c1, H2, c2, H3, c3)[0]
        ls = -np.logaddexp(0.0, -x)                    # log sigmoid(x)
        l1s = -np.logaddexp(0.0, x)                    # log (1 - sigmoid(x))
        tot += -(lab * ls + (1 - lab) * l1s) + alpha * float(z @ z)
        for rows in (g.rows_a, g.rows_b):
            rows = np.asarray(rows).reshape(-1, 6)
            if len(rows):
                pre = rows @ W1.T + b1
                s = O.relu(pre) @ W2.T
                sig += [np.argmax(s, 0).tobytes(), (pre > 0).tobytes(), (s.max(0) + b2 > 0).tobytes()]
        u1 = z @ H1.T + c1
        sig += [(u1 > 0).tobytes(), ((O.relu(u1) @ H2.T + c2) > 0).tobytes()]
    return tot / len(geoms), tuple(sig)


def test_gradients_match_central_differences(batch):
    geoms, y = batch
    w = _weights()
    alpha = 0.5
    bce, reg, grads, _ = T.loss_and_grads(geoms, y, w, alpha)
    base, sig = _loss(geoms, y, w, alpha)
    assert base == pytest.approx(bce + reg, rel=1e-12)
    rng = np.random.default_rng(3)
    h = 1e-6
    checked = 0
    for a in range(10):
        for _ in range(4):
            i = tuple(rng.integers(0, n) for n in w[a].shape)
            if a == 8:
                i = (0,) + i[1:]                       # only the logit row of H3 is trained
            if a == 9:
                i = (0,)
            old = w[a][i]
            w[a][i] = old + h
            lp, sp = _loss(geoms, y, w, alpha)
            w[a][i] = old - h
            lm, sm = _loss(geoms, y, w, alpha)
            w[a][i] = old
            if sp != sig or sm != sig:
                continue
            fd = (lp - lm) / (2 * h)
            scale = max(np.abs(grads[a]).max(), 1e-12)
            assert abs(fd - grads[a][i]) <= 1e-6 * scale + 1e-9, (a, i, fd, grads[a][i])
            checked += 1
    assert checked >= 30
    # the seven untrained outputs get no gradient
    assert not grads[8][1:].any() and not grads[9][1:].any()


def test_adam_matches_torch():
    rng = np.random.default_rng(4)
    w = [rng.standard_normal((5, 3)), rng.standard_normal(7)]
    tw = [torch.tensor(a.copy(), requires_grad=True) for a in w]
    opt = torch.optim.Adam(tw, lr=T.ADAM["lr"], betas=(T.ADAM["b1"], T.ADAM["b2"]), eps=T.ADAM["eps"])
    state = {}
    for step in range(4):
        g = [rng.standard_normal(a.shape) for a in w]
        if step == 2:
            g[1][:] = 0.0                               # zero gradients still move by the momentum
        for p, gg in zip(tw, g):
            p.grad = torch.tensor(gg)
        opt.step()
        T.adam_step(w, g, state)
        for a, p in zip(w, tw):
            np.testing.assert_allclose(a, p.detach().numpy(), rtol=1e-13, atol=1e-15)
