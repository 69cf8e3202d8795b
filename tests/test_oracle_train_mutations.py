"""The training-oracle pins catch plausible mistakes: each mutant rewrites one
line of oracle.train (on the CPU) and a pin must fail."""

import inspect
import types

import pytest

import test_oracle_train as T
from oracle import train as TR

MUTANTS = {
    "cross-entropy derivative with the wrong sign": ("dx = (1.0 / (1.0 + np.exp(-x)) - y) / B",
                                                     "dx = (y - 1.0 / (1.0 + np.exp(-x))) / B"),
    "feature penalty left out of the gradient": ("dz = du1 @ H1 + (2.0 * alpha / B) * z", "dz = du1 @ H1"),
    "ReLU mask of the head's first layer dropped": ("du1 = (du2 @ H2) * (u1 > 0)", "du1 = du2 @ H2"),
    "pooled-maximum mask dropped": ("dm = dz[s * h2:(s + 1) * h2] * (m + b2 > 0)", "dm = dz[s * h2:(s + 1) * h2]"),
    "layer-1 weight gradient halved": ("dW1 += np.outer(dh1, rows[rr])", "dW1 += np.outer(dh1, rows[rr]) * 0.5"),
    "no Adam bias correction": ("w -= lr * (m / (1.0 - b1 ** t)) / (np.sqrt(v / (1.0 - b2 ** t)) + eps)",
                                "w -= lr * m / (np.sqrt(v) + eps)"),
    "second moment without the square": ("v += (1.0 - b2) * gr * gr", "v += (1.0 - b2) * abs(gr)"),
}


@pytest.mark.parametrize("name", list(MUTANTS))
def test_a_pin_catches_the_mutant(name, monkeypatch, batch):
    old, new = MUTANTS[name]
    src = inspect.getsource(TR)
    assert src.count(old) == 1, old
    mod = types.ModuleType("train_mutant")
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src.replace(old, new), "train_mutant", "exec"), mod.__dict__)
    monkeypatch.setattr(T, "T", mod)
    with pytest.raises(AssertionError):   # the gradient pin, else the Adam pin
        T.test_gradients_match_central_differences(batch)
        T.test_adam_matches_torch()


@pytest.fixture(scope="module")
def batch():
    sc, y = T.I.sphere_training_set(n_pairs=12)
    geoms, _, _ = T.O.crop(sc.lib.pts, sc.lib.offsets, sc.pos, sc.quat, sc.shape, sc.pairs, T.K)
    return geoms, y
