"""The pose-gradient pins catch plausible mistakes: each mutant rewrites one
line of oracle.pose_grad (on the CPU) and the finite-difference pin must
fail."""

import inspect
import types

import numpy as np
import pytest

import test_oracle_pose_grad as T
from oracle import pose_grad as PG

MUTANTS = {
    "head mask on the pooled maxima dropped": ("dm_b = df[h2:] * (m_b + b2 > 0)", "dm_b = df[h2:]"),
    "ReLU mask of the head's first layer dropped": ("du1 = (du2 @ H2) * (u1 > 0)", "du1 = du2 @ H2"),
    "normals left out of dR_ab": ("GR += np.outer(dr[:3], p) + np.outer(dr[3:], n)", "GR += np.outer(dr[:3], p)"),
    "translation term of dR_a dropped": ("dRa = Rb @ GR.T + np.outer(d, gt)", "dRa = Rb @ GR.T"),
    "R_a transposed in dR_b": ("dRb = Ra @ GR", "dRb = Ra.T @ GR"),
    "dp_a not negated": ("return logit, -dp_b,", "return logit, dp_b,"),
    "sign of a w-derivative term": ("dw = 2 * (-G[0, 1] * z", "dw = 2 * (G[0, 1] * z"),
    "layer-1 mask at the argmax row dropped": ("dh1 = W2[c] * dm_b[c] * (row @ W1.T + b1 > 0)",
                                              "dh1 = W2[c] * dm_b[c]"),
}


@pytest.mark.parametrize("name", list(MUTANTS))
def test_the_pin_catches_the_mutant(name, monkeypatch, scene, weights):
    old, new = MUTANTS[name]
    src = inspect.getsource(PG)
    assert src.count(old) == 1, old
    mod = types.ModuleType("pose_grad_mutant")
    mod.__dict__["__name__"] = "oracle.pose_grad_mutant"
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src.replace(old, new), "pose_grad_mutant", "exec"), mod.__dict__)
    monkeypatch.setattr(T, "PG", mod)
    with pytest.raises(AssertionError):
        T.test_gradient_matches_central_differences(scene, weights)


@pytest.fixture(scope="module")
def scene():
    return T.I.scale_workload(n_pairs=24)


@pytest.fixture(scope="module")
def weights():
    return T.I.flatten_weights(T.I.gaussian_weights(T.LW, seed=0, bias_std=0.1))
