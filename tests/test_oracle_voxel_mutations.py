"""The voxel-oracle pins catch plausible mistakes: each mutant plants one
error in oracle.voxel_locc (on the CPU, through monkeypatch) and at least one
pin of test_oracle_voxel must fail."""

import numpy as np
import pytest

import test_oracle_voxel as TV
from oracle import voxel_locc as V


def _conv_flipped(orig):
    return lambda x, W, b, pad: orig(x, W[:, :, ::-1, ::-1, ::-1], b, pad)


def _convT_as_conv(orig):
    def f(x, W, b, pad):
        return V.conv3d(np.pad(x, ((0, 0),) + ((2 - 2 * pad, 2 - 2 * pad),) * 3), W, b, pad) if pad == 0 else \
            V.conv3d(x, W, b, pad)
    return f


def _index_no_scale(orig):
    def f(xyz, lo, hi):
        xyz = np.asarray(xyz, np.float64)
        idx = np.zeros(len(xyz), np.int64)
        for k in range(3):
            t = (xyz[:, k] - lo[k]) / max(hi[k] - lo[k], 1e-300)
            idx = idx * V.M + np.minimum(np.floor(t * (V.M - 1)).astype(np.int64), V.M - 1)
        return idx
    return f


def _index_axis_order(orig):
    def f(xyz, lo, hi):
        i = orig(xyz, lo, hi)
        i0, i1, i2 = np.unravel_index(i, (V.M,) * 3)
        return (i2 * V.M + i1) * V.M + i0
    return f


def _embedding_skip_order(orig):
    concat = np.concatenate

    def f(xyz, w, lo=None, hi=None):
        np.concatenate = lambda arrs, *a, **k: concat(arrs[::-1], *a, **k) if len(arrs) == 2 and \
            getattr(arrs[0], "ndim", 0) == 4 else concat(arrs, *a, **k)
        try:
            return orig(xyz, w, lo, hi)
        finally:
            np.concatenate = concat
    return f


def _no_margin(orig):
    def f(Rab, tab, box_a, box_b):
        lo_a, hi_a = box_a
        lo_b, hi_b = box_b
        ca, _ = V.cell_centres(*box_a)
        cb, _ = V.cell_centres(*box_b)
        xa = V.to_b_frame(Rab, tab, ca)
        xb = V.O.transform_points(Rab, tab, cb)
        return (np.all((xa >= lo_b) & (xa <= hi_b), axis=1), np.all((xb >= lo_a) & (xb <= hi_a), axis=1))
    return f


def _to_b_not_transposed(orig):
    return lambda Rab, tab, c: orig(np.asarray(Rab).T, tab, c)


def _pair_sum(orig):
    def f(z_a, z_b, w):
        A1, a1, A2, a2, A3, a3 = w[24:30]
        B1, b1, B2, b2, B3, b3, B4, b4 = w[30:38]

        def mlp1(z):
            h = V.relu(z @ A1.T + a1)
            h = V.relu(h @ A2.T + a2)
            return V.relu(h @ A3.T + a3)

        g = mlp1(z_a) + mlp1(z_b)
        g = V.relu(V.relu(V.relu(g @ B1.T + b1) @ B2.T + b2) @ B3.T + b3)
        return float((g @ B4.T + b4)[0])
    return f


def _pose_not_negated(orig):
    def f(Rab, tab):
        pa, pb = orig(Rab, tab)
        pa = pa.copy()
        pa[:3] *= -1
        return pa, pb
    return f


MUTANTS = {
    "conv kernel flipped": ("conv3d", _conv_flipped),
    "transposed conv computed as conv": ("conv3d_transpose", _convT_as_conv),
    "grid index without the M scale": ("voxel_index", _index_no_scale),
    "grid index axes reversed": ("voxel_index", _index_axis_order),
    "skip concatenated in the other order": ("shape_embedding", _embedding_skip_order),
    "no margin": ("select_cells", _no_margin),
    "cell centre rotated by R instead of R^T": ("to_b_frame", _to_b_not_transposed),
    "pair sum instead of max": ("predictor", _pair_sum),
    "a's translation not negated": ("pose_inputs", _pose_not_negated),
}

PINS = [
    lambda: TV.test_conv_is_scipy_correlation(0),
    lambda: TV.test_conv_is_scipy_correlation(1),
    lambda: TV.test_transposed_conv_is_the_adjoint_of_conv(0),
    lambda: TV.test_transposed_conv_is_the_adjoint_of_conv(1),
    TV.test_voxel_index_against_enumerated_boundaries,
    TV.test_constructed_encoder_gives_the_closed_form,
    TV.test_margin_leaves_no_false_negative,
    TV.test_predictor_closed_forms_and_empty_crops,
    TV.test_pose_inputs_are_each_object_in_the_others_frame,
]


@pytest.mark.parametrize("name", list(MUTANTS))
def test_a_pin_catches_the_mutant(name, monkeypatch):
    attr, make = MUTANTS[name]
    monkeypatch.setattr(V, attr, make(getattr(V, attr)))
    for pin in PINS:
        try:
            pin()
        except (AssertionError, ValueError, IndexError):
            return
    pytest.fail(f"no pin caught the mutant: {name}")
