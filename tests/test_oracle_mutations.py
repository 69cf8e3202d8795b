"""The pins catch plausible mistakes: each mutant below plants one error in
the oracle (on the CPU, through monkeypatch) and at least one pin must fail."""

import numpy as np
import pytest

import test_oracle_geometry as TG
import test_oracle_network as TN
from oracle import locc_oracle as O


def _rot_transposed(orig):
    return lambda q: np.swapaxes(orig(q), -1, -2)


def _rot_sign(orig):
    def f(q):
        R = orig(q).copy()
        R[..., 0, 1] *= -1
        return R
    return f


def _relpose_drop_term(orig):
    def f(Ra, ta, Rb, tb):
        Rab, tab = orig(Ra, ta, Rb, tb)
        d = np.asarray(tb, np.float64) - np.asarray(ta, np.float64)
        return Rab, tab - np.asarray(Ra)[2, :] * d[2]
    return f


def _relpose_not_transposed(orig):
    def f(Ra, ta, Rb, tb):
        return orig(np.swapaxes(np.asarray(Ra), 0, 1), ta, Rb, tb)
    return f


def _box_pad_sign(orig):
    return lambda lo_a, hi_a, lo_b, hi_b, Rab, tab, pad=O.PAD_M: orig(lo_a, hi_a, lo_b, hi_b, Rab, tab, -pad)


def _box_no_abs(orig):
    def f(lo_a, hi_a, lo_b, hi_b, Rab, tab, pad=O.PAD_M):
        cb, eb = 0.5 * (lo_b + hi_b), 0.5 * (hi_b - lo_b)
        c = Rab @ cb + tab
        e = Rab @ eb
        return np.maximum(lo_a, c - e) - pad, np.minimum(hi_a, c + e) + pad
    return f


def _inside_open(orig):
    return lambda q, lo, hi: np.all((lo < np.asarray(q, np.float64)) & (np.asarray(q, np.float64) < hi), axis=1)


def _first_k_last(orig):
    def f(member, K):
        where = np.flatnonzero(member)[::-1]
        idx = np.full(K, -1, np.int32)
        m = min(len(where), K)
        idx[:m] = where[:m]
        return idx, len(where)
    return f


def _rotate_vectors_identity(orig):
    return lambda Rab, n: np.asarray(n, np.float64)


def _encode_no_bias(orig):
    return lambda rows, W1, b1, W2, b2: orig(rows, W1, 0 * b1, W2, b2)


def _head_no_relu(orig):
    def f(z, H1, c1, H2, c2, H3, c3):
        g1 = np.maximum(z @ H1.T + c1, 0)
        return (g1 @ H2.T + c2) @ H3.T + c3
    return f


def _post_no_sign(orig):
    return lambda y, Ra, ta, sgn: orig(y, Ra, ta, 1)


def _post_transposed(orig):
    return lambda y, Ra, ta, sgn: orig(y, np.asarray(Ra).T, ta, sgn)


MUTANTS = {
    "rotation transposed": ("rotation", _rot_transposed),
    "rotation sign flip": ("rotation", _rot_sign),
    "relative pose drops a term": ("relative_pose", _relpose_drop_term),
    "relative pose uses R_a not R_a^T": ("relative_pose", _relpose_not_transposed),
    "pad subtracted": ("crop_box", _box_pad_sign),
    "extent without |R|": ("crop_box", _box_no_abs),
    "open intervals": ("inside", _inside_open),
    "last K instead of first K": ("first_k", _first_k_last),
    "b normals not rotated": ("rotate_vectors", _rotate_vectors_identity),
    "encoder bias dropped": ("encode", _encode_no_bias),
    "head ReLU dropped": ("head", _head_no_relu),
    "normal not negated on swap": ("post", _post_no_sign),
    "world mapping transposed": ("post", _post_transposed),
}


def _pins(scene):
    return [
        TG.test_rotation_matches_scipy_for_unit_quaternions,
        TG.test_relative_pose_composes_back_to_the_world,
        TG.test_points_exactly_on_the_box_faces_are_members,
        TG.test_first_k_keeps_stored_order_and_counts_before_the_cap,
        TG.test_sphere_crop_box_closed_form,
        lambda: TG.test_b_side_rows_are_radial_for_spheres(scene),
        TN.test_constructed_weights_reproduce_closed_form_sphere_contact,
        TN.test_constructed_weights_agree_with_generated_sphere_labels,
        TN.test_empty_crop_pools_to_zero,
        lambda: TN.test_swapping_a_pair_negates_only_the_normal(scene),
        lambda: TN.test_outputs_follow_a_rigid_motion_of_the_world(scene),
        lambda: TG.test_no_false_negatives_within_the_margin(scene),
        lambda: TG.test_crop_membership_matches_exact_rational_geometry(False),
    ]


@pytest.mark.parametrize("name", list(MUTANTS))
def test_a_pin_catches_the_mutant(name, monkeypatch, small_scene):
    attr, make = MUTANTS[name]
    monkeypatch.setattr(O, attr, make(getattr(O, attr)))
    for pin in _pins(small_scene):
        try:
            pin()
        except (AssertionError, ValueError, IndexError):
            return
    pytest.fail(f"no pin caught the mutant: {name}")
