"""Pins of the CPU model of the BF16 and FP8 arithmetic (oracle.quant_model).

The number formats are pinned to PyTorch's own float8_e4m3fn / bfloat16
conversions and to a brute-force nearest-value search over the enumerated
e4m3 codes; the layer chain is pinned by switching every rounding off, which
must give the full-precision network of the FP64 oracle back.
"""

import numpy as np
import pytest
import torch

from oracle import locc_oracle as O
from oracle import quant_model as Q
from paper_2304_09439_amd import inputs as I


def _e4m3_grid():
    """Every finite e4m3 value, from its bit fields (sign, 4-bit exponent, 3-bit mantissa)."""
    vals = []
    for code in range(256):
        s, e, m = code >> 7, (code >> 3) & 15, code & 7
        if e == 15 and m == 7:
            continue  # NaN
        mag = m * 2.0 ** -9 if e == 0 else (1 + m / 8) * 2.0 ** (e - 7)
        vals.append((-mag if s else mag, code))
    return vals


def _samples(rng, n):
    mags = np.exp(rng.uniform(np.log(2.0 ** -12), np.log(600.0), n))
    x = np.concatenate([mags, -mags, [0.0, 448.0, 464.0, 463.9, 500.0, 2.0 ** -10, 3 * 2.0 ** -10, 2.0 ** -6]])
    return x.astype(np.float32)


def test_e4m3_matches_torch_on_clamped_inputs():
    x = _samples(np.random.default_rng(0), 20000)
    ref = torch.from_numpy(np.clip(x, -448, 448)).to(torch.float8_e4m3fn).to(torch.float32).numpy()
    np.testing.assert_array_equal(Q.e4m3(x), ref)


def test_e4m3_is_the_nearest_code_ties_to_even():
    grid = _e4m3_grid()
    vals = np.array([v for v, _ in grid])
    codes = np.array([c for _, c in grid])
    assert vals.max() == 448.0 and np.min(np.abs(vals[vals != 0])) == 2.0 ** -9
    x = _samples(np.random.default_rng(1), 3000)
    # midpoints between neighbours are exactly the ties
    pos = np.unique(vals[vals >= 0])
    x = np.concatenate([x, (pos[1:] + pos[:-1]) / 2, -(pos[1:] + pos[:-1]) / 2]).astype(np.float32)
    got = Q.e4m3(x)
    for xi, gi in zip(x.astype(np.float64), got):
        c = np.clip(xi, -448, 448)
        d = np.abs(vals - c)
        best = np.flatnonzero(d == d.min())
        if len(best) > 1:  # tie: the code with an even mantissa
            best = [b for b in best if codes[b] & 1 == 0]
        assert gi == vals[best[0]], (xi, gi, vals[best])
    # every finite code is a fixed point; beyond 448 saturates
    np.testing.assert_array_equal(Q.e4m3(vals.astype(np.float32)), vals.astype(np.float32))
    np.testing.assert_array_equal(Q.e4m3(np.array([1e4, -1e4], np.float32)), [448.0, -448.0])


def test_bf16_matches_torch():
    x = np.random.default_rng(2).standard_normal(50000).astype(np.float32) * 10.0 ** np.random.default_rng(3).integers(-6, 6, 50000)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(Q.bf16(x), ref)


def test_scales():
    W = np.array([[0.5, -2.25], [1.0, 0.0]], np.float32)
    assert Q.weight_scale(W) == np.float32(2.25) / np.float32(448)
    assert Q.act_scale(0.0) == 1.0 and Q.act_scale(448.0) == 1.0
    # the largest activation maps onto 448 exactly
    assert Q.quant_act(np.float32(3.7), Q.act_scale(3.7)) == pytest.approx(448.0, rel=2 ** -4)


@pytest.fixture(scope="module")
def small():
    sc = I.small_workload()
    w = I.flatten_weights(I.gaussian_weights(I.SMALL_WIDTHS, seed=0, bias_std=0.1))
    widths = (I.SMALL_WIDTHS.h1, I.SMALL_WIDTHS.h2, I.SMALL_WIDTHS.hh)
    ref = O.detect_scene(sc, w, widths, 64)
    return sc, w, widths, ref


def test_model_without_rounding_is_the_full_precision_network(small):
    sc, w, widths, ref = small
    amax = Q.calibrate(ref["geoms"], w, widths)
    out = Q.fp8_detect(ref["geoms"], w, widths, amax, quantise=False)
    ok = ~np.isnan(ref["y"][:, 0])
    assert ok.sum() > 0 and np.array_equal(ok, ~np.isnan(out["y"][:, 0]))
    np.testing.assert_allclose(out["z"][ok], ref["z"][ok], rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(out["y"][ok], ref["y"][ok], rtol=1e-4, atol=1e-5)
    np.testing.assert_allclose(out["contacts"][ok], ref["contacts"][ok], rtol=1e-4, atol=1e-5)


def test_calibration_maxima_are_the_network_maxima(small):
    sc, w, widths, ref = small
    amax = Q.calibrate(ref["geoms"], w, widths)
    ok = ~np.isnan(ref["y"][:, 0])
    # pooled features and head layer 1 from the FP64 oracle (rows not rounded: bf16-level agreement)
    assert amax[1] == pytest.approx(np.nanmax(ref["z"][ok]), rel=2e-2)
    W1, b1, W2, b2, H1, c1, *_ = O.unpack_weights(w, *widths)
    g1 = np.maximum(ref["z"][ok] @ H1.T + c1, 0)
    assert amax[2] == pytest.approx(g1.max(), rel=2e-2)
    h = max(np.maximum(np.asarray(r) @ W1.T + b1, 0).max(initial=0)
            for g in ref["geoms"] if g is not None for r in (g.rows_a, g.rows_b))
    assert amax[0] == pytest.approx(h, rel=2e-2)


def test_quantised_model_is_close_but_not_equal(small):
    sc, w, widths, ref = small
    amax = Q.calibrate(ref["geoms"], w, widths)
    out = Q.fp8_detect(ref["geoms"], w, widths, amax)
    ok = ~np.isnan(ref["y"][:, 0])
    err = np.linalg.norm(out["y"][ok] - ref["y"][ok]) / np.linalg.norm(ref["y"][ok])
    assert 1e-3 < err < 0.3


def test_bf16_model_without_rounding_is_the_full_precision_network(small):
    sc, w, widths, ref = small
    out = Q.bf16_detect(ref["geoms"], w, widths, quantise=False)
    ok = ~np.isnan(ref["y"][:, 0])
    assert ok.sum() > 0 and np.array_equal(ok, ~np.isnan(out["y"][:, 0]))
    np.testing.assert_allclose(out["z"][ok], ref["z"][ok], rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(out["y"][ok], ref["y"][ok], rtol=1e-4, atol=1e-5)
    np.testing.assert_allclose(out["contacts"][ok], ref["contacts"][ok], rtol=1e-4, atol=1e-5)


def test_bf16_model_is_close_but_not_equal(small):
    sc, w, widths, ref = small
    out = Q.bf16_detect(ref["geoms"], w, widths)
    ok = ~np.isnan(ref["y"][:, 0])
    err = np.linalg.norm(out["y"][ok] - ref["y"][ok]) / np.linalg.norm(ref["y"][ok])
    # eight significant bits per rounding: errors of order 2^-9 per value, far below the fp8 model's
    assert 1e-4 < err < 2e-2
    err8 = np.linalg.norm(Q.fp8_detect(ref["geoms"], w, widths, Q.calibrate(ref["geoms"], w, widths))["y"][ok]
                          - ref["y"][ok]) / np.linalg.norm(ref["y"][ok])
    assert err < err8 / 2


def test_fp8_layer_sets(small):
    """The variant with only encoder layer 2 in e4m3 has the BF16 model's head: without rounding every
    variant is the full-precision network, and encoder layer 2 must be one of the e4m3 layers."""
    sc, w, widths, ref = small
    amax = Q.calibrate(ref["geoms"], w, widths)
    ok = ~np.isnan(ref["y"][:, 0])
    for layers in (("enc2",), ("enc2", "head2"), Q.FP8_ALL):
        out = Q.fp8_detect(ref["geoms"], w, widths, amax, quantise=False, fp8_layers=layers)
        np.testing.assert_allclose(out["y"][ok], ref["y"][ok], rtol=1e-4, atol=1e-5)
    with pytest.raises(ValueError):
        Q.fp8_forward(ref["geoms"], w, widths, amax, fp8_layers=("head1",))
    # the same pooled features (encoder layer 2 is e4m3 in both), different heads
    a = Q.fp8_detect(ref["geoms"], w, widths, amax, fp8_layers=("enc2",))
    b = Q.fp8_detect(ref["geoms"], w, widths, amax)
    np.testing.assert_array_equal(a["z"], b["z"])
    assert not np.array_equal(a["y"][ok], b["y"][ok])
    # the head of the encoder-only variant is exactly the BF16 model's head on those features
    W1, b1, W2, b2, H1, c1, H2, c2, H3, c3 = [np.asarray(x, np.float32) for x in O.unpack_weights(w, *widths)]
    z = a["z"][ok]
    g1 = Q.bf16(np.maximum(np.float32(Q.bf16(z).astype(np.float64) @ Q.bf16(H1).astype(np.float64).T) + c1, 0))
    g2 = Q.bf16(np.maximum(np.float32(g1.astype(np.float64) @ Q.bf16(H2).astype(np.float64).T) + c2, 0))
    y = g2.astype(np.float64) @ Q.bf16(H3).astype(np.float64).T + c3
    np.testing.assert_array_equal(a["y"][ok], y)
