"""GPU parity of the FP8 (e4m3) encoder + head kernel.

Two comparisons on the same seeded inputs:
  * against the CPU model of the quantised arithmetic (oracle.quant_model),
    which makes the same rounding decisions in float32.  The model sums
    exactly; the 32x32x64 e4m3 MFMA does not: on this chip its sums differ
    from the exact ones by up to 1.2e-4 of sum |a_k b_k| (measured with
    random e4m3 operands).  Pooled features, one fp8 layer deep, must agree
    within 1e-4 normwise.  In the head such a difference flips the e4m3
    rounding of about 512 x 1.2e-4 / 2^-4 ~ 1 of the 512 layer-1 outputs per
    pair (one step, <= 2^-3 relative, each), and the bf16 rounding of many
    layer-2 outputs; through two layers this moves the raw outputs by a few
    1e-3 normwise.  The bar is 1e-2 per field: a quarter of the format's
    smallest per-field error against the FP64 oracle (0.037, the logit), so
    a kernel that adds an error of the format's size fails; a wrong scale,
    index or layer moves the outputs by O(1).
  * against the FP64 oracle: the error of the format itself, reported per
    field (normwise and per-pair maximum) with the collision-flag agreement,
    and required to stay within the model's own error (+2e-3).
Crop counts must match the oracle bit for bit.  Activation scales come from
the model's calibration on a separate batch of pairs and are installed with
locc_set_activation_amax, so both sides quantise with the same scales.

The lower-error variant (precision "fp8_encoder": e4m3 on encoder layer 2
only, the head in bf16) is held to the same bars against its own CPU model
(fp8_layers = ("enc2",)) and against the oracle, where its logit, point and
normal errors are also required below the FP8 tolerance of 6e-2.
"""

import sys

import numpy as np
import pytest

from oracle import locc_oracle as O
from oracle import quant_model as Q
from paper_2304_09439_amd import binding as B
from paper_2304_09439_amd import inputs as I

from helpers import field_errors, first_object_empty, flag_agreement, normwise_errors, with_first_object_empty

pytestmark = pytest.mark.gpu

SW, LW = I.SMALL_WIDTHS, I.SCALE_WIDTHS
SMALL = (SW.h1, SW.h2, SW.hh)
SCALE = (LW.h1, LW.h2, LW.hh)
Z_TOL = 1e-4     # pooled features vs the model
Y_TOL = 1e-2     # raw outputs and contacts vs the model
ORACLE_SLACK = 2e-3
FP8_TOL = 6e-2   # the stated FP8 tolerance against the FP64 oracle
ENC_ONLY = ("enc2",)   # the layers the fp8_encoder variant runs in e4m3
VARIANTS = [("fp8", "model"), ("fp8_encoder", "model_enc")]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    B.load()
    return t


def _weights(widths):
    return I.flatten_weights(I.gaussian_weights(I.Widths(*widths), seed=0, bias_std=0.1))


def _geoms(scene, pairs, K):
    g, _, _ = O.crop(scene.lib.pts, scene.lib.offsets, scene.pos, scene.quat, scene.shape, pairs, K)
    return g


@pytest.fixture(scope="module")
def scale_case():
    sc = I.scale_workload()
    w = _weights(SCALE)
    # 1,061 pairs: the first 1,024 (the reported subset) plus a ragged tail, two made invalid
    pairs = sc.pairs[:1061].copy()
    pairs[5] = (3, 3)
    pairs[700] = (0, len(sc.shape) + 5)
    ev = I.Scene(sc.lib, sc.pos, sc.quat, sc.shape, pairs)
    calib_pairs = sc.pairs[8192:9216]
    amax = Q.calibrate(_geoms(sc, calib_pairs, 128), w, SCALE)
    say(f"scale case: model calibration maxima {amax}")
    ref = O.detect_scene(ev, w, SCALE, 128)
    model = Q.fp8_detect(ref["geoms"], w, SCALE, amax)
    model_enc = Q.fp8_detect(ref["geoms"], w, SCALE, amax, fp8_layers=ENC_ONLY)
    return dict(scene=ev, full=sc, w=w, K=128, widths=SCALE, amax=amax, ref=ref, model=model,
                model_enc=model_enc, calib=calib_pairs)


@pytest.fixture(scope="module")
def small_case():
    sc = I.small_workload()
    w = _weights(SMALL)
    ref = O.detect_scene(sc, w, SMALL, 64)
    amax = Q.calibrate(ref["geoms"], w, SMALL)
    model = Q.fp8_detect(ref["geoms"], w, SMALL, amax)
    model_enc = Q.fp8_detect(ref["geoms"], w, SMALL, amax, fp8_layers=ENC_ONLY)
    return dict(scene=sc, full=sc, w=w, K=64, widths=SMALL, amax=amax, ref=ref, model=model, model_enc=model_enc,
                calib=sc.pairs)


def _ctx(case, amax=True, precision="fp8"):
    ctx = B.context_for_scene(case["scene"], case["K"], case["widths"], case["w"], precision=precision)
    if amax:
        ctx.set_activation_amax(case["amax"])
    return ctx


def _run(torch, ctx, scene, sched=None):
    if sched:
        ctx.set_schedule(**sched)
    objs, pairs = B.scene_tensors(scene)
    out, counts, z, y = ctx.debug_forward(objs, pairs)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (out, counts, z, y)]


def test_calibration_matches_the_model(torch, scale_case):
    c = scale_case
    ctx = _ctx(c, amax=False)
    objs, _ = B.scene_tensors(c["full"])
    pairs = torch.from_numpy(np.ascontiguousarray(c["calib"], np.int32)).cuda()
    amax = ctx.calibrate(objs, pairs)
    say(f"  device maxima {amax}, model {c['amax']}")
    np.testing.assert_allclose(amax, c["amax"], rtol=1e-4)
    assert ctx.device_errors() == 0
    ctx.close()


@pytest.mark.parametrize("precision,model_key", VARIANTS)
@pytest.mark.parametrize("which", ["small", "scale"])
def test_fp8_matches_the_quantised_model(torch, which, precision, model_key, request):
    c = request.getfixturevalue(f"{which}_case")
    say(f"{precision} vs quantised model, {which}: {c['scene'].n_pairs} pairs")
    ctx = _ctx(c, precision=precision)
    out, counts, z, y = _run(torch, ctx, c["scene"])
    ref, model = c["ref"], c[model_key]
    np.testing.assert_array_equal(counts, ref["counts"])
    bad = np.isnan(ref["y"][:, 0])
    assert np.array_equal(np.isnan(out).any(axis=1), bad) and np.isnan(y[bad]).all()
    ok = ~bad
    ez = float(np.linalg.norm(z[ok] - model["z"][ok]) / np.linalg.norm(model["z"][ok]))
    ey = normwise_errors(y[ok], model["y"][ok])
    ec = normwise_errors(out[ok], model["contacts"][ok])
    say(f"  z normwise {ez:.2e}; y normwise {ey}; per-pair max {field_errors(y[ok], model['y'][ok])}")
    assert ez < Z_TOL
    assert max(ey.values()) < Y_TOL and max(ec.values()) < Y_TOL
    assert ctx.device_errors() == int(bad.sum())
    ctx.close()


@pytest.mark.parametrize("precision,model_key", VARIANTS)
def test_fp8_error_against_the_oracle(torch, scale_case, precision, model_key):
    c = scale_case
    ctx = _ctx(c, precision=precision)
    out, counts, z, y = _run(torch, ctx, c["scene"])
    ctx.close()
    rows = np.arange(1024)
    rows = rows[~np.isnan(c["ref"]["y"][rows, 0])]
    ref_y, model_y = c["ref"]["y"][rows], c[model_key]["y"][rows]
    e_dev = normwise_errors(y[rows], ref_y)
    e_model = normwise_errors(model_y, ref_y)
    say(f"  {precision} vs FP64 oracle on {len(rows)} pairs: normwise {e_dev}")
    say(f"    per-pair max {field_errors(y[rows], ref_y)}")
    say(f"    CPU model of the format: normwise {e_model}")
    say(f"    flag agreement raw {flag_agreement(y[rows, 0], ref_y[:, 0]):.4f}, "
        f"banded(2e-2) {flag_agreement(y[rows, 0], ref_y[:, 0], band=2e-2):.4f}, "
        f"banded(6e-2) {flag_agreement(y[rows, 0], ref_y[:, 0], band=6e-2):.4f}")
    for k in e_dev:
        assert e_dev[k] <= e_model[k] + ORACLE_SLACK, k
    # the collision flag, banded at the FP8 tolerance (pairs whose reference logit lies within 6e-2 RMS of
    # zero are left out, as the bar is stated for a flag the format can decide)
    assert flag_agreement(y[rows, 0], ref_y[:, 0], band=FP8_TOL) >= 0.999
    if precision == "fp8_encoder":
        # the lower-error variant meets the FP8 tolerance on the flag logit, the contact point and the normal;
        # its depth error (0.088 in the CPU model of the roundings) is the format's own, on these untrained weights
        for k in ("logit", "point", "normal"):
            assert e_dev[k] < FP8_TOL, k


@pytest.mark.xfail(strict=True, reason="e4m3 on encoder layer 2 and head layers 1-2: the format's own error on "
                   "these untrained Gaussian weights is 0.037-0.12 normwise per field against the FP64 oracle "
                   "(the CPU model of the roundings, with no kernel involved, gives the same figures)")
def test_fp8_all_layers_within_the_fp8_tolerance_of_the_oracle(torch, scale_case):
    c = scale_case
    ctx = _ctx(c)
    out, counts, z, y = _run(torch, ctx, c["scene"])
    ctx.close()
    rows = np.arange(1024)
    rows = rows[~np.isnan(c["ref"]["y"][rows, 0])]
    e = normwise_errors(y[rows], c["ref"]["y"][rows])
    say(f"  FP8 (all layers) vs FP64 oracle normwise {e}")
    assert max(e.values()) < FP8_TOL


def test_fp8_needs_activation_scales(torch, small_case):
    c = small_case
    ctx = _ctx(c, amax=False)
    objs, pairs = B.scene_tensors(c["scene"])
    with pytest.raises(B.LoccError) as e:
        ctx.detect(objs, pairs)
    assert e.value.status == B.ERR_NOT_READY
    for bad in ([1.0, -1.0, 1.0], [np.inf, 1.0, 1.0], [np.nan, 1, 1]):
        with pytest.raises(B.LoccError) as e:
            ctx.set_activation_amax(bad)
        assert e.value.status == B.ERR_INVALID_ARG
    ctx.set_activation_amax(c["amax"])
    ctx.detect(objs, pairs)
    ctx.upload_weights(c["w"])                  # new weights clear the maxima
    with pytest.raises(B.LoccError) as e:
        ctx.detect(objs, pairs)
    assert e.value.status == B.ERR_NOT_READY
    empty = pairs[:0]
    assert np.array_equal(ctx.calibrate(objs, empty), np.zeros(3, np.float32))
    ctx.close()
    bctx = B.context_for_scene(c["scene"], c["K"], c["widths"], c["w"], precision="bf16")
    with pytest.raises(B.LoccError) as e:
        bctx.calibrate(objs, pairs)
    assert e.value.status == B.ERR_UNSUPPORTED
    bctx.close()


@pytest.mark.parametrize("precision", ["fp8", "fp8_encoder"])
def test_fp8_results_do_not_depend_on_the_schedule_or_graph(torch, scale_case, precision):
    c = scale_case
    ctx = _ctx(c, precision=precision)
    base = _run(torch, ctx, c["scene"])
    for sched in (dict(wg_per_cu=1, claim=1, dynamic=False, crop_unroll=4),
                  dict(wg_per_cu=2, claim=16, dynamic=True, crop_unroll=8)):
        got = _run(torch, ctx, c["scene"], sched)
        for a, b in zip(got, base):
            np.testing.assert_array_equal(a, b)
    objs, pairs = B.scene_tensors(c["scene"])
    P = pairs.shape[0]
    cap = P + 40
    pbuf = torch.zeros((cap, 2), dtype=torch.int32, device="cuda")
    pbuf[:P].copy_(pairs)
    n_dev = torch.tensor([P], dtype=torch.int32, device="cuda")
    out = torch.full((cap, 8), 7.0, dtype=torch.float32, device="cuda")
    g = ctx.capture_graph(objs, pbuf, n_dev, out)
    with pytest.raises(B.LoccError) as e:       # the graph holds the current scales
        ctx.set_activation_amax(c["amax"])
    assert e.value.status == B.ERR_BUSY
    for n in (P, 100, P):
        out.fill_(7.0)
        n_dev.fill_(n)
        g.launch()
        ref, _ = ctx.detect(objs, pairs[:n].contiguous())
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out[:n].cpu().numpy(), ref.cpu().numpy())
        assert torch.all(out[n:] == 7.0)
    g.close()
    ctx.close()


def test_fp8_first_object_empty(torch, scale_case):
    """A pair whose first object (canonical order) selects nothing starts its row tiles with the second
    object's rows: its contacts must be the same alone as in the full batch, whatever other pairs left
    in the row buffers and in LDS."""
    c = scale_case
    sc, rows = with_first_object_empty(c["full"], 256)
    ctx = B.context_for_scene(sc, 128, SCALE, c["w"], precision="fp8")
    ctx.set_activation_amax(c["amax"])
    objs, pairs = B.scene_tensors(sc)
    full, counts = ctx.detect(objs, pairs)
    found = first_object_empty(sc.pairs, counts.cpu().numpy())
    say(f"fp8: {len(found)} pairs whose first object selects nothing")
    assert set(rows) <= set(found)
    for sched in (dict(wg_per_cu=2, claim=4, dynamic=True), dict(wg_per_cu=1, claim=16, dynamic=False)):
        ctx.set_schedule(**sched)
        alone, _ = ctx.detect(objs, torch.from_numpy(sc.pairs[found]).cuda())
        torch.cuda.synchronize()
        np.testing.assert_array_equal(alone.cpu().numpy(), full.cpu().numpy()[found])
    ctx.close()
