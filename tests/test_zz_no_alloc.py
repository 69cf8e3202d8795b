"""locc_detect_noalloc: the detect path with the library's fixed device array as its workspace (for
callers that cannot allocate).  Its contacts and member counts must equal locc_detect's bit for bit (the
results do not depend on the schedule or the workspace), on two calls in a row, the second on a smaller,
different batch, so that the array holds the first call's data when the second starts; batches larger
than the array are refused with RANGE and touch nothing."""

import sys

import numpy as np
import pytest

from paper_2304_09439_amd import binding as B
from paper_2304_09439_amd import inputs as I

pytestmark = pytest.mark.gpu

LW = I.SCALE_WIDTHS
SCALE = (LW.h1, LW.h2, LW.hh)


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
def scene():
    return I.scale_workload(n_pairs=6000)


# wg: workgroups per CU of the BF16 schedule (at split, 1 selects the kernel with W2 in LDS)
@pytest.mark.parametrize("precision,split,wg,first", [("fp32", None, 2, 3000), ("bf16", True, 2, 6000),
                                                      ("bf16", True, 1, 6000), ("bf16", False, 2, 6000),
                                                      ("fp8", None, 2, 6000), ("fp8_encoder", None, 2, 6000)])
def test_noalloc_equals_detect_on_two_calls(torch, scene, precision, split, wg, first):
    say(f"no-allocation detect, {precision} split={split} wg_per_cu={wg}: {first} pairs, then 700 others")
    w = I.flatten_weights(I.gaussian_weights(LW, seed=0, bias_std=0.1))
    ctx = B.context_for_scene(scene, 128, SCALE, w, precision=precision)
    objs, pairs = B.scene_tensors(scene)
    if precision.startswith("fp8"):
        ctx.calibrate(objs, pairs[:1024])
    if split is not None:
        ctx.set_schedule(wg_per_cu=wg, claim=4, dynamic=True, split=split)
    for rows in (np.arange(first), np.arange(5000 - 700, 5000)[::-1].copy()):
        pr = torch.from_numpy(np.ascontiguousarray(scene.pairs[rows])).cuda()
        P = len(rows)
        out = torch.full((P, 8), 7.0, dtype=torch.float32, device="cuda")
        counts = torch.full((P, 2), -7, dtype=torch.int32, device="cuda")
        ctx.detect_noalloc(objs, pr, out, counts)
        ref, ref_counts = ctx.detect(objs, pr)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (precision, P)
        assert torch.equal(counts, ref_counts), (precision, P)
        out2 = torch.full((P, 8), 7.0, dtype=torch.float32, device="cuda")
        ctx.detect_noalloc(objs, pr, out2)          # contacts only
        torch.cuda.synchronize()
        assert torch.equal(out2, ref)
    assert ctx.device_errors() == 0
    ctx.close()


def test_noalloc_refuses_batches_larger_than_its_array(torch, scene):
    w = I.flatten_weights(I.gaussian_weights(LW, seed=0))
    ctx = B.context_for_scene(scene, 128, SCALE, w, precision="fp32")
    objs, pairs = B.scene_tensors(scene)
    out = torch.full((6000, 8), 7.0, dtype=torch.float32, device="cuda")
    with pytest.raises(B.LoccError) as e:
        ctx.detect_noalloc(objs, pairs, out)
    assert e.value.status == B.ERR_RANGE and "at most" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
    empty = pairs[:0]
    ctx.detect_noalloc(objs, empty, out[:0])
    ctx.close()
