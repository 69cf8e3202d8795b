"""Batched simulation steps: device-side pair counts, HIP graph replay, the
autotuner, and parity on uneven environments (4,096 environments, 1-40
objects each, about 2e5 broad-phase pairs per step)."""

import sys

import numpy as np
import pytest

from oracle import locc_oracle as O
from oracle import quant_model as Q
from paper_2304_09439_amd import binding as B
from paper_2304_09439_amd import inputs as I

from helpers import check_low_precision, oracle_crop_all

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
def envs():
    return I.env_workload(steps=3)


def _weights():
    return I.flatten_weights(I.gaussian_weights(LW, seed=0, bias_std=0.1))


def _ctx(envs, precision):
    ctx = B.Context(128, SCALE, precision=precision)
    ctx.upload_shapes(envs.lib.offsets, envs.lib.pts)
    ctx.upload_weights(_weights())
    return ctx


@pytest.mark.parametrize("precision,chunks", [("bf16", 1), ("bf16", 4), ("fp32", 1)])
def test_graph_replays_match_eager_launches(torch, envs, precision, chunks):
    say(f"graph replay vs eager, {precision}, chunks {chunks}, {envs.n_steps} steps of uneven environments")
    ctx = _ctx(envs, precision)
    if chunks > 1:   # runs of pairs whose crop overlaps the previous run's network, on a second stream
        ctx.set_schedule(wg_per_cu=1, claim=4, dynamic=True, split=True, crop_unroll=4, chunks=chunks)
    cap = max(len(p) for p in envs.pairs) + 17
    n_obj = len(envs.shape)
    objs = torch.zeros((n_obj, 8), dtype=torch.float32, device="cuda")
    pairs = torch.zeros((cap, 2), dtype=torch.int32, device="cuda")
    n_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = torch.full((cap, 8), 7.0, dtype=torch.float32, device="cuda")
    counts = torch.zeros((cap, 2), dtype=torch.int32, device="cuda")
    graph = ctx.capture_graph(objs, pairs, n_dev, out, counts)
    for step in [0, 1, 2, 1]:
        sc = envs.scene(step)
        P = sc.n_pairs
        o, pr = B.scene_tensors(sc)
        objs.copy_(o)
        pairs[:P].copy_(pr)
        n_dev.fill_(P)
        out.fill_(7.0)
        graph.launch()
        ref_out, ref_counts = ctx.detect(objs, pr)     # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(out[:P], ref_out), f"step {step}"
        assert torch.equal(counts[:P], ref_counts)
        assert torch.all(out[P:] == 7.0)                # past the count nothing is written
    assert ctx.device_errors() == 0
    graph.close()
    ctx.close()


def test_device_count_is_clamped_to_the_capacity(torch, envs):
    ctx = _ctx(envs, "bf16")
    sc = envs.scene(0).subset(np.arange(1100))
    objs, pairs = B.scene_tensors(sc)
    ctx.reserve(1100)
    ref, _ = ctx.detect(objs, pairs)
    # two runs of 550 pairs: counts that end in either run; both split-schedule kernels (W2 in registers at two
    # workgroups per CU, W2 in LDS at one)
    for wg, chunks in ((2, 1), (2, 2), (1, 1), (1, 2)):
        ctx.set_schedule(wg_per_cu=wg, claim=4, dynamic=True, split=True, crop_unroll=4, chunks=chunks)
        for n, expect in ((10**6, 1100), (-5, 0), (0, 0), (123, 123), (600, 600)):
            out = torch.full((1100, 8), 7.0, dtype=torch.float32, device="cuda")
            n_dev = torch.tensor([n], dtype=torch.int32, device="cuda")
            ctx.detect_device_count(objs, pairs, n_dev, out)
            torch.cuda.synchronize()
            assert torch.equal(out[:expect], ref[:expect]), (wg, chunks, n)
            assert torch.all(out[expect:] == 7.0), (wg, chunks, n)
    ctx.close()


def test_calls_that_would_move_a_graphs_buffers_are_refused(torch, envs):
    """While a captured graph exists, a detect that needs a larger workspace and a new shape library are
    refused (the graph holds the current buffers); replays still match eager launches, and once the
    graph is destroyed both calls work."""
    ctx = _ctx(envs, "bf16")
    small = envs.scene(0).subset(np.arange(1000))
    objs, pairs = B.scene_tensors(small)
    n_dev = torch.tensor([1000], dtype=torch.int32, device="cuda")
    out = torch.full((1000, 8), 7.0, dtype=torch.float32, device="cuda")
    g = ctx.capture_graph(objs, pairs, n_dev, out)
    big_objs, big_pairs = B.scene_tensors(envs.scene(0).subset(np.arange(60000)))
    with pytest.raises(B.LoccError) as e:
        ctx.detect(big_objs, big_pairs)
    assert e.value.status == B.ERR_RANGE
    with pytest.raises(B.LoccError) as e:
        ctx.upload_shapes(envs.lib.offsets, envs.lib.pts)
    assert e.value.status == B.ERR_BUSY
    g.launch()
    ref, _ = ctx.detect(objs, pairs)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    g.close()
    ctx.upload_shapes(envs.lib.offsets, envs.lib.pts)
    full, _ = ctx.detect(big_objs, big_pairs)
    torch.cuda.synchronize()
    assert torch.equal(full[:1000], ref)
    ctx.close()


def test_autotuner_installs_a_schedule_with_identical_results(torch, tmp_path):
    sc = I.scale_workload(n_pairs=4096)
    say("autotune on 4096 pairs")
    ctx = B.context_for_scene(sc, 128, SCALE, _weights(), precision="bf16")
    objs, pairs = B.scene_tensors(sc)
    ref, ref_counts = ctx.detect(objs, pairs)
    cache = tmp_path / "tune.txt"
    best, ms = ctx.autotune(objs, pairs, cache_path=cache)
    say(f"  best {best} {ms:.4f} ms")
    assert ctx.get_schedule() == best and ms > 0
    out, counts = ctx.detect(objs, pairs)
    torch.cuda.synchronize()
    assert torch.equal(out, ref) and torch.equal(counts, ref_counts)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    ctx.set_schedule(wg_per_cu=1, claim=16, dynamic=False, split=False)
    best2, ms2 = ctx.autotune(objs, pairs, cache_path=cache)      # cache hit: no new line
    assert best2 == best and ms2 == pytest.approx(ms, abs=1e-6)   # the cache keeps 6 decimals
    assert len(cache.read_text().splitlines()) == 1
    ctx.close()


def test_uneven_environments_match_the_oracle(torch, envs):
    """One step of the uneven-environment workload (about 2e5 pairs) under the schedule the autotuner picks
    for it: index sets (locc_debug_crop) and member counts of every pair bit for bit against the oracle's
    crop, and the contacts of a seeded sample of 160 pairs within the BF16 bounds of the FP64 oracle."""
    sc = envs.scene(1)
    w = _weights()
    say(f"uneven environments: {sc.n_pairs} pairs, every crop against the oracle")
    ctx = B.context_for_scene(sc, 128, SCALE, w, precision="bf16")
    objs, pairs = B.scene_tensors(sc)
    best, _ = ctx.autotune(objs, pairs, want_counts=False)
    say(f"  autotuned schedule {best}")
    out, counts = ctx.detect(objs, pairs)
    idx, counts2 = ctx.debug_crop(objs, pairs)
    torch.cuda.synchronize()
    out, counts, idx, counts2 = (t.cpu().numpy() for t in (out, counts, idx, counts2))
    assert ctx.device_errors() == 0
    ctx.close()
    ridx, rcounts = oracle_crop_all(sc, 128, workers=8)
    np.testing.assert_array_equal(counts, rcounts)
    np.testing.assert_array_equal(counts2, rcounts)
    np.testing.assert_array_equal(idx, ridx)
    del idx, ridx
    rows = np.sort(np.random.default_rng(9).choice(sc.n_pairs, 160, replace=False))
    ref = O.detect_scene(sc, w, SCALE, 128, rows=rows)
    model = Q.bf16_detect(ref["geoms"], w, SCALE)
    check_low_precision(out[rows], model["contacts"], ref["contacts"], 2e-2, 5e-3, "uneven environments", say)
