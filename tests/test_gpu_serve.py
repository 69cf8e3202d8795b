"""Serving: continuous batching over resident environments (locc_serve_*).

Each request updates the poses of the environments it covers and asks for
their broad-phase pairs; its served result must be bitwise the result of
running it alone on a table holding its own poses, whatever else was in the
batch or in flight.
"""

import sys
import time

import numpy as np
import pytest

from oracle import locc_oracle as O
from oracle import quant_model as Q
from paper_2304_09439_amd import binding as B
from paper_2304_09439_amd import inputs as I

from helpers import check_low_precision

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
def rs():
    lib = I.shape_library(np.random.default_rng(2), 8, 2048, (3, 6), 0.5)
    return I.request_stream(n_requests=300, lib=lib, n_envs=256, versions=3, max_pairs=600)


def _ctx(rs, precision):
    ctx = B.Context(128, SCALE, precision=precision)
    ctx.upload_shapes(rs.lib.offsets, rs.lib.pts)
    ctx.upload_weights(I.flatten_weights(I.gaussian_weights(LW, seed=0, bias_std=0.1)))
    return ctx


def _table(rs):
    return B.pack_objects(rs.pos0, rs.quat0, rs.shape)


def _upd(rs, req):
    ids, pos, quat, pairs = req
    return ids, B.pack_objects(pos, quat, rs.shape[ids]), pairs


def _alone(torch, ctx, rs, req):
    ids, upd, pairs = _upd(rs, req)
    table = _table(rs)
    table[ids] = upd
    out, counts = ctx.detect(torch.from_numpy(table).cuda(), torch.from_numpy(np.ascontiguousarray(pairs)).cuda())
    torch.cuda.synchronize()
    return out.cpu().numpy(), counts.cpu().numpy()


def _drain(srv, ids, timeout_s=60.0):
    res, t0 = {}, time.time()
    pending = list(ids)
    while pending:
        assert time.time() - t0 < timeout_s, "requests did not complete"
        left = []
        for rid in pending:
            r = srv.poll(rid)
            if r is None:
                left.append(rid)
            else:
                res[rid] = r
        pending = left
    return res


@pytest.mark.parametrize("precision,batching", [("bf16", True), ("fp32", False)])
def test_served_results_equal_the_request_run_alone(torch, rs, precision, batching):
    n = 300 if batching else 60
    say(f"serving {precision}, batching={batching}: {n} requests in a burst")
    ctx = _ctx(rs, precision)
    srv = B.Server(ctx, _table(rs), batching=batching, slots=3, max_batch_pairs=4096, max_batch_updates=8192,
                   hbm_budget_bytes=2 << 30)
    ids = [srv.submit(*_upd(rs, rs.requests[k])) for k in range(n)]
    res = _drain(srv, ids)
    st = srv.stats()
    srv.stop()
    say(f"  stats {st}")
    assert st["completed"] == n and st["submitted"] == n
    assert st["pairs_done"] == sum(len(rs.requests[k][3]) for k in range(n))
    if batching:
        assert st["batches"] < n            # requests really were batched together
    else:
        assert st["batches"] == n
    for k in np.random.default_rng(1).choice(n, 25, replace=False):
        out, counts, lat = res[ids[k]]
        ref_out, ref_counts = _alone(torch, ctx, rs, rs.requests[k])
        np.testing.assert_array_equal(out, ref_out)
        np.testing.assert_array_equal(counts, ref_counts)
        assert lat > 0
    assert ctx.device_errors() == 0
    ctx.close()


def test_submit_many_queues_in_order_and_stops_at_the_first_refusal(torch, rs):
    """locc_serve_submit_many: one call queues the requests in order (ids ascending), their results equal
    the requests run alone; against a queue limit it queues the longest prefix that fits (the call holds
    the queue's lock, so the worker cannot drain it meanwhile) and reports BUSY with the ids queued."""
    n = 300
    say(f"serving bf16: {n} requests in one submit_many call")
    ctx = _ctx(rs, "bf16")
    srv = B.Server(ctx, _table(rs), batching=True, slots=3, max_batch_pairs=4096, max_batch_updates=8192,
                   hbm_budget_bytes=2 << 30)
    reqs = [_upd(rs, rs.requests[k]) for k in range(n)]
    ids = srv.submit_many(reqs)
    assert len(ids) == n and ids == sorted(ids) and len(set(ids)) == n
    res = _drain(srv, ids)
    st = srv.stats()
    srv.stop()
    assert st["completed"] == n and st["batches"] < n
    for k in np.random.default_rng(2).choice(n, 20, replace=False):
        out, counts, _ = res[ids[k]]
        ref_out, ref_counts = _alone(torch, ctx, rs, rs.requests[k])
        np.testing.assert_array_equal(out, ref_out)
        np.testing.assert_array_equal(counts, ref_counts)
    limit = 1000
    srv = B.Server(ctx, _table(rs), batching=True, slots=1, max_batch_pairs=4096, max_batch_updates=8192,
                   max_queued_pairs=limit, hbm_budget_bytes=2 << 30)
    sizes = np.cumsum([len(r[2]) for r in reqs])
    fit = int(np.searchsorted(sizes, limit, side="right"))   # the longest prefix within the limit
    assert 0 < fit < n
    with pytest.raises(B.LoccError) as e:
        srv.submit_many(reqs)
    assert e.value.status == B.ERR_BUSY and len(e.value.accepted_ids) == fit
    res = _drain(srv, e.value.accepted_ids)
    srv.stop()
    out, counts, _ = res[e.value.accepted_ids[-1]]
    ref_out, ref_counts = _alone(torch, ctx, rs, rs.requests[fit - 1])
    np.testing.assert_array_equal(out, ref_out)
    np.testing.assert_array_equal(counts, ref_counts)
    assert ctx.device_errors() == 0
    ctx.close()


def test_requests_on_the_same_environment_see_their_own_poses(torch, rs):
    ctx = _ctx(rs, "bf16")
    srv = B.Server(ctx, _table(rs), batching=True, slots=2, max_batch_pairs=4096, max_batch_updates=8192)
    first = rs.requests[0]
    ids0, _, _, pairs0 = first
    # a second request on the same objects with other poses (a later version of the same step)
    other = next(r for r in rs.requests[1:] if np.array_equal(np.sort(r[0]), np.sort(ids0)))  \
        if any(np.array_equal(np.sort(r[0]), np.sort(ids0)) for r in rs.requests[1:]) else None
    rng = np.random.default_rng(4)
    if other is None:
        pos = first[1] + rng.normal(0, 0.003, first[1].shape).astype(np.float32)
        other = (ids0, pos, first[2], pairs0)
    r1 = srv.submit(*_upd(rs, first))
    r2 = srv.submit(*_upd(rs, other))
    res = _drain(srv, [r1, r2])
    srv.stop()
    for rid, req in ((r1, first), (r2, other)):
        ref_out, ref_counts = _alone(torch, ctx, rs, req)
        np.testing.assert_array_equal(res[rid][0], ref_out)
        np.testing.assert_array_equal(res[rid][1], ref_counts)
    ctx.close()


def test_admission_limits(torch, rs):
    ctx = _ctx(rs, "bf16")
    with pytest.raises(B.LoccError) as e:
        B.Server(ctx, _table(rs), hbm_budget_bytes=1 << 16)
    assert e.value.status == B.ERR_OOM
    srv = B.Server(ctx, _table(rs), max_batch_pairs=50, max_queued_pairs=30)
    big = next(r for r in rs.requests if len(r[3]) > 50)
    with pytest.raises(B.LoccError) as e:
        srv.submit(*_upd(rs, big))
    assert e.value.status == B.ERR_RANGE
    mid = next(r for r in rs.requests if 30 < len(r[3]) <= 50)
    with pytest.raises(B.LoccError) as e:
        srv.submit(*_upd(rs, mid))
    assert e.value.status == B.ERR_BUSY
    small = next(r for r in rs.requests if len(r[3]) <= 30)
    rid = srv.submit(*_upd(rs, small))
    _drain(srv, [rid])
    srv.stop()
    ctx.close()


def test_poisson_stream_reports_latencies(torch, rs):
    ctx = _ctx(rs, "bf16")
    srv = B.Server(ctx, _table(rs), batching=True, slots=2, max_batch_pairs=8192, max_batch_updates=16384)
    rng = np.random.default_rng(7)
    arrivals = np.cumsum(rng.exponential(1.0 / 2000.0, 200))
    t0 = time.perf_counter()
    ids = []
    for k, a in enumerate(arrivals):
        while time.perf_counter() - t0 < a:
            pass
        ids.append(srv.submit(*_upd(rs, rs.requests[k])))
    res = _drain(srv, ids)
    srv.stop()
    lat = np.array([res[i][2] for i in ids])
    say(f"  200 requests at 2000/s: p50 {np.percentile(lat, 50):.3f} ms, p99 {np.percentile(lat, 99):.3f} ms")
    assert np.all(lat > 0) and np.percentile(lat, 50) < 1000
    ctx.close()


def test_waiting_requests_are_overtaken_only_on_disjoint_objects(torch, rs):
    """Two versions of each of 40 requests on disjoint objects, submitted version after version: a
    second version conflicts with its first (same objects) and must wait for it, while the other
    requests may join the batch past it.  With one slot, strict first-in-first-out batches would
    hold one environment change each (at least 40 batches); every result equals the request run
    alone on its own poses."""
    ctx = _ctx(rs, "bf16")
    srv = B.Server(ctx, _table(rs), batching=True, slots=1, max_batch_pairs=16384, max_batch_updates=16384)
    used, envs = set(), []   # 40 requests on pairwise disjoint objects
    for req in rs.requests:
        objs = set(req[0].tolist()) | set(np.asarray(req[3]).ravel().tolist())
        if not objs & used:
            used |= objs
            envs.append(req)
        if len(envs) == 40:
            break
    assert len(envs) == 40
    rng = np.random.default_rng(7)
    reqs = []
    for req in envs:
        ids, pos, quat, pairs = req
        reqs.append(req)
        reqs.append((ids, pos + rng.normal(0, 0.003, pos.shape).astype(np.float32), quat, pairs))
    ids = [srv.submit(*_upd(rs, r)) for r in reqs]
    res = _drain(srv, ids)
    st = srv.stats()
    srv.stop()
    say(f"  {len(reqs)} requests in {st['batches']} batches")
    assert st["completed"] == len(reqs) and st["batches"] < 20
    for rid, req in zip(ids, reqs):
        ref_out, ref_counts = _alone(torch, ctx, rs, req)
        np.testing.assert_array_equal(res[rid][0], ref_out)
        np.testing.assert_array_equal(res[rid][1], ref_counts)
    ctx.close()


def test_served_results_match_the_oracle_on_the_serving_library(torch):
    """The serving workload's own library (128 shapes x 4096 points, 4096 resident environments): a burst of
    120 requests served with continuous batching; for 6 sampled requests (their first 150 pairs) the member
    counts equal the FP64 oracle's bit for bit and the contacts are within the BF16 bounds of the oracle
    on each request's own poses."""
    rs = I.request_stream(n_requests=120)
    say(f"serving library: {rs.lib.n_shapes} shapes x {int(rs.lib.offsets[1])} points, "
        f"{len(rs.shape)} resident objects, 120 requests")
    w = I.flatten_weights(I.gaussian_weights(LW, seed=0, bias_std=0.0))
    ctx = B.Context(128, SCALE, precision="bf16")
    ctx.upload_shapes(rs.lib.offsets, rs.lib.pts)
    ctx.upload_weights(w)
    srv = B.Server(ctx, _table(rs), batching=True, slots=3, max_batch_pairs=32768, max_batch_updates=65536,
                   hbm_budget_bytes=4 << 30)
    ids = [srv.submit(*_upd(rs, r)) for r in rs.requests]
    res = _drain(srv, ids, timeout_s=120.0)
    st = srv.stats()
    srv.stop()
    assert st["completed"] == len(ids) and st["batches"] < len(ids)
    assert ctx.device_errors() == 0
    ctx.close()
    outs, refs, models = [], [], []
    for k in np.random.default_rng(3).choice(len(ids), 6, replace=False):
        upd_ids, pos, quat, pairs = rs.requests[k]
        P = min(150, len(pairs))
        gpos, gquat = rs.pos0.copy(), rs.quat0.copy()
        gpos[upd_ids], gquat[upd_ids] = pos, quat
        ref = O.detect(rs.lib.pts, rs.lib.offsets, gpos, gquat, rs.shape, pairs[:P], w, SCALE, 128)
        out, counts, _ = res[ids[k]]
        np.testing.assert_array_equal(counts[:P], ref["counts"])
        outs.append(out[:P])
        refs.append(ref["contacts"])
        models.append(Q.bf16_detect(ref["geoms"], w, SCALE)["contacts"])
    check_low_precision(np.concatenate(outs), np.concatenate(models), np.concatenate(refs), 2e-2, 5e-3,
                        "served vs oracle (4096-point shapes)", say)
