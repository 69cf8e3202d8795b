"""GPU parity of the voxel-embedding variant (include/locc_voxel.h) against the
float64 oracle of oracle.voxel_locc.

Tolerances (float32 kernels against float64): a float32 dot product of n
terms carries a relative error of about u sqrt(n) times its condition number
(u = 2^-24); the longest sum here has n = 6,912 (the first convolution), and
with a condition number up to 20 over ten layers that is about 1e-4.  So
embeddings, mean embeddings, logits and probabilities are compared normwise
(per shape, or over the pairs) at 1e-4.  The cell selection is a float64
decision taken in the same order on both sides, so the selected-cell counts
are compared exactly."""

import sys

import numpy as np
import pytest

from oracle import voxel_locc as V
from paper_2304_09439_amd import binding as B
from paper_2304_09439_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-4


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
def setup():
    """8 shapes of the 2048-point library, He weights with N(0, 0.1^2) biases, oracle embeddings."""
    lib = I.scale_library(n_shapes=8)
    w = I.flatten_weights(I.voxel_weights(seed=0, bias_std=0.1))
    emb = V.library_embeddings(lib.pts, lib.offsets, w)
    return lib, w, emb


def _ctx(lib, w):
    ctx = B.VoxelContext()
    ctx.upload_weights(w)
    ctx.upload_shapes(lib.offsets, lib.pts)
    return ctx


def _normwise(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def test_shape_embeddings_match_the_oracle(torch, setup):
    lib, w, emb = setup
    ctx = _ctx(lib, w)
    E = ctx.embeddings().cpu().numpy()
    torch.cuda.synchronize()
    errs = [_normwise(E[s], emb[s]) for s in range(lib.n_shapes)]
    say(f"embedding normwise errors {['%.2e' % e for e in errs]}")
    assert max(errs) < TOL
    # uploading the shapes before the weights gives the same embeddings
    ctx2 = B.VoxelContext()
    ctx2.upload_shapes(lib.offsets, lib.pts)
    with pytest.raises(B.LoccError):
        ctx2.embeddings()                                  # no weights yet
    ctx2.upload_weights(w)
    assert torch.equal(ctx2.embeddings(), ctx.embeddings())
    ctx.close()
    ctx2.close()


def test_ragged_and_degenerate_shapes_match_the_oracle(torch, setup):
    """Point counts off the encoder's 64-point tiles (1, 63, 64, 65, 130, 777, 2048) and a shape whose
    points all coincide (zero extent: every point in cell 0), against the oracle's embeddings."""
    lib, w, _ = setup
    counts = [1, 63, 64, 65, 130, 777, 2048, 40]
    clouds = [lib.pts[lib.offsets[s]:lib.offsets[s] + n] for s, n in enumerate(counts)]
    clouds[-1] = np.repeat(lib.pts[lib.offsets[7]:lib.offsets[7] + 1], counts[-1], axis=0)
    pts = np.concatenate(clouds).astype(np.float32)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    ref = V.library_embeddings(pts, offsets, w)
    ctx = B.VoxelContext()
    ctx.upload_weights(w)
    ctx.upload_shapes(offsets, pts)
    E = ctx.embeddings().cpu().numpy()
    torch.cuda.synchronize()
    errs = [_normwise(E[s], ref[s]) for s in range(len(counts))]
    say(f"ragged embedding normwise errors {['%.2e' % e for e in errs]}")
    assert max(errs) < TOL
    ctx.close()


def _scene(lib, n_objs=64, n_pairs=3000, seed=21, spread=0.06):
    rng = np.random.default_rng(seed)
    pos = (rng.standard_normal((n_objs, 3)) * spread).astype(np.float32)
    quat = I.uniform_quaternions(rng, n_objs).astype(np.float32)
    shape = rng.integers(0, lib.n_shapes, n_objs).astype(np.int32)
    i = rng.integers(0, n_objs, n_pairs)
    j = (i + 1 + rng.integers(0, n_objs - 1, n_pairs)) % n_objs
    pairs = np.stack([i, j], axis=1).astype(np.int32)
    pairs[5] = [3, 3]                       # i == j
    pairs[17] = [2, n_objs + 4]             # out of range
    shape[9] = lib.n_shapes                 # shape id out of range
    pos[60] = [4.0, 0.0, 0.0]               # far from everything: no cell selected
    pairs[40] = [60, 1]
    return pos, quat, shape, pairs


@pytest.mark.parametrize("n_pairs", [3000, 31, 1])
def test_pairs_match_the_oracle(torch, setup, n_pairs):
    lib, w, emb = setup
    pos, quat, shape, pairs = _scene(lib)
    pairs = pairs[:n_pairs] if n_pairs < len(pairs) else pairs
    say(f"voxel pairs: {len(pairs)} pairs (ragged tile tail {len(pairs) % 32})")
    ref = V.detect(lib.pts, lib.offsets, pos, quat, shape, pairs, w, emb=emb)
    ctx = _ctx(lib, w)
    objs = torch.from_numpy(B.pack_objects(pos, quat, shape)).cuda()
    pr = torch.from_numpy(pairs).cuda()
    out, counts, pooled = ctx.detect(objs, pr, want_pooled=True)
    torch.cuda.synchronize()
    out, counts, pooled = out.cpu().numpy(), counts.cpu().numpy(), pooled.cpu().numpy()
    np.testing.assert_array_equal(counts, ref["counts"])
    bad = np.isnan(ref["logit"])
    assert np.array_equal(np.isnan(out[:, 0]), bad) and np.array_equal(np.isnan(out[:, 1]), bad)
    ok = ~bad
    if ok.sum() == 0:
        ctx.close()
        return
    e_pool = _normwise(pooled[ok], ref["pooled"][ok])
    e_logit = _normwise(out[ok, 0], ref["logit"][ok])
    e_prob = _normwise(out[ok, 1], ref["prob"][ok])
    say(f"  normwise: pooled {e_pool:.2e}, logit {e_logit:.2e}, prob {e_prob:.2e}; "
        f"{int((ref['counts'][ok] == 0).all(axis=1).sum())} pairs with no cell")
    assert e_pool < TOL and e_logit < TOL and e_prob < TOL
    assert ctx.device_errors() == int(bad.sum())
    ctx.close()


def test_swapped_pairs_and_batch_invariance(torch, setup):
    lib, w, _ = setup
    pos, quat, shape, pairs = _scene(lib, n_pairs=700, seed=22)
    ctx = _ctx(lib, w)
    objs = torch.from_numpy(B.pack_objects(pos, quat, shape)).cuda()
    out, counts, _ = ctx.detect(objs, torch.from_numpy(pairs).cuda())
    out_s, counts_s, _ = ctx.detect(objs, torch.from_numpy(np.ascontiguousarray(pairs[:, ::-1])).cuda())
    sub = np.arange(3, 700, 7)
    out_b, counts_b, _ = ctx.detect(objs, torch.from_numpy(pairs[sub]).cuda())
    torch.cuda.synchronize()
    assert torch.equal(out.isnan(), out_s.isnan())
    ok = ~out[:, 0].isnan()
    assert torch.equal(out[ok], out_s[ok])                    # the caller's order does not matter
    assert torch.equal(counts, counts_s.flip(1))              # counts follow the caller's order
    assert torch.equal(out[sub][ok[sub]], out_b[ok[sub]]) and torch.equal(counts[sub], counts_b)
    ctx.close()


def test_upload_and_argument_errors(torch, setup):
    lib, w, _ = setup
    ctx = B.VoxelContext()
    with pytest.raises(B.LoccError):
        ctx.upload_weights(w[:-1])
    bad = w.copy()
    bad[7] = np.nan
    with pytest.raises(B.LoccError):
        ctx.upload_weights(bad)
    off = np.array([0, 10, 10], np.int64)
    with pytest.raises(B.LoccError):
        ctx.upload_shapes(off, lib.pts[:10])                  # empty shape
    objs = torch.zeros((2, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(B.LoccError):
        ctx.detect(objs, torch.zeros((1, 2), dtype=torch.int32, device="cuda"))   # nothing uploaded
    ctx.upload_weights(w)
    ctx.upload_shapes(lib.offsets, lib.pts)
    out, _, _ = ctx.detect(objs, torch.zeros((0, 2), dtype=torch.int32, device="cuda"))
    assert out.shape == (0, 2)
    ctx.close()
