"""Shared test helpers: constructed-weight networks, sphere scenes and error metrics."""

import json
import multiprocessing as mp
import os

import numpy as np

from paper_2304_09439_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

FIELDS = {"logit": slice(0, 1), "point": slice(1, 4), "normal": slice(4, 7), "depth": slice(7, 8)}


def sphere_cases():
    with open(os.path.join(GOLDEN, "sphere_contact_cases.json")) as f:
        return json.load(f)["cases"]


def sphere_probe_weights(widths: I.Widths, beta: float = 4.0):
    """Weights under which the network computes the sphere-sphere contact exactly.

    Encoder: unit 0 = ReLU(x + 1), unit 1 = ReLU(1 - x), passed through layer 2,
    so the per-object max-pool gives (1 + max x, 1 - min x) over the crop.
    Head: g0 = f_a[0] = 1 + max_a x, g1 = f_b[1] = 1 - min_b x, and
      logit = beta (g0 + g1 - 2), point_x = (g0 - g1) / 2, normal = (1, 0, 0),
      depth = g0 + g1 - 2 = max_a x - min_b x.
    For spheres on the x axis with both x-poles in the crop that is
    ra + rb - d and (ra + d - rb) / 2.
    Three more units have negative pre-activations (ReLU(-x - 1),
    ReLU(-f_a[0]), ReLU(-g1[0])) and feed the outputs, so a missing hidden
    ReLU changes point_x or point_y.
    """
    h1, h2, hh = widths.h1, widths.h2, widths.hh
    W1 = np.zeros((h1, 6), np.float32); b1 = np.zeros(h1, np.float32)
    W1[0, 0], b1[0] = 1, 1
    W1[1, 0], b1[1] = -1, 1
    W1[2, 0], b1[2] = -1, -1
    W2 = np.zeros((h2, h1), np.float32); b2 = np.zeros(h2, np.float32)
    W2[0, 0] = W2[1, 1] = 1
    W2[0, 2] = 1
    H1 = np.zeros((hh, 2 * h2), np.float32); c1 = np.zeros(hh, np.float32)
    H1[0, 0] = 1
    H1[1, h2 + 1] = 1
    H1[2, 0] = -1
    H2 = np.zeros((hh, hh), np.float32); c2 = np.zeros(hh, np.float32)
    H2[0, 0] = H2[1, 1] = 1
    H2[0, 2] = 1
    H2[2, 0] = -1
    H3 = np.zeros((8, hh), np.float32); c3 = np.zeros(8, np.float32)
    H3[0, :2], c3[0] = beta, -2 * beta
    H3[1, :2] = 0.5, -0.5
    H3[2, 2] = 1
    c3[4] = 1
    H3[7, :2], c3[7] = 1, -2
    return I.flatten_weights([W1, b1, W2, b2, H1, c1, H2, c2, H3, c3])


def sphere_case_scene(cases, n_points=1024, seed=5, swap_every_other=True):
    """One pair per case: sphere a at the origin (identity), sphere b at (d, 0, 0)
    turned by theta about x (its x-poles stay on the axis exactly)."""
    rng = np.random.default_rng(seed)
    radii = []
    for c in cases:
        radii += [c["ra"], c["rb"]]
    lib = I.sphere_library(rng, len(radii), n_points, radii)
    n = len(cases)
    pos = np.zeros((2 * n, 3), np.float32)
    quat = np.zeros((2 * n, 4), np.float32)
    quat[:, 0] = 1
    for k, c in enumerate(cases):
        pos[2 * k + 1, 0] = c["d"]
        th = c["theta"]
        quat[2 * k + 1] = [np.cos(th / 2), np.sin(th / 2), 0, 0]
    pairs = np.stack([2 * np.arange(n), 2 * np.arange(n) + 1], axis=1).astype(np.int32)
    if swap_every_other:
        pairs[1::2] = pairs[1::2, ::-1]
    return I.Scene(lib, pos, quat, np.arange(2 * n, dtype=np.int32), pairs)


def pair_errors(out: np.ndarray, ref: np.ndarray) -> dict:
    """Per-field relative error of every pair: |y_f - ref_f| / max(|ref_f|, RMS over the pairs of |ref_f|)."""
    errs = {}
    for name, sl in FIELDS.items():
        d = np.linalg.norm(np.asarray(out, np.float64)[:, sl] - ref[:, sl], axis=1)
        r = np.linalg.norm(ref[:, sl], axis=1)
        rms = np.sqrt(np.mean(r ** 2)) if len(r) else 1.0
        errs[name] = d / np.maximum(r, max(rms, 1e-30))
    return errs


def field_errors(out: np.ndarray, ref: np.ndarray) -> dict:
    """Per-field relative error: max over pairs of |y_f - ref_f| / max(|ref_f|, RMS |ref_f|)."""
    return {k: float(v.max()) if len(v) else 0.0 for k, v in pair_errors(out, ref).items()}


def check_low_precision(got: np.ndarray, model: np.ndarray, ref: np.ndarray, normwise_tol: float,
                        model_tol: float, label: str, say=print):
    """Kernel outputs `got` against the FP64 oracle `ref` and the CPU model of the same rounding decisions
    `model`, per field, on the same pairs:
      * normwise ||got_f - ref_f|| / ||ref_f|| < normwise_tol;
      * every pair within 1.5 x the model's largest per-pair error against the oracle + 2e-3 (the tail of
        the format's own error, measured without the kernel, bounds each pair);
      * normwise ||got_f - model_f|| / ||model_f|| < model_tol (the kernel takes the model's rounding
        decisions, up to the order of its float32 sums).
    Returns the per-field bounds used."""
    ny = normwise_errors(got, ref)
    pe_got, pe_model = pair_errors(got, ref), pair_errors(model, ref)
    nm = normwise_errors(got, model)
    bounds = {k: 1.5 * float(pe_model[k].max(initial=0.0)) + 2e-3 for k in FIELDS}
    fmt = lambda d: "{" + ", ".join(f"{k} {v:.2e}" for k, v in d.items()) + "}"
    say(f"  {label}: vs oracle normwise {fmt(ny)}, per-pair max {fmt({k: v.max(initial=0) for k, v in pe_got.items()})}"
        f"; model per-pair max {fmt({k: v.max(initial=0) for k, v in pe_model.items()})}; vs model normwise {fmt(nm)}")
    for k in FIELDS:
        assert ny[k] < normwise_tol, (label, k, ny[k])
        worst = int(np.argmax(pe_got[k])) if len(pe_got[k]) else 0
        assert np.all(pe_got[k] <= bounds[k]), (label, k, "pair", worst, pe_got[k][worst], "bound", bounds[k])
        assert nm[k] < model_tol, (label, k, nm[k])
    return bounds


def normwise_errors(out: np.ndarray, ref: np.ndarray) -> dict:
    """Per-field normwise relative error over all pairs: ||y_f - ref_f||_F / ||ref_f||_F."""
    errs = {}
    for name, sl in FIELDS.items():
        d = np.linalg.norm(np.asarray(out, np.float64)[:, sl] - ref[:, sl])
        r = np.linalg.norm(ref[:, sl])
        errs[name] = float(d / max(r, 1e-30))
    return errs


def flag_agreement(logit_out, logit_ref, band: float = 0.0):
    """Fraction of pairs whose (logit > 0) agrees; pairs with |ref| < band * RMS(ref) excluded."""
    logit_out = np.asarray(logit_out, np.float64).ravel()
    logit_ref = np.asarray(logit_ref, np.float64).ravel()
    keep = np.abs(logit_ref) >= band * np.sqrt(np.mean(logit_ref ** 2))
    if not keep.any():
        return 1.0
    return float(np.mean((logit_out[keep] > 0) == (logit_ref[keep] > 0)))



def first_object_empty(pairs: np.ndarray, counts: np.ndarray) -> np.ndarray:
    """Rows of pairs whose first object in canonical order (the lower index) selects no point while
    the second selects some; counts are in the caller's order."""
    i, j = pairs[:, 0], pairs[:, 1]
    first = np.where(i < j, counts[:, 0], counts[:, 1])
    second = np.where(i < j, counts[:, 1], counts[:, 0])
    return np.flatnonzero((first == 0) & (second > 0))


def with_first_object_empty(base: "I.Scene", n: int, every: int = 16, seed: int = 11):
    """base plus n pairs whose first object in canonical order selects nothing: a sphere of radius
    0.5 (the lower object index) and a sphere of radius 0.03 centred at (0.4, 0.4, 0.4) in the large
    sphere's frame.  The crop box (the small sphere's box, padded, inside the large sphere's box)
    lies at distance > 0.5 from the large sphere's centre, so it holds every point of the small
    sphere and none of the large one's surface.  Random common orientations; every other pair is
    given in reversed order.  The new pairs are placed at every `every`-th position among base's.
    Returns (Scene, rows of the new pairs)."""
    rng = np.random.default_rng(seed)
    n_pts = int(base.lib.offsets[1] - base.lib.offsets[0])
    sph = I.sphere_library(rng, 2, n_pts, radii=[0.5, 0.03])
    lib = I.ShapeLibrary.concat([base.lib, sph])
    big, small = base.lib.n_shapes, base.lib.n_shapes + 1
    q = I.uniform_quaternions(rng, n).astype(np.float64)
    w, v = q[:, :1], q[:, 1:]
    c = np.array([0.4, 0.4, 0.4])
    # R(q) c = c + 2 w (v x c) + 2 v x (v x c)
    vc = np.cross(v, c)
    off = c + 2 * w * vc + 2 * np.cross(v, vc)
    pa = rng.uniform(-5, 5, (n, 3))
    n0 = base.n_objects
    pos = np.concatenate([base.pos, np.repeat(pa, 2, 0).astype(np.float32)])
    pos[n0 + 1::2] = (pa + off).astype(np.float32)
    quat = np.concatenate([base.quat, np.repeat(q, 2, 0).astype(np.float32)])
    shape = np.concatenate([base.shape, np.tile([big, small], n).astype(np.int32)])
    new = np.stack([n0 + 2 * np.arange(n), n0 + 2 * np.arange(n) + 1], 1).astype(np.int32)
    new[1::2] = new[1::2, ::-1]
    P = base.n_pairs + n
    rows = np.arange(n) * every
    assert rows[-1] < P
    pairs = np.empty((P, 2), np.int32)
    mask = np.zeros(P, bool)
    mask[rows] = True
    pairs[mask] = new
    pairs[~mask] = base.pairs[:P - n]
    return I.Scene(lib, pos, quat, shape, pairs), rows


# ---------------------------------------------------------------- oracle crop over a process pool

_POOL_SCENE = {}


def _crop_chunk(rows):
    from oracle import locc_oracle as O
    s = _POOL_SCENE
    _, idx, counts = O.crop(s["pts"], s["offsets"], s["pos"], s["quat"], s["shape"], s["pairs"][rows], s["K"])
    return idx, counts


def oracle_crop_all(scene, K, workers=None):
    """The oracle's crop (O1-O7: index sets and member counts, no network) of every pair of `scene`, in
    chunks over a fork pool of worker processes (at most 16).  Returns idx [P, 2, K], counts [P, 2]."""
    _POOL_SCENE.update(pts=scene.lib.pts, offsets=scene.lib.offsets, pos=scene.pos, quat=scene.quat,
                       shape=scene.shape, pairs=scene.pairs, K=K)
    P = scene.n_pairs
    workers = workers or max(1, min(16, len(os.sched_getaffinity(0))))
    chunks = [c for c in np.array_split(np.arange(P), max(1, min(P, workers * 8))) if len(c)]
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_crop_chunk, chunks)
    _POOL_SCENE.clear()
    if not parts:
        return np.zeros((0, 2, K), np.int32), np.zeros((0, 2), np.int32)
    return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])
