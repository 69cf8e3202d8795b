"""Seeded synthetic inputs for the LOCC crop-collision path.

This module only draws inputs: procedural non-convex shapes sampled on their
surfaces, sphere shapes, rigid poses, object pairs, environments, request
streams and network weights.  It holds none of the method's arithmetic (no
crop box, no membership test, no network); both the HIP library and the CPU
oracle consume what it returns.

The paper trains and tests on household-object meshes (Google Scanned Objects,
YCB, EGAD; Sec. IV) with K=1500 surface points per object (Sec. III).  None of
those datasets or trained weights is available here, so procedural shapes of
the same physical scale (components of 0.02-0.08 m semi-axes) stand in for
them, with 1024/2048/4096 stored points and Gaussian-initialised weights.

Every generator is deterministic in its seed.  A workload's master seed is
split with ``numpy.random.SeedSequence(master).spawn(5)`` into the streams
[shapes, poses, spheres/environments, calibration, requests]; weights always
come from ``numpy.random.default_rng(seed)`` on their own.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial.transform import Rotation

STREAM_SHAPES, STREAM_POSES, STREAM_ENVS, STREAM_CALIB, STREAM_REQUESTS = range(5)


def streams(master: int):
    """Five independent generators split from one master seed."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(master).spawn(5)]


# ----------------------------------------------------------------------------
# shapes
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class ShapeLibrary:
    """Surface point clouds of S shapes, concatenated.

    pts     float32 [sum N_s, 6]: x, y, z, nx, ny, nz in the shape's own frame
    offsets int64   [S + 1]: shape s owns rows offsets[s]:offsets[s+1]
    radius  float32 [S]: sphere radius for sphere shapes, NaN otherwise
    """
    pts: np.ndarray
    offsets: np.ndarray
    radius: np.ndarray

    @property
    def n_shapes(self) -> int:
        return len(self.offsets) - 1

    def shape_points(self, s: int) -> np.ndarray:
        return self.pts[self.offsets[s]:self.offsets[s + 1]]

    @staticmethod
    def concat(libs) -> "ShapeLibrary":
        pts = np.concatenate([lb.pts for lb in libs])
        counts = np.concatenate([np.diff(lb.offsets) for lb in libs])
        offsets = np.zeros(len(counts) + 1, np.int64)
        np.cumsum(counts, out=offsets[1:])
        return ShapeLibrary(pts, offsets, np.concatenate([lb.radius for lb in libs]))


def uniform_quaternions(rng, n: int) -> np.ndarray:
    """Uniform random rotations (Shoemake's subgroup algorithm), (w, x, y, z), float64."""
    u1, u2, u3 = rng.random((3, n))
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    t2, t3 = 2.0 * np.pi * u2, 2.0 * np.pi * u3
    return np.stack([b * np.cos(t3), a * np.sin(t2), a * np.cos(t2), b * np.sin(t3)], axis=1)


def _scipy_rot(q_wxyz: np.ndarray) -> Rotation:
    q = np.asarray(q_wxyz, np.float64)
    return Rotation.from_quat(np.concatenate([q[..., 1:], q[..., :1]], axis=-1))


def _unit_sphere(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


class _Ellipsoid:
    def __init__(self, rng, centre_half_width):
        self.ax = rng.uniform(0.02, 0.08, 3)
        self.c = rng.uniform(-centre_half_width, centre_half_width, 3)
        self.rot = _scipy_rot(uniform_quaternions(rng, 1)[0])
        a, b, c = self.ax
        p = 1.6075  # Knud Thomsen's surface-area approximation
        self.area = 4 * np.pi * (((a * b) ** p + (a * c) ** p + (b * c) ** p) / 3) ** (1 / p)

    def sample(self, rng, n):
        a, b, c = self.ax
        out_p, out_n, have = [], [], 0
        gmax = max(b * c, a * c, a * b)
        while have < n:
            u = _unit_sphere(rng, 2 * n + 16)
            g = np.sqrt((b * c * u[:, 0]) ** 2 + (a * c * u[:, 1]) ** 2 + (a * b * u[:, 2]) ** 2)
            keep = rng.random(len(u)) * gmax <= g  # area-element rejection
            u = u[keep]
            x = u * self.ax
            nrm = x / self.ax ** 2
            nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
            out_p.append(x)
            out_n.append(nrm)
            have += len(x)
        x = np.concatenate(out_p)[:n]
        nrm = np.concatenate(out_n)[:n]
        return self.rot.apply(x) + self.c, self.rot.apply(nrm)

    def strictly_inside(self, p):
        loc = self.rot.inv().apply(p - self.c)
        return np.sum((loc / self.ax) ** 2, axis=1) < 1.0


class _Box:
    def __init__(self, rng, centre_half_width):
        self.h = rng.uniform(0.02, 0.08, 3)
        self.c = rng.uniform(-centre_half_width, centre_half_width, 3)
        self.rot = _scipy_rot(uniform_quaternions(rng, 1)[0])
        hx, hy, hz = self.h
        self.area = 8 * (hx * hy + hy * hz + hx * hz)

    def sample(self, rng, n):
        h = self.h
        face_area = np.array([h[1] * h[2], h[1] * h[2], h[0] * h[2], h[0] * h[2], h[0] * h[1], h[0] * h[1]])
        face = rng.choice(6, size=n, p=face_area / face_area.sum())
        axis, sign = face // 2, np.where(face % 2 == 0, 1.0, -1.0)
        x = rng.uniform(-1.0, 1.0, (n, 3)) * h
        x[np.arange(n), axis] = sign * h[axis]
        nrm = np.zeros((n, 3))
        nrm[np.arange(n), axis] = sign
        return self.rot.apply(x) + self.c, self.rot.apply(nrm)

    def strictly_inside(self, p):
        loc = self.rot.inv().apply(p - self.c)
        return np.all(np.abs(loc) < self.h, axis=1)


def union_shape(rng, n_points: int, n_comp: int, box_fraction: float) -> np.ndarray:
    """Surface samples of a union of ellipsoids and boxes, float32 [n_points, 6].

    A component is picked in proportion to its (approximate) area, a point is
    drawn uniformly on its surface, and the point is dropped if it lies
    strictly inside another component, so only the union's outer surface is
    kept.  Points come out in i.i.d. order.  The cloud is re-centred on its
    axis-aligned bounding-box centre (in float64) before rounding to float32.
    """
    comps = [(_Box if rng.random() < box_fraction else _Ellipsoid)(rng, 0.02) for _ in range(n_comp)]
    areas = np.array([c.area for c in comps])
    pts, nrms, have = [], [], 0
    while have < n_points:
        m = 2 * (n_points - have) + 64
        which = rng.choice(n_comp, size=m, p=areas / areas.sum())
        p = np.empty((m, 3))
        nr = np.empty((m, 3))
        for ci, comp in enumerate(comps):
            sel = which == ci
            if sel.any():
                p[sel], nr[sel] = comp.sample(rng, int(sel.sum()))
        keep = np.ones(m, bool)
        for ci, comp in enumerate(comps):
            others = which != ci
            keep[others] &= ~comp.strictly_inside(p[others])
        pts.append(p[keep])
        nrms.append(nr[keep])
        have += int(keep.sum())
    p = np.concatenate(pts)[:n_points]
    nr = np.concatenate(nrms)[:n_points]
    p -= 0.5 * (p.min(axis=0) + p.max(axis=0))
    nr /= np.linalg.norm(nr, axis=1, keepdims=True)
    return np.concatenate([p, nr], axis=1).astype(np.float32)


def sphere_shape(rng, radius: float, n_points: int) -> np.ndarray:
    """Sphere of the given (float32) radius: the 6 axis poles first, then uniform points."""
    r = float(np.float32(radius))
    poles = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.float64)
    u = np.concatenate([poles, _unit_sphere(rng, n_points - 6)])
    p = np.clip(u * r, -r, r)
    return np.concatenate([p, u], axis=1).astype(np.float32)


def shape_library(rng, n_shapes: int, n_points: int, comp_range=(3, 3), box_fraction=0.0) -> ShapeLibrary:
    clouds = [union_shape(rng, n_points, int(rng.integers(comp_range[0], comp_range[1] + 1)), box_fraction)
              for _ in range(n_shapes)]
    offsets = np.arange(n_shapes + 1, dtype=np.int64) * n_points
    return ShapeLibrary(np.concatenate(clouds), offsets, np.full(n_shapes, np.nan, np.float32))


def sphere_library(rng, n_shapes: int, n_points: int, radii=None) -> ShapeLibrary:
    if radii is None:
        radii = rng.uniform(0.02, 0.08, n_shapes)
    radii = np.asarray(radii, np.float32)
    clouds = [sphere_shape(rng, r, n_points) for r in radii]
    offsets = np.arange(n_shapes + 1, dtype=np.int64) * n_points
    return ShapeLibrary(np.concatenate(clouds), offsets, radii)


# ----------------------------------------------------------------------------
# poses and pairs
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Scene:
    """Objects placed in the world plus the pairs to test.

    pos   float32 [n, 3]   position of the object frame origin
    quat  float32 [n, 4]   orientation, Hamilton quaternion (w, x, y, z)
    shape int32   [n]      index into the shape library
    pairs int32   [P, 2]   (i, j) object indices; order is the caller's
    """
    lib: ShapeLibrary
    pos: np.ndarray
    quat: np.ndarray
    shape: np.ndarray
    pairs: np.ndarray

    @property
    def n_objects(self) -> int:
        return len(self.pos)

    @property
    def n_pairs(self) -> int:
        return len(self.pairs)

    def subset(self, pair_rows) -> "Scene":
        return Scene(self.lib, self.pos, self.quat, self.shape, np.ascontiguousarray(self.pairs[pair_rows]))


def _world_extent(lib: ShapeLibrary, shape: int, q_wxyz) -> tuple[np.ndarray, np.ndarray]:
    """Min / max of the rotated point cloud relative to the object origin."""
    p = _scipy_rot(np.asarray(q_wxyz, np.float64)).apply(lib.shape_points(shape)[:, :3].astype(np.float64))
    return p.min(axis=0), p.max(axis=0)


def overlapping_pair_poses(rng, lib: ShapeLibrary, shape_a, shape_b, spread: float = 1.0):
    """Poses for object pairs whose world-frame bounding boxes overlap.

    Position a is uniform in [-spread, spread]^3, both orientations are
    uniform, and position b is uniform in the box of offsets for which the
    two world-frame bounding boxes of the rotated clouds intersect.
    """
    n = len(shape_a)
    qa = uniform_quaternions(rng, n).astype(np.float32)
    qb = uniform_quaternions(rng, n).astype(np.float32)
    ta = rng.uniform(-spread, spread, (n, 3)).astype(np.float32)
    tb = np.empty_like(ta)
    for k in range(n):
        lo_a, hi_a = _world_extent(lib, int(shape_a[k]), qa[k])
        lo_b, hi_b = _world_extent(lib, int(shape_b[k]), qb[k])
        tb[k] = ta[k] + rng.uniform(lo_a - hi_b, hi_a - lo_b)
    return ta, qa, tb, qb


def _interleave_pairs(rng, n_pairs: int, swap_fraction: float = 0.5) -> np.ndarray:
    """Pairs (2k, 2k+1), each reversed to (2k+1, 2k) with the given probability."""
    pairs = np.stack([2 * np.arange(n_pairs), 2 * np.arange(n_pairs) + 1], axis=1).astype(np.int32)
    swap = rng.random(n_pairs) < swap_fraction
    pairs[swap] = pairs[swap][:, ::-1]
    return pairs


def _pack_pair_scene(lib, ta, qa, tb, qb, sa, sb, pairs):
    n = len(ta)
    pos = np.empty((2 * n, 3), np.float32)
    quat = np.empty((2 * n, 4), np.float32)
    shape = np.empty(2 * n, np.int32)
    pos[0::2], pos[1::2] = ta, tb
    quat[0::2], quat[1::2] = qa, qb
    shape[0::2], shape[1::2] = sa, sb
    return Scene(lib, pos, quat, shape, pairs)


def sphere_pair_poses(rng, radii_a, radii_b, gap_std: float = 0.020):
    """Sphere pairs at centre distance r_a + r_b + g, g ~ N(0, gap_std).

    The gap spread follows the paper's distance manipulation, which draws the
    target separation from a zero-mean normal with 0.020 m deviation
    (Sec. III-A).  Gaps are clipped so the centres stay apart.
    """
    n = len(radii_a)
    ra = np.asarray(radii_a, np.float64)
    rb = np.asarray(radii_b, np.float64)
    gap = np.maximum(rng.normal(0.0, gap_std, n), -0.5 * (ra + rb))
    d = ra + rb + gap
    ta = rng.uniform(-1.0, 1.0, (n, 3))
    tb = ta + _unit_sphere(rng, n) * d[:, None]
    qa = uniform_quaternions(rng, n).astype(np.float32)
    qb = uniform_quaternions(rng, n).astype(np.float32)
    return ta.astype(np.float32), qa, tb.astype(np.float32), qb


def sphere_labels(scene: Scene, rows=None) -> dict:
    """Closed-form sphere-sphere contact for sphere pairs (float64).

    For centres c_i, c_j and radii r_i, r_j at distance d: flag = d < r_i + r_j,
    depth = r_i + r_j - d, normal = (c_j - c_i) / d and contact point
    c_i + normal (r_i + d - r_j) / 2 (midpoint of the two deepest points).
    """
    pairs = scene.pairs if rows is None else scene.pairs[rows]
    i, j = pairs[:, 0], pairs[:, 1]
    ci = scene.pos[i].astype(np.float64)
    cj = scene.pos[j].astype(np.float64)
    ri = scene.lib.radius[scene.shape[i]].astype(np.float64)
    rj = scene.lib.radius[scene.shape[j]].astype(np.float64)
    d = np.linalg.norm(cj - ci, axis=1)
    n = (cj - ci) / d[:, None]
    return dict(flag=d < ri + rj, depth=ri + rj - d, normal=n, point=ci + n * ((ri + d - rj) / 2)[:, None])


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def sphere_training_set(master: int = 5, n_shapes: int = 32, n_points: int = 1024, n_pairs: int = 4096,
                        gap_std: float = 0.020):
    """Labelled sphere pairs for fitting the network: shapes drawn with replacement from a library of
    spheres (radii U[0.02, 0.08] m), centre distance r_a + r_b + g with g ~ N(0, gap_std) (the paper's
    distance manipulation, Sec. III-A), uniform orientations, about half the pairs reversed.
    Returns (Scene, labels float32 [n_pairs]: 1 where the spheres overlap, from the closed form)."""
    g = streams(master)
    lib = sphere_library(g[STREAM_SHAPES], n_shapes, n_points)
    rng = g[STREAM_POSES]
    sa = rng.integers(0, n_shapes, n_pairs).astype(np.int32)
    sb = rng.integers(0, n_shapes, n_pairs).astype(np.int32)
    ta, qa, tb, qb = sphere_pair_poses(rng, lib.radius[sa], lib.radius[sb], gap_std)
    scene = _pack_pair_scene(lib, ta, qa, tb, qb, sa, sb, _interleave_pairs(rng, n_pairs))
    return scene, sphere_labels(scene)["flag"].astype(np.float32)



def small_workload(master: int = 0, n_points: int = 1024, n_nonconvex_pairs: int = 64, n_sphere_pairs: int = 16):
    """Plain, CPU-checkable case: 64 pairs of 3-ellipsoid unions + 16 sphere pairs.

    Object k uses shape k; non-convex pairs join shapes (2k, 2k+1); sphere
    pairs follow them.  Pair order is reversed for about half the pairs.
    """
    g = streams(master)
    ns = 2 * n_nonconvex_pairs
    lib_nc = shape_library(g[STREAM_SHAPES], ns, n_points, (3, 3), 0.0)
    lib_sp = sphere_library(g[STREAM_ENVS], 2 * n_sphere_pairs, n_points)
    lib = ShapeLibrary.concat([lib_nc, lib_sp])
    sa = np.arange(0, ns, 2)
    sb = sa + 1
    ta, qa, tb, qb = overlapping_pair_poses(g[STREAM_POSES], lib, sa, sb)
    spa = ns + np.arange(0, 2 * n_sphere_pairs, 2)
    spb = spa + 1
    sta, sqa, stb, sqb = sphere_pair_poses(g[STREAM_ENVS], lib.radius[spa], lib.radius[spb])
    n = n_nonconvex_pairs + n_sphere_pairs
    pairs = _interleave_pairs(g[STREAM_POSES], n)
    return _pack_pair_scene(lib, np.concatenate([ta, sta]), np.concatenate([qa, sqa]),
                            np.concatenate([tb, stb]), np.concatenate([qb, sqb]),
                            np.concatenate([sa, spa]).astype(np.int32), np.concatenate([sb, spb]).astype(np.int32),
                            pairs)


def scale_library(master: int = 1, n_shapes: int = 32, n_points: int = 2048) -> ShapeLibrary:
    """32 shapes, each a union of 3-6 ellipsoids and boxes (half each on average)."""
    return shape_library(streams(master)[STREAM_SHAPES], n_shapes, n_points, (3, 6), 0.5)


def scale_workload(master: int = 1, n_pairs: int = 16384, n_shapes: int = 32, n_points: int = 2048):
    """At-scale case: pairs of shapes drawn with replacement from a 32-shape library.

    2 * n_pairs objects; pair k joins objects (2k, 2k+1), order reversed for
    about half of the pairs.
    """
    g = streams(master)
    lib = scale_library(master, n_shapes, n_points)
    sa = g[STREAM_POSES].integers(0, n_shapes, n_pairs).astype(np.int32)
    sb = g[STREAM_POSES].integers(0, n_shapes, n_pairs).astype(np.int32)
    ta, qa, tb, qb = overlapping_pair_poses(g[STREAM_POSES], lib, sa, sb)
    pairs = _interleave_pairs(g[STREAM_POSES], n_pairs)
    return _pack_pair_scene(lib, ta, qa, tb, qb, sa, sb, pairs)


# ----------------------------------------------------------------------------
# network weights
# ----------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Widths:
    """Encoder 6 -> h1 -> h2 (per point), head 2*h2 -> hh -> hh -> 8 (per pair)."""
    h1: int
    h2: int
    hh: int

    def layer_shapes(self):
        return [(self.h1, 6), (self.h2, self.h1), (self.hh, 2 * self.h2), (self.hh, self.hh), (8, self.hh)]

    def n_floats(self) -> int:
        return sum(o * i + o for o, i in self.layer_shapes())


SMALL_WIDTHS = Widths(64, 128, 256)
SCALE_WIDTHS = Widths(128, 256, 512)


def gaussian_weights(widths: Widths, seed: int = 0, bias_std: float = 0.0):
    """He-initialised weights, W ~ N(0, 2 / fan_in), float32.

    Drawn from ``default_rng(seed)`` in the order W1, b1, W2, b2, H1, c1, H2,
    c2, H3, c3 (W row-major [out][in]).  Biases are zero unless bias_std > 0.
    """
    rng = np.random.default_rng(seed)
    out = []
    for o, i in widths.layer_shapes():
        out.append((rng.standard_normal((o, i)) * math.sqrt(2.0 / i)).astype(np.float32))
        b = rng.standard_normal(o) * bias_std if bias_std > 0 else np.zeros(o)
        out.append(b.astype(np.float32))
    return out


# Weight layout of the voxel-embedding variant (shape encoder: point MLP 3-256-256-256, 3D U-Net of 128
# channels with 3x3x3 kernels, linear 384 -> 16; predictor: 28-128-128-128 per object, 128-128-128-128,
# 128 -> 1), each entry (W shape, bias length) with W [out][in...].
VOXEL_LAYERS = (
    [((256, 3), 256), ((256, 256), 256), ((256, 256), 256)]
    + [((128, 256, 3, 3, 3), 128)] + [((128, 128, 3, 3, 3), 128)] * 3
    + [((128, 128, 3, 3, 3), 128)] + [((128, 256, 3, 3, 3), 128)] * 3
    + [((16, 384), 16)]
    + [((128, 28), 128), ((128, 128), 128), ((128, 128), 128)]
    + [((128, 128), 128)] * 3 + [((1, 128), 1)]
)


def voxel_weights(seed: int = 0, bias_std: float = 0.0):
    """He-initialised weights of the voxel-embedding variant, W ~ N(0, 2 / fan_in) (fan_in = the product
    of W's input dimensions), float32, drawn from ``default_rng(seed)`` layer by layer (W, then bias)."""
    rng = np.random.default_rng(seed)
    out = []
    for wshape, nb in VOXEL_LAYERS:
        fan_in = int(np.prod(wshape[1:]))
        out.append((rng.standard_normal(wshape) * math.sqrt(2.0 / fan_in)).astype(np.float32))
        b = rng.standard_normal(nb) * bias_std if bias_std > 0 else np.zeros(nb)
        out.append(b.astype(np.float32))
    return out


def flatten_weights(layers) -> np.ndarray:
    return np.concatenate([np.asarray(a, np.float32).ravel() for a in layers])


# ----------------------------------------------------------------------------
# uneven environments (a batched simulation) and its host broad phase
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class EnvSteps:
    """Objects of many independent environments over several simulation steps.

    Every environment shares one world region (as vectorised simulations do);
    objects only pair with objects of their own environment.
      shape  int32 [n]            shape id per object
      env    int32 [n]            environment of each object
      pos    float32 [S, n, 3]    positions per step
      quat   float32 [S, n, 4]    orientations per step (w, x, y, z)
      pairs  list of int32 [P_s, 2]: broad-phase pairs of step s (i < j)
    """
    lib: ShapeLibrary
    shape: np.ndarray
    env: np.ndarray
    pos: np.ndarray
    quat: np.ndarray
    pairs: list
    side: float

    @property
    def n_steps(self) -> int:
        return len(self.pairs)

    @property
    def env_offsets(self) -> np.ndarray:
        """int32 [E + 1]: objects of environment e are env_offsets[e] .. env_offsets[e+1] - 1."""
        n_env = int(self.env.max()) + 1 if len(self.env) else 0
        return np.concatenate([[0], np.cumsum(np.bincount(self.env, minlength=n_env))]).astype(np.int32)

    def scene(self, step: int) -> Scene:
        return Scene(self.lib, self.pos[step], self.quat[step], self.shape, self.pairs[step])


def _local_boxes(lib: ShapeLibrary):
    """Centre and half extent of each shape's point cloud (float64 [S, 3])."""
    c = np.empty((lib.n_shapes, 3))
    e = np.empty((lib.n_shapes, 3))
    for s in range(lib.n_shapes):
        p = lib.shape_points(s)[:, :3].astype(np.float64)
        lo, hi = p.min(axis=0), p.max(axis=0)
        c[s], e[s] = 0.5 * (lo + hi), 0.5 * (hi - lo)
    return c, e


def broad_phase(lib_boxes, shape, env_slices, pos, quat) -> np.ndarray:
    """All pairs (i < j) of one environment whose world bounding boxes overlap.

    The world box of an object is the axis-aligned hull of its rotated local
    box, computed with scipy's rotation matrices.  Returns int32 [P, 2].
    """
    c_loc, e_loc = lib_boxes
    R = _scipy_rot(quat).as_matrix()
    cw = np.einsum("nij,nj->ni", R, c_loc[shape]) + pos
    ew = np.einsum("nij,nj->ni", np.abs(R), e_loc[shape])
    lo, hi = cw - ew, cw + ew
    out = []
    for n, starts in env_slices:
        iu, ju = np.triu_indices(n, 1)
        if len(iu) == 0:
            continue
        I = starts[:, None] + iu[None, :]
        J = starts[:, None] + ju[None, :]
        ok = np.all((lo[I] <= hi[J]) & (lo[J] <= hi[I]), axis=-1)
        out.append(np.stack([I[ok], J[ok]], axis=1))
    return np.concatenate(out).astype(np.int32) if out else np.zeros((0, 2), np.int32)


def env_workload(master: int = 3, n_envs: int = 4096, max_objects: int = 40, steps: int = 200,
                 target_pairs: float = 2e5, lib: ShapeLibrary = None, jitter_m: float = 0.002,
                 jitter_rad: float = 0.02) -> EnvSteps:
    """Uneven environments: n_e ~ U{1..max_objects} objects per environment.

    Shapes are drawn from the 32-shape library of the at-scale workload,
    orientations are uniform, positions uniform in a cube whose side is set
    (by bisection on the first step) so that the broad phase yields about
    target_pairs pairs; each later step jitters every pose slightly.
    """
    g = streams(master)
    if lib is None:
        lib = scale_library()
    rng = g[STREAM_ENVS]
    sizes = rng.integers(1, max_objects + 1, n_envs)
    n = int(sizes.sum())
    env = np.repeat(np.arange(n_envs, dtype=np.int32), sizes)
    starts_all = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    env_slices = [(int(k), starts_all[sizes == k]) for k in np.unique(sizes)]
    shape = rng.integers(0, lib.n_shapes, n).astype(np.int32)
    boxes = _local_boxes(lib)
    q0 = uniform_quaternions(rng, n)
    u0 = rng.random((n, 3)) - 0.5

    def count(side):
        return len(broad_phase(boxes, shape, env_slices, u0 * side, q0))

    lo_s, hi_s = 0.05, 5.0
    for _ in range(30):
        mid = np.sqrt(lo_s * hi_s)
        if count(mid) > target_pairs:
            lo_s = mid
        else:
            hi_s = mid
    side = float(np.sqrt(lo_s * hi_s))
    pos = np.empty((steps, n, 3), np.float32)
    quat = np.empty((steps, n, 4), np.float32)
    t = u0 * side
    q = q0.copy()
    pairs = []
    for s in range(steps):
        if s:
            t = t + rng.normal(0.0, jitter_m, t.shape)
            axis = rng.normal(size=(n, 3))
            axis /= np.linalg.norm(axis, axis=1, keepdims=True)
            ang = rng.normal(0.0, jitter_rad, n)
            dq = np.concatenate([np.cos(ang / 2)[:, None], axis * np.sin(ang / 2)[:, None]], axis=1)
            r = _scipy_rot(dq) * _scipy_rot(q)
            xyzw = r.as_quat()
            q = np.concatenate([xyzw[:, 3:], xyzw[:, :3]], axis=1)
        pos[s] = t
        quat[s] = q
        pairs.append(broad_phase(boxes, shape, env_slices, pos[s].astype(np.float64), quat[s]))
    return EnvSteps(lib, shape, env, pos, quat, pairs, side)


# ----------------------------------------------------------------------------
# serving: a stream of simulation-step requests over resident environments
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class RequestStream:
    """Requests over a resident object table.

    shape, pos0, quat0   the initial table (every object of every environment)
    requests             list of (upd_ids int32 [u], pos float32 [u, 3],
                         quat float32 [u, 4], pairs int32 [p, 2]); a request
                         updates every object of the environments it covers,
                         so its result depends only on its own data
    """
    lib: ShapeLibrary
    shape: np.ndarray
    pos0: np.ndarray
    quat0: np.ndarray
    requests: list

    @property
    def pairs_per_request(self) -> np.ndarray:
        return np.array([len(r[3]) for r in self.requests])


def serve_library(master: int = 4, n_shapes: int = 128, n_points: int = 4096) -> ShapeLibrary:
    """128 shapes of 4096 points, drawn like the at-scale library (3-6 ellipsoids / boxes)."""
    return shape_library(streams(master)[STREAM_SHAPES], n_shapes, n_points, (3, 6), 0.5)


def request_stream(master: int = 4, n_requests: int = 10000, lib: ShapeLibrary = None, n_envs: int = 4096,
                   versions: int = 4, min_pairs: int = 8, max_pairs: int = 2000) -> RequestStream:
    """Simulation-step requests: pairs per request ~ log-uniform[min_pairs, max_pairs].

    The environments (uneven, 1-40 objects) are stepped `versions` times;
    each request takes distinct random environments of one random version
    until it has enough broad-phase pairs, updates all their objects to that
    version's poses and keeps the first n of their pairs.
    """
    g = streams(master)
    if lib is None:
        lib = serve_library(master)
    env = env_workload(master, n_envs=n_envs, steps=versions, lib=lib, target_pairs=2e5 * n_envs / 4096)
    rng = g[STREAM_REQUESTS]
    members = np.split(np.arange(len(env.shape)), np.flatnonzero(np.diff(env.env)) + 1)
    by_env = []
    for v in range(versions):
        pr = env.pairs[v]
        owner = env.env[pr[:, 0]]
        order = np.argsort(owner, kind="stable")
        cuts = np.searchsorted(owner[order], np.arange(n_envs + 1))
        by_env.append([pr[order[cuts[e]:cuts[e + 1]]] for e in range(n_envs)])
    targets = np.exp(rng.uniform(np.log(min_pairs), np.log(max_pairs), n_requests)).astype(int)
    reqs = []
    for t in targets:
        v = int(rng.integers(versions))
        envs, have = [], 0
        for e in rng.permutation(n_envs):
            if len(by_env[v][e]) == 0:
                continue
            envs.append(e)
            have += len(by_env[v][e])
            if have >= t:
                break
        ids = np.concatenate([members[e] for e in envs]).astype(np.int32)
        pairs = np.concatenate([by_env[v][e] for e in envs])[:t].astype(np.int32)
        reqs.append((ids, env.pos[v][ids], env.quat[v][ids], pairs))
    return RequestStream(lib, env.shape, env.pos[0], env.quat[0], reqs)
