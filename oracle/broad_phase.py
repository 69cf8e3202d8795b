"""CPU float64 oracle of the broad phase that feeds the LOCC path.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module; the product path never calls it and shares no code with
it.

The paper rules out object pairs that are far apart in the broad phase of
collision detection before any narrow-phase test (Sec. II, footnote on the
broad phase); its simulations run many environments at once, each object
pairing only with objects of its own environment.  What this oracle
computes, per simulation step:

  B1  world box of every object: the axis-aligned hull of its shape's box
      (O1 of the path oracle) after the object's rotation (O3) and
      translation, in centre / half-extent form,
        c_w[i] = ((R[i][0] c0 + R[i][1] c1) + R[i][2] c2) + p_i
        e_w[i] = (|R[i][0]| e0 + |R[i][1]| e1) + |R[i][2]| e2
      with c = (lo + hi) / 2, e = (hi - lo) / 2 of the shape box, every
      product and sum a separately rounded float64 operation, and
      lo_w = c_w - e_w, hi_w = c_w + e_w;
  B2  for every environment e (objects env_offsets[e] .. env_offsets[e+1]-1)
      every pair i < j whose world boxes overlap on all three axes (closed
      intervals: lo_i <= hi_j and lo_j <= hi_i);
  B3  the pairs listed by environment, then i, then j, ascending.

Readings for input the paper does not consider: an object whose shape id is
out of range has a NaN box, and NaN compares false, so it is in no pair (as
is an object whose pose holds a NaN); each environment bound is clamped to
[0, n], and an empty or reversed range holds no object.
"""

from __future__ import annotations

import numpy as np

from . import locc_oracle as O


def shape_boxes(lib_pts, lib_offsets):
    """O1 per shape, as centre and half extent (float64 [S, 3] each)."""
    S = len(lib_offsets) - 1
    c = np.empty((S, 3))
    e = np.empty((S, 3))
    for s in range(S):
        lo, hi = O.aabb(lib_pts[lib_offsets[s]:lib_offsets[s + 1]])
        c[s] = 0.5 * (lo + hi)
        e[s] = 0.5 * (hi - lo)
    return c, e


def world_boxes(lib_pts, lib_offsets, pos, quat, shape):
    """B1: lo, hi float64 [n, 3] of every object."""
    c_loc, e_loc = shape_boxes(lib_pts, lib_offsets)
    n = len(shape)
    lo = np.empty((n, 3))
    hi = np.empty((n, 3))
    for k in range(n):
        if not 0 <= shape[k] < len(c_loc):
            lo[k] = hi[k] = np.nan
            continue
        R = O.rotation(quat[k])
        c, e = c_loc[shape[k]], e_loc[shape[k]]
        p = np.asarray(pos[k], np.float64)
        for i in range(3):
            cw = ((R[i, 0] * c[0] + R[i, 1] * c[1]) + R[i, 2] * c[2]) + p[i]
            ew = (abs(R[i, 0]) * e[0] + abs(R[i, 1]) * e[1]) + abs(R[i, 2]) * e[2]
            lo[k, i] = cw - ew
            hi[k, i] = cw + ew
    return lo, hi


def broad_phase(lo, hi, env_offsets):
    """B2-B3: int32 [P, 2] pairs (i < j) of overlapping world boxes, per environment."""
    out = []
    n = len(lo)
    for e in range(len(env_offsets) - 1):
        a, b = (min(max(int(v), 0), n) for v in env_offsets[e:e + 2])
        for i in range(a, b):
            j = np.arange(i + 1, b)
            if len(j) == 0:
                continue
            ok = np.all((lo[i] <= hi[j]) & (lo[j] <= hi[i]), axis=1)
            out.extend((i, int(jj)) for jj in j[ok])
    return np.array(out, np.int32).reshape(-1, 2)
