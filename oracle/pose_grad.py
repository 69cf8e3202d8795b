"""CPU float64 oracle of the pose gradients of the collision logit.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module; the product path never calls it and shares no code with
it.

The paper obtains contact force and torque directions from the gradient of
the collision network's output with respect to the objects' poses (Sec. II,
the paragraph on collision resolution with an object collision network).  For the crop-point path of
``oracle.locc_oracle`` this is the derivative of the logit y0 (O10) with
respect to each object's position p and quaternion q (the four components as
given, not renormalised: R(q) is the polynomial of O3), by reverse-mode
differentiation in this order:

  G1  forward as O9-O10, keeping per object and channel c of the encoder's
      second layer the row r*(c) where the raw sum s[r][c] = W2[c] . h1[r]
      is largest (the first such row on ties) and m[c] = s[r*][c], so that
      f[c] = ReLU(m[c] + b2[c]) (an empty crop gives f = 0 and no gradient);
  G2  head backward: dy0 = 1; du2 = H3[0] (u2 > 0); dg1 = H2^T du2;
      du1 = dg1 (u1 > 0); df = H1^T du1; dm[c] = df[c] (m[c] + b2[c] > 0);
  G3  encoder backward, second object only (the first object's rows are its
      own stored points, which do not depend on the poses): for each channel
      c, row r = r*(c): dh1[r] += W2[c] dm[c]; dr[r] = W1^T (dh1[r] (W1 r +
      b1 > 0)) -- six values per row: the point (dx) and the normal (dn);
  G4  the rows are q = R_ab p + t_ab and R_ab n with (p, n) the stored point
      and normal of b:  dR_ab = sum_r dx_r p_r^T + dn_r n_r^T,
      dt_ab = sum_r dx_r;
  G5  R_ab = R_a^T R_b, t_ab = R_a^T (p_b - p_a):  dR_a = R_b dR_ab^T +
      (p_b - p_a) dt_ab^T, dR_b = R_a dR_ab, dp_b = R_a dt_ab, dp_a = -dp_b;
  G6  dq_k = sum_ij dR[i][j] dR[i][j]/dq_k with the partial derivatives of
      the polynomial R(w, x, y, z);
  G7  the 14 values (dp, dq of the caller's first object, then of its
      second) in the caller's order; NaN for invalid pairs.

The crop selection is piecewise constant in the poses and contributes
nothing; away from selection boundaries and argmax ties the result is the
derivative of the logit.  At a tie every row attaining the maximum gives a
valid one-sided derivative, so the argmax rows of the second object may be
given (argmax_b) instead of taken as the first maximum.
"""

from __future__ import annotations

import numpy as np

from . import locc_oracle as O


def rotation_grad(q, G):
    """G6: d/dq of sum_ij G[i][j] R(q)[i][j] for R(q) of O3 (q = w, x, y, z as given)."""
    w, x, y, z = (float(v) for v in q)
    G = np.asarray(G, np.float64)
    dw = 2 * (-G[0, 1] * z + G[0, 2] * y + G[1, 0] * z - G[1, 2] * x - G[2, 0] * y + G[2, 1] * x)
    dx = 2 * (G[0, 1] * y + G[0, 2] * z + G[1, 0] * y - 2 * G[1, 1] * x - G[1, 2] * w + G[2, 0] * z
              + G[2, 1] * w - 2 * G[2, 2] * x)
    dy = 2 * (-2 * G[0, 0] * y + G[0, 1] * x + G[0, 2] * w + G[1, 0] * x + G[1, 2] * z - G[2, 0] * w
              + G[2, 1] * z - 2 * G[2, 2] * y)
    dz = 2 * (-2 * G[0, 0] * z - G[0, 1] * w + G[0, 2] * x + G[1, 0] * w - 2 * G[1, 1] * z + G[1, 2] * y
              + G[2, 0] * x + G[2, 1] * y)
    return np.array([dw, dx, dy, dz])


def encoder_argmax(rows, W1, b1, W2):
    """G1: raw maxima m [h2] and argmax rows r* [h2] (-1 for an empty set)."""
    rows = np.asarray(rows, np.float64).reshape(-1, 6)
    if len(rows) == 0:
        return np.full(W2.shape[0], -np.inf), np.full(W2.shape[0], -1, np.int64)
    s = O.relu(rows @ W1.T + b1) @ W2.T
    r = np.argmax(s, axis=0)                      # first maximum on ties
    return s[r, np.arange(s.shape[1])], r


def pair_gradient(g, pts_b, qa, pa, qb, pb, weights, argmax_b=None):
    """G1-G6 for one canonical pair: (logit, dp_a, dq_a, dp_b, dq_b, r*_b), r*_b the first maxima.
    argmax_b: the second object's argmax rows to use instead (each must attain its channel's maximum
    up to the caller's tolerance)."""
    W1, b1, W2, b2, H1, c1, H2, c2, H3, c3 = weights
    h2 = W2.shape[0]
    m_a, _ = encoder_argmax(g.rows_a, W1, b1, W2)
    m_b, first_b = encoder_argmax(g.rows_b, W1, b1, W2)
    r_b = first_b if argmax_b is None or len(g.rows_b) == 0 else np.asarray(argmax_b, np.int64)
    f = np.concatenate([O.relu(m_a + b2), O.relu(m_b + b2)])       # -inf + b2 -> 0 for an empty crop
    u1 = f @ H1.T + c1
    u2 = O.relu(u1) @ H2.T + c2
    logit = float(O.relu(u2) @ H3[0] + c3[0])
    du2 = H3[0] * (u2 > 0)
    du1 = (du2 @ H2) * (u1 > 0)
    df = du1 @ H1
    dm_b = df[h2:] * (m_b + b2 > 0)
    GR = np.zeros((3, 3))
    gt = np.zeros(3)
    sel = g.idx_b[g.idx_b >= 0]
    for c in range(h2):
        r = r_b[c]
        if r < 0 or dm_b[c] == 0.0:
            continue
        row = g.rows_b[r]
        dh1 = W2[c] * dm_b[c] * (row @ W1.T + b1 > 0)
        dr = dh1 @ W1
        p = np.asarray(pts_b[sel[r], :3], np.float64)
        n = np.asarray(pts_b[sel[r], 3:6], np.float64)
        GR += np.outer(dr[:3], p) + np.outer(dr[3:], n)
        gt += dr[:3]
    Ra, Rb = O.rotation(qa), O.rotation(qb)
    d = np.asarray(pb, np.float64) - np.asarray(pa, np.float64)
    dRa = Rb @ GR.T + np.outer(d, gt)
    dRb = Ra @ GR
    dp_b = Ra @ gt
    return logit, -dp_b, rotation_grad(qa, dRa), dp_b, rotation_grad(qb, dRb), first_b


def pose_gradients(lib_pts, lib_offsets, pos, quat, shape, pairs, weights_flat, widths, K, pad=O.PAD_M,
                   argmax_b=None):
    """G1-G7 for every pair: dict(logit [P], grad [P, 14], first_argmax_b [P, h2] (the first maxima of the
    canonical second object)).  argmax_b [P, h2], optional: that object's argmax rows to use per pair."""
    h1, h2, hh = widths
    weights = O.unpack_weights(weights_flat, h1, h2, hh)
    geoms, _, _ = O.crop(lib_pts, lib_offsets, pos, quat, shape, pairs, K, pad)
    P = len(pairs)
    logit = np.full(P, np.nan)
    grad = np.full((P, 14), np.nan)
    first_argmax_b = np.full((P, h2), -1, np.int64)
    for p, g in enumerate(geoms):
        if g is None:
            continue
        sb = int(shape[g.b])
        pts_b = lib_pts[lib_offsets[sb]:lib_offsets[sb + 1]]
        lg, dpa, dqa, dpb, dqb, rb = pair_gradient(g, pts_b, quat[g.a], pos[g.a], quat[g.b], pos[g.b], weights,
                                                   None if argmax_b is None else argmax_b[p])
        logit[p] = lg
        first_argmax_b[p] = rb
        first = np.concatenate([dpa, dqa])
        second = np.concatenate([dpb, dqb])
        grad[p] = np.concatenate([first, second]) if g.sgn > 0 else np.concatenate([second, first])
    return dict(logit=logit, grad=grad, first_argmax_b=first_argmax_b, geoms=geoms)
