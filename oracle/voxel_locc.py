"""CPU float64 oracle of the paper's own LOCC variant (voxel shape embedding).  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module; the product path never calls it and shares no code with
it.

The paper's LOCC (Sec. III, appendix "Architecture Details") has two parts.

Shape encoder, once per shape:
  V1  a per-point MLP on the stored xyz of the shape (object frame):
      3 -> 256 -> 256 -> 256, ReLU after each layer;
  V2  a grid of M x M x M cells (M = 6) on the shape's axis-aligned box
      [lo, hi]; point p goes to cell i_k = min(M - 1, floor(((p_k - lo_k) M)
      / (hi_k - lo_k))) per axis (0 on an axis of zero extent), flat index
      (i_0 M + i_1) M + i_2; each cell keeps the channel-wise max of its
      points' features, an empty cell keeps 0;
  V3  a 3D U-Net over the grid (channel-major tensors x[c][i0][i1][i2]):
        c1 = ReLU(conv(g, 256 -> 128, no padding))          6^3 -> 4^3
        c2 = ReLU(conv(c1, 128 -> 128, padding 1))          4^3
        c3 = ReLU(conv(c2)),  c4 = ReLU(conv(c3))            4^3
        glob = [max over cells of c4, mean over cells of c4]   (256)
        d1 = ReLU(convT(c4, 128 -> 128, padding 1))
        d2 = ReLU(convT([d1, c3], 256 -> 128, padding 1))
        d3 = ReLU(convT([d2, c2], 256 -> 128, padding 1))
        d4 = ReLU(convT([d3, c1], 256 -> 128, no padding))   4^3 -> 6^3
        E[cell] = L [d4[cell], glob] + l                    (384 -> F = 16, linear)
      with 3x3x3 kernels, where
        conv:  y[o][x] = b[o] + sum_c sum_u W[o][c][u] in[c][x + u - pad]
        convT: y[o][x] = b[o] + sum_c sum_u W[o][c][u] in[c][x - u + pad]
      (positions outside the input read 0; u over {0, 1, 2}^3, W[o][c][u0][u1][u2]).

Collision predictor, per pair (canonical order a = min(i, j), as in the
crop path; relative pose T_ab = (R_ab, t_ab) of O3-O4, float64):
  V4  cell centres c = lo + (i + 1/2) s, cell size s = (hi - lo) / M, margin
      eps = sqrt((s_0^2 + s_1^2) + s_2^2) / 2 (the centre-to-vertex distance
      of the cell under test);
  V5  a's cell is selected when its centre, taken to b's frame
      (x_i = (R[0][i] d_0 + R[1][i] d_1) + R[2][i] d_2, d = c - t_ab), lies in
      b's box widened by a's eps on every axis (closed); b's cell when its
      centre taken to a's frame (x_i = ((R[i][0] c_0 + R[i][1] c_1) +
      R[i][2] c_2) + t_i) lies in a's box widened by b's eps;
  V6  per object the mean of the selected cells' embeddings (0 if none);
  V7  per object the input [mean (16), t (3), R row-major (9)] with (R, t)
      the object's pose in the other object's frame: (R_ab^T, -R_ab^T t_ab)
      for a, (R_ab, t_ab) for b; rounded to float32;
  V8  a shared MLP 28 -> 128 -> 128 -> 128 (ReLU) per object, the
      element-wise max over the two objects, an MLP 128 -> 128 -> 128 -> 128
      (ReLU), a linear layer 128 -> 1 giving the logit, and the sigmoid.
  Invalid pairs (index out of range, i == j, shape id out of range) give
  NaN logit and probability and counts -1.

Weights (float32, flat, W row-major [out][in...]) in the order
  P1 [256][3], p1, P2 [256][256], p2, P3 [256][256], p3,
  C1 [128][256][3][3][3], k1, C2..C4 [128][128][3][3][3], k2..k4,
  D1 [128][128][3][3][3], e1, D2..D4 [128][256][3][3][3], e2..e4,
  L [16][384], l,
  A1 [128][28], a1, A2 [128][128], a2, A3 [128][128], a3,
  B1 [128][128], b1, B2 [128][128], b2, B3 [128][128], b3, B4 [1][128], b4.
"""

from __future__ import annotations

import numpy as np

from . import locc_oracle as O

M = 6
H_POINT = 256
C_CONV = 128
F_EMB = 16
H_PRED = 128
POSE_DIM = 12
IN_PRED = F_EMB + POSE_DIM


def layer_shapes():
    """Shapes of the weight arrays in their flat order."""
    k3 = (3, 3, 3)
    s = [(H_POINT, 3), (H_POINT,), (H_POINT, H_POINT), (H_POINT,), (H_POINT, H_POINT), (H_POINT,)]
    s += [(C_CONV, H_POINT) + k3, (C_CONV,)] + [(C_CONV, C_CONV) + k3, (C_CONV,)] * 3
    s += [(C_CONV, C_CONV) + k3, (C_CONV,)] + [(C_CONV, 2 * C_CONV) + k3, (C_CONV,)] * 3
    s += [(F_EMB, C_CONV + 2 * C_CONV), (F_EMB,)]
    s += [(H_PRED, IN_PRED), (H_PRED,)] + [(H_PRED, H_PRED), (H_PRED,)] * 2
    s += [(H_PRED, H_PRED), (H_PRED,)] * 3 + [(1, H_PRED), (1,)]
    return s


def n_weights() -> int:
    return int(sum(np.prod(s) for s in layer_shapes()))


def unpack(flat):
    """Flat float vector -> list of float64 arrays in the order of layer_shapes()."""
    flat = np.asarray(flat)
    out, o = [], 0
    for s in layer_shapes():
        n = int(np.prod(s))
        out.append(flat[o:o + n].astype(np.float64).reshape(s))
        o += n
    if o != len(flat):
        raise ValueError(f"expected {o} weights, got {len(flat)}")
    return out


def relu(x):
    return np.maximum(x, 0.0)


# ---------------------------------------------------------------- encoder --

def point_mlp(xyz, w):
    """V1: [n, 3] -> [n, 256]."""
    P1, p1, P2, p2, P3, p3 = w[:6]
    h = relu(np.asarray(xyz, np.float64) @ P1.T + p1)
    h = relu(h @ P2.T + p2)
    return relu(h @ P3.T + p3)


def voxel_index(xyz, lo, hi):
    """V2: flat cell index per point (float64, in the order written above)."""
    xyz = np.asarray(xyz, np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    idx = np.zeros(len(xyz), np.int64)
    for k in range(3):
        ext = hi[k] - lo[k]
        if ext > 0:
            t = ((xyz[:, k] - lo[k]) * float(M)) / ext
            i = np.minimum(np.floor(t).astype(np.int64), M - 1)
        else:
            i = np.zeros(len(xyz), np.int64)
        idx = idx * M + i
    return idx


def voxel_max(feat, idx):
    """V2: [M^3, H] channel-wise max per cell; empty cells 0."""
    g = np.zeros((M ** 3, feat.shape[1]))
    for c in range(M ** 3):
        sel = feat[idx == c]
        if len(sel):
            g[c] = np.maximum(sel.max(axis=0), 0.0)
    return g


def conv3d(x, W, b, pad):
    """V3 conv: x [C, D, D, D] -> [O, D + 2 pad - 2, ...] (correlation, zero padding)."""
    C, D = x.shape[0], x.shape[1]
    Do = D + 2 * pad - 2
    xp = np.zeros((C, D + 2 * pad, D + 2 * pad, D + 2 * pad))
    xp[:, pad:pad + D, pad:pad + D, pad:pad + D] = x
    y = np.zeros((W.shape[0], Do, Do, Do)) + b[:, None, None, None]
    for u0 in range(3):
        for u1 in range(3):
            for u2 in range(3):
                tap = xp[:, u0:u0 + Do, u1:u1 + Do, u2:u2 + Do].reshape(C, -1)
                y += (W[:, :, u0, u1, u2] @ tap).reshape(y.shape)
    return y


def conv3d_transpose(x, W, b, pad):
    """V3 convT: x [C, D, D, D] -> [O, D + 2 - 2 pad, ...]; in[x - u + pad], 0 outside."""
    C, D = x.shape[0], x.shape[1]
    Do = D + 2 - 2 * pad
    q = 2 - pad   # zero border so that in[x - u + pad] = xp[x - u + 2]
    xp = np.zeros((C, D + 2 * q, D + 2 * q, D + 2 * q))
    xp[:, q:q + D, q:q + D, q:q + D] = x
    y = np.zeros((W.shape[0], Do, Do, Do)) + b[:, None, None, None]
    for u0 in range(3):
        for u1 in range(3):
            for u2 in range(3):
                tap = xp[:, 2 - u0:2 - u0 + Do, 2 - u1:2 - u1 + Do, 2 - u2:2 - u2 + Do].reshape(C, -1)
                y += (W[:, :, u0, u1, u2] @ tap).reshape(y.shape)
    return y


def shape_embedding(xyz, w, lo=None, hi=None):
    """V1-V3: E [M^3, F] of one shape (lo / hi default to the stored points' box, O1)."""
    if lo is None:
        lo, hi = O.aabb(xyz)
    feat = point_mlp(np.asarray(xyz)[:, :3], w)
    g = voxel_max(feat, voxel_index(np.asarray(xyz)[:, :3], lo, hi))
    x = g.T.reshape(H_POINT, M, M, M)
    C1, k1, C2, k2, C3, k3, C4, k4 = w[6:14]
    D1, e1, D2, e2, D3, e3, D4, e4 = w[14:22]
    L, l = w[22:24]
    c1 = relu(conv3d(x, C1, k1, 0))
    c2 = relu(conv3d(c1, C2, k2, 1))
    c3 = relu(conv3d(c2, C3, k3, 1))
    c4 = relu(conv3d(c3, C4, k4, 1))
    flat4 = c4.reshape(C_CONV, -1)
    glob = np.concatenate([flat4.max(axis=1), flat4.mean(axis=1)])
    d1 = relu(conv3d_transpose(c4, D1, e1, 1))
    d2 = relu(conv3d_transpose(np.concatenate([d1, c3]), D2, e2, 1))
    d3 = relu(conv3d_transpose(np.concatenate([d2, c2]), D3, e3, 1))
    d4 = relu(conv3d_transpose(np.concatenate([d3, c1]), D4, e4, 0))
    cells = np.concatenate([d4.reshape(C_CONV, -1).T, np.tile(glob, (M ** 3, 1))], axis=1)
    return cells @ L.T + l


def library_embeddings(lib_pts, lib_offsets, weights_flat):
    """E [S, M^3, F] for every shape of a library."""
    w = unpack(weights_flat)
    S = len(lib_offsets) - 1
    return np.stack([shape_embedding(lib_pts[lib_offsets[s]:lib_offsets[s + 1], :3], w) for s in range(S)])


# -------------------------------------------------------------- predictor --

def cell_centres(lo, hi):
    """V4: [M^3, 3] centres in flat-index order, and the margin eps."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    s = (hi - lo) / float(M)
    i = np.arange(M, dtype=np.float64)
    c = [lo[k] + (i + 0.5) * s[k] for k in range(3)]
    g0, g1, g2 = np.meshgrid(c[0], c[1], c[2], indexing="ij")
    centres = np.stack([g0.ravel(), g1.ravel(), g2.ravel()], axis=1)
    eps = np.sqrt((s[0] * s[0] + s[1] * s[1]) + s[2] * s[2]) * 0.5
    return centres, eps


def to_b_frame(Rab, tab, c):
    """V5 (a side): x_i = (R[0][i] d0 + R[1][i] d1) + R[2][i] d2, d = c - t_ab."""
    d = np.asarray(c, np.float64) - tab
    x = np.empty_like(d)
    for i in range(3):
        x[:, i] = (Rab[0, i] * d[:, 0] + Rab[1, i] * d[:, 1]) + Rab[2, i] * d[:, 2]
    return x


def select_cells(Rab, tab, box_a, box_b):
    """V5: boolean masks [M^3] of a's and b's selected cells.  box = (lo, hi) float64."""
    ca, eps_a = cell_centres(*box_a)
    cb, eps_b = cell_centres(*box_b)
    xa = to_b_frame(Rab, tab, ca)
    sel_a = np.all((xa >= box_b[0] - eps_a) & (xa <= box_b[1] + eps_a), axis=1)
    xb = O.transform_points(Rab, tab, cb)
    sel_b = np.all((xb >= box_a[0] - eps_b) & (xb <= box_a[1] + eps_b), axis=1)
    return sel_a, sel_b


def pose_inputs(Rab, tab):
    """V7: the 12 pose values of a (in b's frame) and of b (in a's frame)."""
    Rba = Rab.T
    tba = np.empty(3)
    for i in range(3):
        tba[i] = -((Rab[0, i] * tab[0] + Rab[1, i] * tab[1]) + Rab[2, i] * tab[2])
    return np.concatenate([tba, Rba.ravel()]), np.concatenate([tab, Rab.ravel()])


def predictor(z_a, z_b, w):
    """V8: logit from the two per-object inputs (28 values each)."""
    A1, a1, A2, a2, A3, a3 = w[24:30]
    B1, b1, B2, b2, B3, b3, B4, b4 = w[30:38]

    def mlp1(z):
        h = relu(z @ A1.T + a1)
        h = relu(h @ A2.T + a2)
        return relu(h @ A3.T + a3)

    g = np.maximum(mlp1(z_a), mlp1(z_b))
    g = relu(g @ B1.T + b1)
    g = relu(g @ B2.T + b2)
    g = relu(g @ B3.T + b3)
    return float((g @ B4.T + b4)[0])


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def detect(lib_pts, lib_offsets, pos, quat, shape, pairs, weights_flat, emb=None, rows=None):
    """V4-V8 for the pairs (or the listed rows of them).  Returns dict with
    logit [P], prob [P], counts [P, 2] (caller order), pooled [P, 2, 16]
    (caller order) and the embeddings used."""
    w = unpack(weights_flat)
    if emb is None:
        emb = library_embeddings(lib_pts, lib_offsets, weights_flat)
    S = len(lib_offsets) - 1
    boxes = [O.aabb(lib_pts[lib_offsets[s]:lib_offsets[s + 1], :3]) for s in range(S)]
    rows = range(len(pairs)) if rows is None else rows
    R = len(rows)
    logit = np.full(R, np.nan)
    counts = np.full((R, 2), -1, np.int32)
    pooled = np.full((R, 2, F_EMB), np.nan)
    for r, p in enumerate(rows):
        i, j = int(pairs[p][0]), int(pairs[p][1])
        if not O.pair_valid(i, j, len(pos), shape, S):
            continue
        a, b, sgn = O.canonical(i, j)
        Ra, Rb = O.rotation(quat[a]), O.rotation(quat[b])
        Rab, tab = O.relative_pose(Ra, pos[a], Rb, pos[b])
        sa, sb = int(shape[a]), int(shape[b])
        sel_a, sel_b = select_cells(Rab, tab, boxes[sa], boxes[sb])
        m_a = emb[sa][sel_a].mean(axis=0) if sel_a.any() else np.zeros(F_EMB)
        m_b = emb[sb][sel_b].mean(axis=0) if sel_b.any() else np.zeros(F_EMB)
        pose_a, pose_b = pose_inputs(Rab, tab)
        z_a = np.concatenate([m_a, pose_a]).astype(np.float32).astype(np.float64)
        z_b = np.concatenate([m_b, pose_b]).astype(np.float32).astype(np.float64)
        logit[r] = predictor(z_a, z_b, w)
        first, second = (0, 1) if sgn > 0 else (1, 0)
        counts[r, first], counts[r, second] = int(sel_a.sum()), int(sel_b.sum())
        pooled[r, first], pooled[r, second] = m_a, m_b
    return dict(logit=logit, prob=sigmoid(logit), counts=counts, pooled=pooled, emb=emb)
