"""CPU model of the library's BF16 and FP8 network arithmetic.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module; the product path never calls it and shares no code with
it.  It consumes the crop geometry of ``oracle.locc_oracle`` (the paper's
path, Sec. III and the appendix "Architecture Details") and re-runs the
network of O9-O10 with the reduced precision the FP8 variant uses.  The
paper trains and evaluates in full precision: the quantisation below is this
library's, stated here so that its kernel can be compared element by element
with a model written from the number formats, not from the kernel.

  Q1  bfloat16: float32 rounded to 8 significant bits, nearest even.
  Q2  e4m3 (OCP 8-bit floating point, E4M3 with no infinities): 4 exponent
      bits (bias 7), 3 mantissa bits, subnormal step 2^-9, largest finite
      magnitude 448; round to nearest even after clamping |x| to 448.
  Q3  per-layer scales: a weight matrix W is stored as e4m3(W / s_W) with
      s_W = amax|W| / 448; a layer input x enters as e4m3(min(x / s_x, 448))
      with the static s_x = amax_x / 448 (amax over a calibration batch, or
      1 when that maximum is 0).  Scales are float32; the two scales of a
      layer are multiplied once, after the sum.
  Q4  layer precisions: encoder layer 1 bf16 x bf16 in units of the scale
      s_x of its output (weights and bias stored as bf16(W1 * (1 / s_x)),
      bf16(b1 * (1 / s_x)), products in float32; rows rounded float64 ->
      float32 -> bf16), its output entering encoder layer 2 as
      e4m3(min(ReLU(h), 448)); encoder layer 2 e4m3 x e4m3, the max-pool on
      the unscaled sums, then scale s_x s_W2, bias and ReLU; head layers 1 and
      2 e4m3 x e4m3; head layer 2's output rounded to bf16; head layer 3 bf16
      x bf16.  A head layer that is not e4m3 runs as in Q5 (its input and
      weights bf16), so the variant with only encoder layer 2 in e4m3 has the
      BF16 head.
  Q5  the BF16 variant: every layer bf16 x bf16.  Encoder layer 1 on rows
      rounded float64 -> float32 -> bf16 with bf16(W1) and bf16(b1) (the bias
      enters the sum as a product with the constant input 1), output ReLU then
      bf16; encoder layer 2 with bf16(W2), the max-pool on the raw sums, then
      + b2 (float32) and ReLU, giving the pooled feature f in float32; the
      head on bf16(f): g1 = bf16(ReLU(bf16(H1) . + c1)), g2 likewise with H2
      and c2, y = bf16(H3) g2 + c3, biases c1..c3 float32.
  Every sum is float32 in the kernels; here sums are float64 and the result is
  rounded to float32 where a quantisation decision follows, so both sides
  take each decision in float32.
"""

from __future__ import annotations

import numpy as np

from . import locc_oracle as O

E4M3_MAX = 448.0


def bf16(x) -> np.ndarray:
    """Q1: float32 values rounded to the nearest bfloat16 (ties to even), as float32."""
    x = np.ascontiguousarray(x, np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def e4m3(x) -> np.ndarray:
    """Q2: nearest e4m3 value (ties to even) of |x| clamped to 448, as float32."""
    x = np.asarray(x, np.float64)
    a = np.minimum(np.abs(x), E4M3_MAX)
    _, e = np.frexp(np.maximum(a, 2.0 ** -6))   # a = f 2^e, f in [0.5, 1): binade 2^(e-1)
    step = np.where(a < 2.0 ** -6, 2.0 ** -9, np.ldexp(1.0, e - 4))
    q = np.minimum(np.round(a / step) * step, E4M3_MAX)   # np.round: ties to even
    return (np.sign(x) * q).astype(np.float32)


def f32(x) -> np.ndarray:
    return np.asarray(x, np.float32)


def weight_scale(W) -> np.float32:
    """Q3: s_W = amax|W| / 448 in float32."""
    return np.float32(np.abs(f32(W)).max()) / np.float32(E4M3_MAX)


def act_scale(amax) -> np.float32:
    """Q3: s_x = amax / 448 in float32 (1 when amax is 0)."""
    a = np.float32(amax)
    return a / np.float32(E4M3_MAX) if a > 0 else np.float32(1.0)


def quant_act(x, s) -> np.ndarray:
    """Q3: e4m3(min(x * (1 / s), 448)) with the reciprocal and the product in float32."""
    inv = np.float32(1.0) / np.float32(s)
    return e4m3(np.minimum(f32(x) * inv, np.float32(E4M3_MAX)))


def _valid(geoms):
    return [p for p, g in enumerate(geoms) if g is not None]


def calibrate(geoms, weights_flat, widths):
    """Activation maxima (encoder layer-1 output, pooled features, head layer-1
    output) of the float32 network on bf16 rows over the valid pairs."""
    h1w, h2w, hhw = widths
    W1, b1, W2, b2, H1, c1, *_ = [f32(w) for w in O.unpack_weights(weights_flat, h1w, h2w, hhw)]
    m_h = m_z = m_g = 0.0
    for p in _valid(geoms):
        g = geoms[p]
        z = []
        for rows in (g.rows_a, g.rows_b):
            r = bf16(f32(rows)).astype(np.float64)
            h = np.maximum(f32(r @ W1.T.astype(np.float64) + b1), 0)
            if len(h):
                m_h = max(m_h, float(h.max()))
            o = np.maximum(f32(h.astype(np.float64) @ W2.T.astype(np.float64) + b2), 0)
            z.append(np.max(o, axis=0, initial=0.0))
        z = np.concatenate(z)
        m_z = max(m_z, float(z.max()))
        g1 = np.maximum(f32(z.astype(np.float64) @ H1.T.astype(np.float64) + c1), 0)
        m_g = max(m_g, float(g1.max()))
    return np.array([m_h, m_z, m_g], np.float32)


FP8_ALL = ("enc2", "head1", "head2")


def fp8_forward(geoms, weights_flat, widths, amax, quantise=True, fp8_layers=FP8_ALL):
    """Q1-Q4: raw head outputs y [P, 8] (a's frame) and pooled features z
    [P, 2 h2] (float32 values before their quantisation); NaN for invalid
    pairs.  fp8_layers names the layers run e4m3 x e4m3 (encoder layer 2 is
    always one of them); the others run as in Q5.  quantise=False replaces
    every rounding by the identity (the scales stay), which must give the
    full-precision network back."""
    if "enc2" not in fp8_layers:
        raise ValueError("the FP8 variants all run encoder layer 2 in e4m3")
    h1w, h2w, hhw = widths
    W1, b1, W2, b2, H1, c1, H2, c2, H3, c3 = [f32(w) for w in O.unpack_weights(weights_flat, h1w, h2w, hhw)]
    qb = bf16 if quantise else f32
    q8 = e4m3 if quantise else f32
    s_w2, s_h1, s_h2 = weight_scale(W2), weight_scale(H1), weight_scale(H2)
    s_x, s_z, s_g = (act_scale(a) for a in amax)
    inv_x = np.float32(1.0) / s_x
    W1q, b1q = [qb(f32(w) * inv_x).astype(np.float64) for w in (W1, b1)]   # layer 1 in units of s_x
    H3q = qb(H3).astype(np.float64)
    W2q = q8(W2 / s_w2).astype(np.float64)
    f8h1, f8h2 = "head1" in fp8_layers, "head2" in fp8_layers
    H1q = (q8(H1 / s_h1) if f8h1 else qb(H1)).astype(np.float64)
    H2q = (q8(H2 / s_h2) if f8h2 else qb(H2)).astype(np.float64)
    s_enc, s_hd1, s_hd2 = np.float32(s_x * s_w2), np.float32(s_z * s_h1), np.float32(s_g * s_h2)
    qa = quant_act if quantise else (lambda x, s: f32(x) * (np.float32(1.0) / np.float32(s)))
    P = len(geoms)
    z = np.full((P, 2 * h2w), np.nan, np.float32)
    y = np.full((P, 8), np.nan)
    for p in _valid(geoms):
        g = geoms[p]
        feats = []
        for rows in (g.rows_a, g.rows_b):
            r = qb(f32(rows)).astype(np.float64)
            h = np.maximum(f32(r @ W1q.T + b1q), 0)                 # already divided by s_x
            acc = q8(np.minimum(h, np.float32(E4M3_MAX))).astype(np.float64) @ W2q.T
            raw = acc.max(axis=0) if len(acc) else np.full(h2w, -np.inf)
            feats.append(np.maximum(f32(raw * np.float64(s_enc) + b2), 0))   # one rounding, as a fused multiply-add
        z[p] = np.concatenate(feats)
        if f8h1:
            g1 = np.maximum(f32((qa(z[p], s_z).astype(np.float64) @ H1q.T) * np.float64(s_hd1) + c1), 0)
        else:
            g1 = np.maximum(f32(qb(z[p]).astype(np.float64) @ H1q.T) + c1, 0)
        if f8h2:
            g2 = np.maximum(f32((qa(g1, s_g).astype(np.float64) @ H2q.T) * np.float64(s_hd2) + c2), 0)
        else:
            g2 = np.maximum(f32(qb(g1).astype(np.float64) @ H2q.T) + c2, 0)
        y[p] = qb(g2).astype(np.float64) @ H3q.T + c3
    return y, z


def bf16_forward(geoms, weights_flat, widths, quantise=True):
    """Q1, Q5: raw head outputs y [P, 8] (a's frame) and pooled features z
    [P, 2 h2] (float32, before the bf16 rounding the head applies); NaN for
    invalid pairs.  quantise=False replaces every bf16 rounding by the
    identity, which must give the full-precision network back."""
    h1w, h2w, hhw = widths
    W1, b1, W2, b2, H1, c1, H2, c2, H3, c3 = [f32(w) for w in O.unpack_weights(weights_flat, h1w, h2w, hhw)]
    qb = bf16 if quantise else f32
    W1q, b1q, W2q, H1q, H2q, H3q = [qb(w).astype(np.float64) for w in (W1, b1, W2, H1, H2, H3)]
    P = len(geoms)
    z = np.full((P, 2 * h2w), np.nan, np.float32)
    y = np.full((P, 8), np.nan)
    for p in _valid(geoms):
        g = geoms[p]
        feats = []
        for rows in (g.rows_a, g.rows_b):
            r = qb(f32(rows)).astype(np.float64)
            h = qb(np.maximum(f32(r @ W1q.T + b1q), 0)).astype(np.float64)
            acc = f32(h @ W2q.T)
            raw = acc.max(axis=0) if len(acc) else np.full(h2w, -np.inf, np.float32)
            feats.append(np.maximum(raw + b2, np.float32(0)))
        z[p] = np.concatenate(feats)
        g1 = qb(np.maximum(f32(qb(z[p]).astype(np.float64) @ H1q.T) + c1, 0)).astype(np.float64)
        g2 = qb(np.maximum(f32(g1 @ H2q.T) + c2, 0)).astype(np.float64)
        y[p] = g2 @ H3q.T + c3
    return y, z


def _world(geoms, y):
    contacts = np.full((len(geoms), 8), np.nan)
    for p in _valid(geoms):
        g = geoms[p]
        contacts[p] = O.post(y[p], g.Ra, g.ta, g.sgn)
    return contacts


def bf16_detect(geoms, weights_flat, widths, quantise=True):
    """Contacts [P, 8] in the world frame (oracle O11 on the model's y), y and z of the BF16 variant."""
    y, z = bf16_forward(geoms, weights_flat, widths, quantise)
    return dict(contacts=_world(geoms, y), y=y, z=z)


def fp8_detect(geoms, weights_flat, widths, amax, quantise=True, fp8_layers=FP8_ALL):
    """Contacts [P, 8] in the world frame (oracle O11 on the model's y), y and z."""
    y, z = fp8_forward(geoms, weights_flat, widths, amax, quantise, fp8_layers)
    return dict(contacts=_world(geoms, y), y=y, z=z)
