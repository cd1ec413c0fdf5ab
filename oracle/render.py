"""Classification and front-to-back compositing of a ray's piecewise polynomial field.

Sec. 2, third pass: per ray, the accumulated field is classified and
composited; the introduction refers to emission-absorption volume rendering
(classification maps field values to light emission and absorption).  The
paper fixes neither the transfer function nor the integration scheme; this
is this implementation's reading:

* Transfer function: n RGBA control points equally spaced over [v_min, v_max];
  x = clamp((v - v_min) / (v_max - v_min) * (n - 1), 0, n - 1) and linear
  interpolation between control points floor(x) and min(floor(x) + 1, n - 1);
  r, g, b are emission densities and a is the extinction coefficient.
* Sampling: each piece [t_a, t_b] is clipped to [t_min, t_max] -> [a', b'];
  S = max(1, ceil((b' - a') / step)) equal sub-segments of length
  delta = (b' - a') / S, sampled at their midpoints (u in the piece's [0, 1]
  coordinate), v = P(u).
* Each sub-segment with constant emission e and extinction sigma contributes
  T * e * (1 - exp(-sigma delta)) / sigma (T * e * delta when sigma = 0) and
  multiplies the transmittance T by exp(-sigma delta), in front-to-back order.
* Pixel = (C_r, C_g, C_b, 1 - T).
"""
from __future__ import annotations

import math

import numpy as np


def tf_lookup(tf, v_min, v_max, v):
    tf = np.asarray(tf, dtype=np.float64)
    n = len(tf)
    x = (v - v_min) / (v_max - v_min) * (n - 1)
    x = min(max(x, 0.0), float(n - 1))
    i0 = int(math.floor(x))
    i1 = min(i0 + 1, n - 1)
    f = x - i0
    return (1.0 - f) * tf[i0] + f * tf[i1]


def composite(nodes_out, t_min, t_max, tf, v_min, v_max, step):
    """RGBA of one ray from its pieces [(t_a, t_b, power coefficients in u)], front to back."""
    C = np.zeros(3)
    T = 1.0
    for (ta, tb, c) in nodes_out:
        a = max(ta, t_min)
        b = min(tb, t_max)
        if not b > a:
            continue
        S = max(1, int(math.ceil((b - a) / step)))
        delta = (b - a) / S
        for j in range(S):
            t = a + (j + 0.5) * delta
            u = (t - ta) / (tb - ta)
            v = float(np.polyval(np.asarray(c)[::-1], u))
            rgba = tf_lookup(tf, v_min, v_max, v)
            e = rgba[:3]
            sg = rgba[3]
            x = sg * delta
            frac = delta if x == 0.0 else -math.expm1(-x) / sg
            C = C + T * e * frac
            T = T * math.exp(-x)
    return np.array([C[0], C[1], C[2], 1.0 - T])
