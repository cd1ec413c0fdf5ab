"""Float accumulation variant (Sec. 4.1): the update rule swept along a ray in float32, with
optional reinitialization knots.  Test infrastructure: a plain, slow reference.

The paper quantizes because a front-to-back float sweep of the update rule (Eq.
accumulation-rule) propagates rounding errors of the higher-order coefficients, so that the
field does not return to zero behind the particles ("sprinkling", Fig. 2a).  Reinitialization
knots at fixed positions carry every covering particle's own localized coefficients and replace
the swept state there (Fig. 2b).  This module computes that sweep; its definition (this
implementation's reading, the paper gives no formulas for it) is:

Per hit (same hit test, closest point t_chi, distance parameter and nearest table entry as the
exact path), with tc, zf, vf the float32 roundings of t_chi, zeta and the amplitude:
  knots at tc - zf*theta_k (kidx P - k), tc + zf*theta_k (kidx P + k), and tc (kidx P, even K),
  each position plus +0.0 (no negative zero);
  with inv = 1/zf, base = vf*inv*inv*inv and sc_d = sc_{d-1}*inv (sc_0 = base), the jump of order
  d >= 1 at +theta_k is float32(s-hat_kd)*sc_d, at -theta_k that times (-1)^(d+1), at the middle
  knot float32(s-mid_d)*sc_d; order 0 is zero.
Knots are ordered by (position, particle input index, kidx).  One sweep: the state (D+1
coefficients, localized at the previous event) is shifted to each knot by the in-place Taylor
shift (for i = 0..D-1, for j = D-1 down to i: a_j = a_j + a_{j+1}*delta) and the jump is added
(the first knot only adds).  Reinitialization knots sit at T_s = t0 + s*step, s = 1..S, with
t0, t1 the float32 ray ends and step = (t1 - t0)/(S + 1); T_s takes effect after every knot at
positions <= T_s: the state becomes the sum, over the covering particles (first knot <= T_s <
last knot) in increasing input index, of each particle's own localized coefficients at T_s (its
own sweep over its knots <= T_s, in kidx order, then shifted to T_s).  Pieces: one per gap between
consecutive event positions (start, end, state), and a last one from the final event to t1.

Every arithmetic step goes through the number type `num` (float32 by default; the exact
Fraction type serves the pins): each operation rounds to float32 in the default mode.

Pinned by tests/test_oracle_floatpath.py: with exact arithmetic the sweep equals the direct sum
of every knot's jump polynomial (and each reinitialization knot equals that sum), a particle's
encoded function matches the table's piecewise polynomial scaled to the particle, and the
float32 sweep stays within its rounding bound of the exact one near the particles.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from . import geometry, lut as lut_mod

F32 = np.float32


class Exact:
    """Exact rational arithmetic on the float32 inputs (for the pins)."""

    @staticmethod
    def of(x):
        return Fraction(float(np.float32(x)))


class Float32:
    @staticmethod
    def of(x):
        return F32(x)


def particle_knots(tchi, zeta, value, theta_row, shat_row, smid_row, K, D, num=Float32):
    """[(t, kidx, [c_0..c_D])] of one hit, in kidx order."""
    P = (K + 1) // 2
    tc = num.of(F32(np.float64(tchi)))
    zf = num.of(F32(zeta))
    vf = num.of(F32(value))
    inv = num.of(1.0) / zf
    base = vf * inv * inv * inv
    sc = [base]
    for _ in range(D):
        sc.append(sc[-1] * inv)
    zero = num.of(0.0)
    out = []
    for kidx in range(2 * P + 1):
        k = kidx - P
        if k == 0 and K % 2 == 1:
            continue
        m = abs(k) - 1
        if m >= 0:
            off = zf * num.of(F32(np.float64(theta_row[m])))
            t = tc - off if k < 0 else tc + off
        else:
            t = tc
        t = t + zero
        c = [zero] * (D + 1)
        for d in range(1, D + 1):
            s = shat_row[m][d] if m >= 0 else smid_row[d]
            x = num.of(F32(np.float64(s))) * sc[d]
            if k < 0 and d % 2 == 0:
                x = -x
            c[d] = x
        out.append((t, kidx, c))
    return out


def shift(a, delta):
    """In-place Taylor shift by delta, top coefficient down (Eq. accumulation-rule without the
    jump), in the arithmetic of the entries."""
    a = list(a)
    D = len(a) - 1
    for i in range(D):
        for j in range(D - 1, i - 1, -1):
            a[j] = a[j] + a[j + 1] * delta
    return a


def local_at(own, T, num):
    """A particle's localized coefficients at T from its own knots (kidx order)."""
    D = len(own[0][2]) - 1
    st = [num.of(0.0)] * (D + 1)
    prev = own[0][0]
    for i, (t, _, c) in enumerate(own):
        if t > T:
            break
        if i > 0:
            st = shift(st, t - prev)
        st = [x + y for x, y in zip(st, c)]
        prev = t
    return shift(st, T - prev)


def reinit_positions(t_min, t_max, n_reinit, num=Float32):
    t0 = num.of(F32(t_min))
    t1 = num.of(F32(t_max))
    step = (t1 - t0) / num.of(F32(n_reinit + 1))
    return [t0 + num.of(F32(s + 1)) * step for s in range(n_reinit)]


def ray_pieces(o, v, t_min, t_max, xyz, zeta, value, table, K, D, kind, n_reinit=0, num=Float32, hits=None):
    """Pieces [(t_start, t_end, [c_0..c_D])] of the float sweep along one ray.

    table: dict with 'theta' [n, P], 'shat' [n, P, D+1] and 'smid' [n, D+1] (float64)."""
    q = 2.0
    if hits is None:
        hits = geometry.ray_hits(o, v, t_min, t_max, xyz, zeta, q)
    chi = geometry.widen(xyz)
    z = geometry.widen(zeta)
    val = geometry.widen(value)
    o = np.asarray(o, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    n_lut = len(table["theta"])
    per = {}
    for pid in sorted(int(p) for p in hits):
        lam2, tchi = geometry.pair_terms(o, v, chi[pid], z[pid])
        li = lut_mod.lut_index(kind, math.sqrt(float(lam2)), n_lut)
        per[pid] = particle_knots(float(tchi), z[pid], val[pid], table["theta"][li], table["shat"][li],
                                  table["smid"][li], K, D, num)
    knots = sorted(((t, pid, kidx, c) for pid, kn in per.items() for (t, kidx, c) in kn),
                   key=lambda e: (e[0], e[1], e[2]))
    Ts = reinit_positions(t_min, t_max, n_reinit, num)
    attached = []
    for T in Ts:
        acc = [num.of(0.0)] * (D + 1)
        for pid in sorted(per):
            own = per[pid]
            if own[0][0] <= T < own[-1][0]:
                loc = local_at(own, T, num)
                acc = [x + y for x, y in zip(acc, loc)]
        attached.append(acc)
    pieces = []
    st = [num.of(0.0)] * (D + 1)
    have = False
    prev = num.of(0.0)
    s = 0

    def reinit_before(t, inclusive):
        nonlocal st, have, prev, s
        while s < len(Ts):
            T = Ts[s]
            if not inclusive and not (T < t):
                break
            if have and T > prev:
                pieces.append((prev, T, list(st)))
            st = list(attached[s])
            prev = T
            have = True
            s += 1

    for (t, _, _, c) in knots:
        reinit_before(t, False)
        if have and t > prev:
            pieces.append((prev, t, list(st)))
        if have:
            st = shift(st, t - prev)
        st = [x + y for x, y in zip(st, c)]
        prev = t
        have = True
    reinit_before(None, True)
    t1 = num.of(F32(t_max))
    if have and prev < t1:
        pieces.append((prev, t1, list(st)))
    return pieces
