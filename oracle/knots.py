"""Quantized knots of one particle on one ray (Sec. 4.3, derivation in App. A.3).

Given the particle's closest-point parameter t_chi, smoothing length zeta and
amplitude value = m*alpha/rho, the table row (theta_1..theta_P, s^_kd) of the
normalized distance closest to Lambda, and the quanta tau and sigma:

  t0 = round(t_chi / tau);  o_k = round(zeta * theta_k / tau);
  positions t0 + o_k and t0 - o_k for k = 1..P, plus t0 itself when K is even
  (Eq. quantized-middle-knot-position and Eq. quantized-knot-positions);
  a_kd = round(tau^d * value * s^_kd / (sigma * zeta^(d+3)))   for k >= 1,
         except k = 1 with odd d when K is odd
         (Eq. quantized-jumps-starting-from-lut);
  a_{-k,d} = (-1)^(d+1) a_kd  (Eq. contribution-spline-jumps-condition);
  even K: a_0d = -2 sum_{k=-P..-1} sum_{j=d..D} C(j,d) a_kj (t0 - t_k)^(j-d)
          for odd d, 0 for even d (Eq. quantized-middle-jumps-computation);
  odd K:  for odd d in decreasing order
          a_{-1,d} = -sum_{k=-P..-2} a_kd
                     - sum_{j=d+1..D} C(j,d) sum_{k=-P..-1} a_kj (t0 - t_k)^(j-d)
          and a_{1,d} = (-1)^(d+1) a_{-1,d}
          (Eq. quantized-jumps-uneven-pieces-count-computation);
  a_k0 = 0 for every knot.

Rounding: round half to even (the paper leaves the tie rule open).  The
floating-point expression for a_kd is evaluated in float64 as
    u = tau / zeta;  base = value / (sigma * (zeta * zeta * zeta));
    a_kd = rint(s^_kd * (base * u^d)),  u^d by repeated multiplication;
which equals the paper's expression up to rounding.  The closure is done in
Python integers, so it is exact.

Knot identity: kidx = k + P for the knots t0 + o_k (k = -P..P; kidx = P is the
middle knot of even K; odd K has no middle knot).

Pinned by tests/test_oracle_knots.py: exact zero tail of every particle's own
accumulation, shifted evenness of the piecewise polynomial it encodes, the
symmetry of the positions, and closeness of the encoded function to the
scaled, shifted table approximation.  The wrap-around accumulation of the
bit-length study (accumulate_wrapped) is pinned by the closed form of the
rule's result (each jump polynomial re-expanded about the last knot, summed)
and by direct evaluation of the encoded polynomial at sample points.
"""
from __future__ import annotations

from math import comb

import numpy as np


def rint(x) -> int:
    """Nearest integer, ties to even, of a float64 (as C's rint)."""
    return int(np.rint(np.float64(x)))


def pair_knots(tchi, zeta, value, theta_row, shat_row, tau, sigma, K, D):
    """List of knots (t, kidx, [a_0..a_D]) of one particle on one ray, in kidx order."""
    P = (K + 1) // 2
    tchi = np.float64(tchi)
    zeta = np.float64(zeta)
    value = np.float64(value)
    tau = np.float64(tau)
    sigma = np.float64(sigma)
    t0 = rint(tchi / tau)
    offs = [rint(zeta * np.float64(theta_row[k - 1]) / tau) for k in range(1, P + 1)]
    u = tau / zeta
    base = value / (sigma * (zeta * zeta * zeta))
    scale = [np.float64(1.0)] * (D + 1)
    p = np.float64(1.0)
    for d in range(1, D + 1):
        p = p * u
        scale[d] = base * p
    # coefficient table a[k][d] for k = -P..P (dict), all start at 0
    a = {k: [0] * (D + 1) for k in range(-P, P + 1)}
    pos = {k: t0 + (offs[k - 1] if k > 0 else -offs[-k - 1]) for k in range(-P, P + 1) if k != 0}
    pos[0] = t0
    for k in range(1, P + 1):
        for d in range(1, D + 1):
            if K % 2 == 1 and k == 1 and d % 2 == 1:
                continue
            a[k][d] = rint(np.float64(shat_row[k - 1][d]) * scale[d])
            a[-k][d] = (-1) ** (d + 1) * a[k][d]
    if K % 2 == 0:
        for d in range(1, D + 1, 2):
            acc = 0
            for k in range(-P, 0):
                for j in range(d, D + 1):
                    acc += comb(j, d) * a[k][j] * (t0 - pos[k]) ** (j - d)
            a[0][d] = -2 * acc
    else:
        for d in sorted(range(1, D + 1, 2), reverse=True):
            acc = 0
            for k in range(-P, -1):
                acc += a[k][d]
            for j in range(d + 1, D + 1):
                inner = 0
                for k in range(-P, 0):
                    inner += a[k][j] * (t0 - pos[k]) ** (j - d)
                acc += comb(j, d) * inner
            a[-1][d] = -acc
            a[1][d] = (-1) ** (d + 1) * a[-1][d]
    out = []
    for k in range(-P, P + 1):
        if k == 0 and K % 2 == 1:
            continue
        out.append((pos[k], k + P, list(a[k])))
    return out


def shift(coefs, delta):
    """Localized coefficients moved forward by delta (Eq. accumulation-rule without the jump)."""
    D = len(coefs) - 1
    return [sum(comb(j, d) * coefs[j] * delta ** (j - d) for j in range(d, D + 1)) for d in range(D + 1)]


def accumulate(knots):
    """Sequential exact accumulation (Eq. accumulation-rule) over knots sorted by position.

    Returns the list of (position, coefficients after the knot).
    """
    out = []
    state = None
    prev = None
    for t, _, jump in knots:
        if state is None:
            state = list(jump)
        else:
            state = shift(state, t - prev)
            state = [s + j for s, j in zip(state, jump)]
        prev = t
        out.append((t, list(state)))
    return out


def accumulate_wrapped(dist, jumps, g, steps, bits):
    """Final state of accumulator g of the integer bit-length study (Sec. 5.1): the accumulation
    rule (Eq. accumulation-rule) over `steps` knots in wrap-around `bits`-bit integers.

    dist: table of knot distances (distance from the previous knot); jumps: table of jump
    coefficient lists (integers, any sign).  Knot s of accumulator g is table entry
    (g + s mod 4) mod len(dist); knot 0 sits at position 0 and knot s > 0 at the previous position
    plus that entry's distance.  The accumulation is done exactly (accumulate above) and reduced
    modulo 2^bits at the end, which equals reducing after every multiply and add because reduction
    modulo 2^bits is a ring homomorphism of the integers.  Returns the D + 1 residues in
    [0, 2^bits)."""
    n = len(dist)
    seq = []
    t = 0
    for s in range(steps):
        k = (g + s % 4) % n
        if s > 0:
            t += int(dist[k])
        seq.append((t, k, [int(x) for x in jumps[k]]))
    final = accumulate(seq)[-1][1]
    m = 1 << bits
    return [x % m for x in final]
