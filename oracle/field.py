"""Per-ray field: sort, exact accumulation, exact pieces, peak and merge.

Sec. 2 (three passes): every contributing particle emits its knots onto the
ray, the ray's knots are sorted by position, and one sweep applies the
integer accumulation rule (Eq. accumulation-rule) to obtain, at every knot,
the localized coefficients of the piece that starts there.

Order: knots are sorted by (position t, particle input index, kidx); knots at
equal positions simply add, so the order among them does not change the field,
but it is fixed so that it can be compared.

Exact pieces: one piece per distinct knot position except the last, from that
position to the next one, with the coefficients after the last knot at that
position.  Because every particle's knots cancel exactly (App. A.3), the
coefficients after the ray's last knot are zero, and the field is zero outside
the pieces.

Peak (this implementation's reading of the ray's peak value): sigma times the
largest |a_0| over the starts of the exact pieces.

Merge (the paper has no merge step; this is this implementation's definition,
a plain greedy pass over the whole ray): starting at the first exact piece, the
current merged interval [a, b] is extended by the next exact piece as long as
the extension passes, and a new merged interval starts at the first piece whose
addition fails.  An interval passes when the squared L2 distance r of the
exact field F from P, the L2 projection of F onto polynomials of degree <= D
on the interval, satisfies r <= (tol * peak)^2 * (b - a) (lengths in world
units), i.e. the RMS error is at most tol * peak.  A single exact piece always
passes (F is itself a polynomial of degree <= D there).  P and r are computed
directly from the exact pieces of the interval, with no incremental update:
Gauss-Legendre quadrature with D + 1 nodes on every exact piece (exact for the
degree-2D integrands), P in the shifted Legendre basis of the interval,
r = sum over the pieces of the quadrature of (F - P)^2.  With tol = 0 nothing
is merged.  The smallest relative distance of any decision from its threshold
is kept as the ray's margin (decisions closer than rounding to the threshold
may differ between two float64 evaluations).

check_merged validates any merged field given as (start, end, coefficients)
against the exact pieces, independently of how it was produced: breakpoints on
exact piece boundaries, contiguous cover of the exact pieces, every merged
piece within the tolerance (residual of the projection, recomputed here) and
its coefficients equal to that projection within a stated bar.

Pinned by tests/test_oracle_field.py: the accumulation against brute-force
evaluation of every particle's own polynomial, the zero tail, the merge
partition invariants, the merge's decisions against the same greedy pass run
in exact rational arithmetic (monomial moments and a Gram solve with Python
fractions, a different formulation), moments 0..D of every merged piece, and
the checker against planted mistakes.
"""
from __future__ import annotations

import math

import numpy as np

from . import geometry, knots as knots_mod, lut as lut_mod



def ray_knots(o, v, t_min, t_max, xyz, zeta, value, table, quanta, K, D, kind, hits=None, transverse=None):
    """All knots of one ray, sorted by (t, pid, kidx).

    table: dict with 'theta' [n, P] and 'shat' [n, P, D+1]; quanta: (tau, sigma).
    transverse = a (0, 1, 2): every pair's amplitude is the particle's value times the pair factor
    m = ((o + t_chi v - chi) . e_a) / zeta of the transverse gradient fields (oracle.gradient).
    Returns (hits, sorted list of (t, pid, kidx, coefs)).
    """
    q = 2.0
    if hits is None:
        hits = geometry.ray_hits(o, v, t_min, t_max, xyz, zeta, q)
    tau, sigma = quanta
    n_lut = len(table["theta"])
    out = []
    chi = geometry.widen(xyz)
    z = geometry.widen(zeta)
    val = geometry.widen(value)
    o = np.asarray(o, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    for pid in hits:
        lam2, tchi = geometry.pair_terms(o, v, chi[pid], z[pid])
        lam = math.sqrt(float(lam2))
        li = lut_mod.lut_index(kind, lam, n_lut)
        amp = val[pid]
        if transverse is not None:
            from .gradient import pair_factor

            amp = np.float64(val[pid]) * np.float64(pair_factor(o, v, chi[pid], z[pid], transverse))
        for (t, kidx, coefs) in knots_mod.pair_knots(float(tchi), z[pid], amp, table["theta"][li],
                                                   table["shat"][li], tau, sigma, K, D):
            out.append((t, int(pid), kidx, coefs))
    out.sort(key=lambda e: (e[0], e[1], e[2]))
    return hits, out


def exact_pieces(sorted_knots):
    """(pieces, tail) where pieces = [(t_start, t_end, coefs, knot_index)] and tail = final state.

    knot_index is the sorted-knot index of the last knot at t_start (where the piece starts).
    """
    acc = knots_mod.accumulate([(t, k, c) for (t, _, k, c) in sorted_knots])
    pieces = []
    for i, (t, state) in enumerate(acc):
        last_of_group = (i + 1 == len(acc)) or (acc[i + 1][0] != t)
        if last_of_group and i + 1 < len(acc):
            pieces.append((t, acc[i + 1][0], state, i))
    tail = acc[-1][1] if acc else []
    return pieces, tail


def peak(pieces, sigma):
    """sigma * max |a_0| over the starts of the exact pieces (0 for an empty ray)."""
    if not pieces:
        return 0.0
    return float(sigma) * float(max(abs(p[2][0]) for p in pieces))


# ---------------------------------------------------------------- merge machinery

def _shifted_legendre(D):
    """Shifted Legendre polynomials P~_j(u) = P_j(2u - 1), j = 0..D, as power-basis rows [j, power]."""
    from numpy.polynomial import legendre as L
    from numpy.polynomial import polynomial as Pw

    rows = []
    for j in range(D + 1):
        c = np.zeros(j + 1)
        c[j] = 1.0
        pw = L.leg2poly(c)  # in x
        acc = np.zeros(1)
        for m, cm in enumerate(pw):
            acc = Pw.polyadd(acc, cm * Pw.polypow([-1.0, 2.0], m))
        row = np.zeros(D + 1)
        row[: len(acc)] = acc
        rows.append(row)
    return np.array(rows)


class Projector:
    """L2 projections of a ray's exact field onto polynomials of degree <= D on unions of
    consecutive exact pieces, computed directly from the pieces (float64)."""

    def __init__(self, pieces, D, tau, sigma):
        self.D = D
        self.tau = float(tau)
        self.sigma = float(sigma)
        self.L = _shifted_legendre(D)
        xg, wg = np.polynomial.legendre.leggauss(D + 1)
        self.xg = 0.5 * (xg + 1.0)   # nodes on [0, 1]
        self.wg = 0.5 * wg
        n = len(pieces)
        self.start = np.array([p[0] for p in pieces], dtype=np.int64)
        self.end = np.array([p[1] for p in pieces], dtype=np.int64)
        lens = (self.end - self.start).astype(np.float64)
        # F at the Gauss nodes of every piece: sigma * sum_d a_d x^d, x in quanta from the piece start
        F = np.zeros((n, D + 1))
        for i, p in enumerate(pieces):
            x = lens[i] * self.xg
            F[i] = self.sigma * sum(float(p[2][d]) * x ** d for d in range(D + 1))
        self.F = F
        self.lens = lens

    def legendre_at(self, u):
        return np.array([np.polyval(self.L[j][::-1], u) for j in range(self.D + 1)])

    def node(self, lo, hi):
        """Projection and residual of the union of pieces lo..hi (inclusive)."""
        a, b = int(self.start[lo]), int(self.end[hi])
        Lq = float(b - a)
        off = (self.start[lo:hi + 1] - a).astype(np.float64)
        x = off[:, None] + self.lens[lo:hi + 1, None] * self.xg[None, :]       # quanta from a
        w = self.lens[lo:hi + 1, None] * self.wg[None, :]                      # quanta
        F = self.F[lo:hi + 1]
        Pj = self.legendre_at(x / Lq)                                          # [j, piece, node]
        g = np.array([(2 * j + 1) / Lq * np.sum(w * F * Pj[j]) for j in range(self.D + 1)])
        P = np.tensordot(g, Pj, axes=1)
        r = self.tau * float(np.sum(w * (F - P) ** 2))
        return {"a": a, "b": b, "g": g, "r": r, "lo": lo, "hi": hi}

    def threshold(self, node, tol, pk):
        return (tol * pk) ** 2 * (float(node["b"] - node["a"]) * self.tau)

    def to_power(self, node):
        """Coefficients c_d of the node's polynomial in powers of u = (t - t_a) / (t_b - t_a)."""
        return node["g"] @ self.L


def merge(pieces, tol, tau, sigma, D):
    """Greedy merge over the whole ray (definition in the module docstring).

    Returns (nodes, projector, margin)."""
    M = Projector(pieces, D, tau, sigma)
    margin = float("inf")
    n = len(pieces)
    if n == 0:
        return [], M, margin
    if tol <= 0.0:
        return [M.node(i, i) for i in range(n)], M, margin
    pk = peak(pieces, sigma)
    nodes = []
    s = 0
    while s < n:
        cur = M.node(s, s)
        e = s
        while e + 1 < n:
            cand = M.node(s, e + 1)
            thr = M.threshold(cand, tol, pk)
            if thr > 0.0:
                margin = min(margin, abs(cand["r"] - thr) / thr)
            if cand["r"] <= thr:
                cur = cand
                e += 1
            else:
                break
        nodes.append(cur)
        s = e + 1
    return nodes, M, margin


def check_merged(pieces, merged, tol, tau, sigma, D, coef_tol=1e-5, resid_slack=1e-9, ends=None):
    """Validity of a merged field against the ray's exact pieces.

    merged: [(qa, qb, coef)] with qa, qb the piece ends in length quanta (integers) and coef the
    power coefficients in u = (t - qa tau) / ((qb - qa) tau), or, when ends = [(ta, tb)] is given
    (world positions, one pair per merged piece, e.g. roundings of the exact ends), in
    u = (t - ta) / (tb - ta) (a piece with ta = tb is the constant coef[0]).  Checks that the breakpoints are exact
    piece boundaries, that the merged pieces cover the exact pieces contiguously, that each merged
    piece's projection residual is within (tol * peak)^2 * length (up to a relative slack for the
    rounding of the two float64 evaluations), and that its coefficients equal that projection within
    coef_tol * peak at 17 points of the piece.  Returns a dict with 'errors' (empty when valid),
    'n' (merged pieces), 'max_coef_err' and 'max_resid_ratio' (relative to the peak / threshold)."""
    errors = []
    out = {"errors": errors, "n": len(merged), "max_coef_err": 0.0, "max_resid_ratio": 0.0}
    if not pieces:
        if merged:
            errors.append("pieces on an empty ray")
        return out
    if not merged:
        errors.append("no pieces on a non-empty ray")
        return out
    M = Projector(pieces, D, tau, sigma)
    pk = peak(pieces, sigma)
    index_of_start = {int(s): i for i, s in enumerate(M.start)}
    index_of_end = {int(e): i for i, e in enumerate(M.end)}
    if int(merged[0][0]) != int(M.start[0]):
        errors.append("first merged piece does not start at the first exact piece")
    if int(merged[-1][1]) != int(M.end[-1]):
        errors.append("last merged piece does not end at the last exact piece")
    for (qa, _, _), (_, qb_prev, _) in zip(merged[1:], merged[:-1]):
        if int(qa) != int(qb_prev):
            errors.append(f"gap or overlap at {qa} / {qb_prev}")
    us = np.linspace(0.0, 1.0, 17)
    for i, (qa, qb, coef) in enumerate(merged):
        qa, qb = int(qa), int(qb)
        if qa not in index_of_start or qb not in index_of_end or qb <= qa:
            errors.append(f"merged piece [{qa}, {qb}) not on exact piece boundaries")
            continue
        lo, hi = index_of_start[qa], index_of_end[qb]
        node = M.node(lo, hi)
        if tol <= 0.0:
            if lo != hi:
                errors.append(f"merged piece [{qa}, {qb}) joins exact pieces with merging off")
        else:
            thr = M.threshold(node, tol, pk)
            ratio = node["r"] / thr if thr > 0 else (0.0 if node["r"] == 0 else float("inf"))
            out["max_resid_ratio"] = max(out["max_resid_ratio"], ratio)
            if lo != hi and node["r"] > thr * (1.0 + resid_slack):
                errors.append(f"merged piece [{qa}, {qb}) exceeds the tolerance (ratio {ratio})")
        ref = np.polyval(M.to_power(node)[::-1], us)
        cf = np.asarray(coef, dtype=np.float64)
        if ends is None:
            got = np.polyval(cf[::-1], us)
        else:
            ta, tb = float(ends[i][0]), float(ends[i][1])
            ts = (qa + us * (qb - qa)) * float(tau)
            got = np.polyval(cf[::-1], (ts - ta) / (tb - ta)) if tb != ta else np.full_like(us, cf[0])
        err = float(np.max(np.abs(got - ref))) / pk if pk > 0 else float(np.max(np.abs(got - ref)))
        out["max_coef_err"] = max(out["max_coef_err"], err)
        if err > coef_tol:
            errors.append(f"merged piece [{qa}, {qb}) coefficients off the projection by {err} of the peak")
    return out


def ray_field(o, v, t_min, t_max, xyz, zeta, value, table, quanta, K, D, kind, tol, hits=None, transverse=None):
    """Everything the oracle knows about one ray (dict); transverse: as in ray_knots."""
    hits, sk = ray_knots(o, v, t_min, t_max, xyz, zeta, value, table, quanta, K, D, kind, hits=hits,
                         transverse=transverse)
    pieces, tail = exact_pieces(sk)
    tau, sigma = quanta
    nodes, M, margin = merge(pieces, tol, tau, sigma, D)
    return {"hits": hits, "knots": sk, "pieces": pieces, "tail": tail, "peak": peak(pieces, sigma),
            "nodes": nodes, "merger": M, "margin": margin}


def node_output(node, M):
    """(t_start, t_end, power coefficients in u) in world units (float64)."""
    return node["a"] * M.tau, node["b"] * M.tau, M.to_power(node)


def node_output_q(node, M):
    """(start, end in length quanta, power coefficients in u), the form check_merged takes."""
    return node["a"], node["b"], M.to_power(node)
