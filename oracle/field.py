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

Merge (the paper has no merge step; this is this implementation's definition):
the sorted knots are cut into chunks of MERGE_CHUNK consecutive knots, and the
exact piece that starts at knot i belongs to chunk floor(i / MERGE_CHUNK)
(a piece starts at the last knot of each group of equal positions).  Within a
chunk, pieces are merged greedily from left to right; then, for levels
l = 0, 1, ..., the node lists of chunk groups [g, g + 2^l) and
[g + 2^l, g + 2^(l+1)) are joined and their two boundary nodes merged when
the result passes.  A merged node over [a, b] carries the L2 projection P of
the exact field F onto polynomials of degree <= D on [a, b] and its residual
r = int_a^b (F - P)^2 dt; it passes when r <= (tol * peak)^2 * (b - a).
Projections use the shifted Legendre basis on [0, 1]; the projection of a
union and its residual follow exactly from the parts because F - P_part is
orthogonal to polynomials of degree <= D on the part:
  P_U = projection of (P_A on A, P_B on B);
  r_U = r_A + r_B + int_A (P_A - P_U)^2 + int_B (P_B - P_U)^2.
With tol = 0 nothing is merged.

Pinned by tests/test_oracle_field.py: the accumulation against brute-force
evaluation of every particle's own polynomial, the zero tail, the merge
partition invariants, residuals against exact rational arithmetic and the
greedy maximality of each chunk.
"""
from __future__ import annotations

import math

import numpy as np

from . import geometry, knots as knots_mod, lut as lut_mod

MERGE_CHUNK = 16


def ray_knots(o, v, t_min, t_max, xyz, zeta, value, table, quanta, K, D, kind, hits=None):
    """All knots of one ray, sorted by (t, pid, kidx).

    table: dict with 'theta' [n, P] and 'shat' [n, P, D+1]; quanta: (tau, sigma).
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
        for (t, kidx, coefs) in knots_mod.pair_knots(float(tchi), z[pid], val[pid], table["theta"][li],
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
    """Shifted Legendre polynomials P~_j(u) = P_j(2u - 1), j = 0..D, as power-basis rows."""
    from numpy.polynomial import legendre as L
    from numpy.polynomial import polynomial as Pw

    rows = []
    for j in range(D + 1):
        c = np.zeros(j + 1)
        c[j] = 1.0
        pw = L.leg2poly(c)  # in x
        # substitute x = 2u - 1
        acc = np.zeros(1)
        for m, cm in enumerate(pw):
            acc = Pw.polyadd(acc, cm * Pw.polypow([-1.0, 2.0], m))
        row = np.zeros(D + 1)
        row[: len(acc)] = acc
        rows.append(row)
    return np.array(rows)  # [j, power]


class Merger:
    """Legendre-basis L2 projections on intervals of the quantized line."""

    def __init__(self, D, tau, sigma):
        self.D = D
        self.tau = float(tau)
        self.sigma = float(sigma)
        self.L = _shifted_legendre(D)               # P~_j in powers of u
        xg, wg = np.polynomial.legendre.leggauss(D + 1)
        self.u = 0.5 * (xg + 1.0)                    # nodes on [0, 1]
        self.wu = 0.5 * wg
        self.Pu = self._leg_at(self.u)               # [j, node]

    def _leg_at(self, u):
        return np.array([np.polyval(self.L[j][::-1], u) for j in range(self.D + 1)])

    def leaf(self, t_a, t_b, coefs):
        """Node of an exact piece: F(u) = sigma * sum_d a_d (L u)^d, L = t_b - t_a quanta."""
        Lq = t_b - t_a
        beta = np.array([self.sigma * float(coefs[d]) * float(Lq) ** d for d in range(self.D + 1)])
        # Legendre coefficients: gamma_j = (2j+1) int_0^1 F P~_j du (exact by Gauss-Legendre)
        F = np.polyval(beta[::-1], self.u)
        gamma = np.array([(2 * j + 1) * np.sum(self.wu * F * self.Pu[j]) for j in range(self.D + 1)])
        return {"a": t_a, "b": t_b, "g": gamma, "r": 0.0}

    def eval(self, node, u):
        return np.sum(node["g"][:, None] * self._leg_at(np.atleast_1d(u)), axis=0)

    def combine(self, A, B):
        """Projection and residual of the union of adjacent nodes A = [a, b], B = [b, c]."""
        a, b, c = A["a"], A["b"], B["b"]
        lam = float(b - a) / float(c - a)
        uA = lam * self.u                 # A's nodes in union coordinates
        uB = lam + (1.0 - lam) * self.u   # B's nodes in union coordinates
        FA = self.eval(A, self.u)
        FB = self.eval(B, self.u)
        PA = self._leg_at(uA)
        PB = self._leg_at(uB)
        g = np.array([(2 * j + 1) * (lam * np.sum(self.wu * FA * PA[j]) + (1.0 - lam) * np.sum(self.wu * FB * PB[j]))
                      for j in range(self.D + 1)])
        U = {"a": a, "b": c, "g": g}
        dA = FA - np.sum(g[:, None] * PA, axis=0)
        dB = FB - np.sum(g[:, None] * PB, axis=0)
        lenA = float(b - a) * self.tau
        lenB = float(c - b) * self.tau
        U["r"] = A["r"] + B["r"] + lenA * np.sum(self.wu * dA * dA) + lenB * np.sum(self.wu * dB * dB)
        return U

    def passes(self, node, tol, pk):
        thr = (tol * pk) ** 2 * (float(node["b"] - node["a"]) * self.tau)
        if thr > 0.0:
            self.margin = min(self.margin, abs(node["r"] - thr) / thr)
        return node["r"] <= thr

    margin = float("inf")  # smallest relative distance of a merge decision from its threshold

    def to_power(self, node):
        """Coefficients c_d of the node's polynomial in powers of u = (t - t_a) / (t_b - t_a)."""
        return node["g"] @ self.L


def merge(sorted_knots, pieces, tol, tau, sigma, D, chunk=MERGE_CHUNK):
    """Merged nodes of one ray (definition in the module docstring)."""
    M = Merger(D, tau, sigma)
    pk = peak(pieces, sigma)
    if not pieces:
        return [], M
    leaves = [(M.leaf(a, b, c), ki) for (a, b, c, ki) in pieces]
    if tol <= 0.0:
        return [n for n, _ in leaves], M
    n_chunks = (len(sorted_knots) + chunk - 1) // chunk
    per_chunk = [[] for _ in range(n_chunks)]
    for node, ki in leaves:
        per_chunk[ki // chunk].append(node)
    groups = []
    for lst in per_chunk:
        out = []
        cur = None
        for node in lst:
            if cur is None:
                cur = node
                continue
            cand = M.combine(cur, node)
            if M.passes(cand, tol, pk):
                cur = cand
            else:
                out.append(cur)
                cur = node
        if cur is not None:
            out.append(cur)
        groups.append(out)
    width = 1
    while width < n_chunks:
        new_groups = []
        for g in range(0, len(groups), 2):
            left = groups[g]
            right = groups[g + 1] if g + 1 < len(groups) else None
            if right is None:
                new_groups.append(left)
                continue
            if left and right:
                cand = M.combine(left[-1], right[0])
                if M.passes(cand, tol, pk):
                    new_groups.append(left[:-1] + [cand] + right[1:])
                    continue
            new_groups.append(left + right)
        groups = new_groups
        width *= 2
    return groups[0], M


def ray_field(o, v, t_min, t_max, xyz, zeta, value, table, quanta, K, D, kind, tol, hits=None):
    """Everything the oracle knows about one ray (dict)."""
    hits, sk = ray_knots(o, v, t_min, t_max, xyz, zeta, value, table, quanta, K, D, kind, hits=hits)
    pieces, tail = exact_pieces(sk)
    tau, sigma = quanta
    nodes, M = merge(sk, pieces, tol, tau, sigma, D)
    return {"hits": hits, "knots": sk, "pieces": pieces, "tail": tail, "peak": peak(pieces, sigma),
            "nodes": nodes, "merger": M, "margin": M.margin}


def node_output(node, M):
    """(t_start, t_end, power coefficients in u) in world units (float64)."""
    return node["a"] * M.tau, node["b"] * M.tau, M.to_power(node)
