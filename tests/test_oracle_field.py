"""Pins of oracle.field (exact accumulation, pieces, merge), oracle.render and
oracle.geometry / oracle.grid."""
import math
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import field, geometry, grid, kernels, knots, lut, quanta, render


@pytest.fixture(scope="module")
def setup():
    kind, K, D, n = "cubic", 4, 2, 32
    _, th, _ = lut.knot_table(kind, K, D, n)
    sh, _ = lut.lut_entries(kind, K, D, th)
    xyz, h, val = synth.random_scene(5, 400, h_lo=0.04, h_hi=0.12)
    amax = grid.a_max(kind, xyz, h, val)
    hr, phr = grid.representatives(h, val)
    tau, sigma = quanta.choose_quanta(kind, D, amax, hr, phr)
    return dict(kind=kind, K=K, D=D, table={"theta": th, "shat": sh}, xyz=xyz, h=h, val=val, q=(tau, sigma))


def _ray(seed):
    o, v = synth.random_rays(seed, 1)
    return o[0].astype(np.float64), v[0].astype(np.float64)


def test_accumulation_equals_sum_of_particles(setup):
    """Eq. accumulation-rule on the merged knot list gives, at every integer position,
    exactly the sum of the particles' own encoded polynomials (Sec. 2)."""
    s = setup
    o, v = _ray(11)
    hits, sk = field.ray_knots(o, v, -10.0, 10.0, s["xyz"], s["h"], s["val"], s["table"], s["q"], s["K"], s["D"], s["kind"])
    assert len(hits) > 5
    pieces, tail = field.exact_pieces(sk)
    assert tail == [0] * (s["D"] + 1)
    per = {}
    for (t, pid, kidx, a) in sk:
        per.setdefault(pid, []).append((t, kidx, a))

    def own(pid, x):
        return sum(sum(a[d] * (x - t) ** d for d in range(len(a))) for t, _, a in per[pid] if t <= x)

    rng = np.random.default_rng(0)
    for (ta, tb, coefs, _) in pieces[:: max(1, len(pieces) // 25)]:
        for x in {ta, int(rng.integers(ta, tb)), tb - 1}:
            ray_val = sum(coefs[d] * (x - ta) ** d for d in range(len(coefs)))
            assert ray_val == sum(own(p, x) for p in per)


def test_knot_order_and_pieces(setup):
    s = setup
    o, v = _ray(12)
    hits, sk = field.ray_knots(o, v, -10.0, 10.0, s["xyz"], s["h"], s["val"], s["table"], s["q"], s["K"], s["D"], s["kind"])
    keys = [(t, p, k) for (t, p, k, _) in sk]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    assert len(sk) == (s["K"] + 1) * len(hits)
    pieces, _ = field.exact_pieces(sk)
    distinct = sorted({t for t, _, _, _ in sk})
    assert [p[0] for p in pieces] == distinct[:-1] and [p[1] for p in pieces] == distinct[1:]


def test_empty_ray(setup):
    s = setup
    f = field.ray_field(np.array([5.0, 5.0, 5.0]), np.array([0.0, 0.0, 1.0]), 0.0, 1.0, s["xyz"], s["h"], s["val"],
                        s["table"], s["q"], s["K"], s["D"], s["kind"], 1e-3)
    assert len(f["hits"]) == 0 and f["pieces"] == [] and f["peak"] == 0.0 and f["nodes"] == []


def _exact_poly(coefs, ta, tb, sigma):
    """Exact field on a piece as rational polynomial coefficients in u in [0, 1]."""
    L = tb - ta
    return [Fraction(sigma) * coefs[d] * L ** d for d in range(len(coefs))]


def _legendre_exact(D):
    from numpy.polynomial import legendre as Lg
    rows = []
    for j in range(D + 1):
        c = [0] * j + [1]
        pw = [Fraction(x).limit_denominator(10 ** 6) for x in Lg.leg2poly(c)]
        # substitute x = 2u - 1
        acc = [Fraction(0)] * (D + 1)
        for m, cm in enumerate(pw):
            term = [Fraction(1)]
            for _ in range(m):
                term = [a * -1 for a in term] + [Fraction(0)]
                term = [term[i] + (2 * (term[i - 1] if i > 0 else 0) if False else 0) for i in range(len(term))]
            # expand (2u - 1)^m exactly
            poly = [Fraction(math.comb(m, i)) * Fraction(2) ** i * Fraction(-1) ** (m - i) for i in range(m + 1)]
            for i, pc in enumerate(poly):
                acc[i] += cm * pc
        rows.append(acc)
    return rows


def _int_poly(p, lo, hi):
    """int_lo^hi of a rational polynomial in u."""
    return sum(c * (Fraction(hi) ** (i + 1) - Fraction(lo) ** (i + 1)) / (i + 1) for i, c in enumerate(p))


def _pmul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _compose_affine(p, s0, s1):
    """p(s0 + s1 u) as coefficients in u (exact)."""
    out = [Fraction(0)]
    for i, c in enumerate(p):
        term = [Fraction(1)]
        for _ in range(i):
            term = _pmul(term, [Fraction(s0), Fraction(s1)])
        out = [x + y for x, y in zip(out + [Fraction(0)] * (len(term) - len(out)), [c * t for t in term] + [Fraction(0)] * (len(out) - len(term)))]
    return out


@pytest.mark.parametrize("tol", [1e-2, 1e-3])
def test_merge_invariants_exact(setup, tol):
    """Merged nodes partition the exact pieces; each node's residual, recomputed in exact
    rational arithmetic from the integer pieces, is within tol * peak in the RMS sense, and
    the node polynomial reproduces the field's moments 0..D (it is the L2 projection)."""
    s = setup
    D = s["D"]
    tau, sigma = s["q"]
    o, v = _ray(13)
    f = field.ray_field(o, v, -10.0, 10.0, s["xyz"], s["h"], s["val"], s["table"], s["q"], s["K"], D, s["kind"], tol)
    pieces, nodes, M = f["pieces"], f["nodes"], f["merger"]
    assert pieces and nodes
    assert nodes[0]["a"] == pieces[0][0] and nodes[-1]["b"] == pieces[-1][1]
    starts = {p[0] for p in pieces}
    for A, B in zip(nodes[:-1], nodes[1:]):
        assert A["b"] == B["a"] and B["a"] in starts
    assert len(nodes) < len(pieces)
    pk = Fraction(f["peak"])
    for node in nodes[:: max(1, len(nodes) // 6)]:
        a, b = node["a"], node["b"]
        inside = [p for p in pieces if a <= p[0] and p[1] <= b]
        Lw = Fraction(b - a)
        # exact field pieces in the node's u-coordinate
        segs = []
        for (ta, tb, coefs, _) in inside:
            p = _exact_poly(coefs, ta, tb, sigma)            # in u_p on [0,1]
            lo, hi = Fraction(ta - a) / Lw, Fraction(tb - a) / Lw
            # u_p = (u - lo) / (hi - lo)
            segs.append((lo, hi, _compose_affine(p, -lo / (hi - lo), 1 / (hi - lo))))
        Pn = [Fraction(x) for x in M.to_power(node)]
        # moments: int F u^j = int P u^j, j <= D
        for j in range(D + 1):
            mono = [Fraction(0)] * j + [Fraction(1)]
            mf = sum(_int_poly(_pmul(pp, mono), lo, hi) for lo, hi, pp in segs)
            mp = _int_poly(_pmul(Pn, mono), 0, 1)
            scale = sum(_int_poly(_pmul(pp, pp), lo, hi) for lo, hi, pp in segs)
            assert abs(float(mf - mp)) <= 1e-9 * math.sqrt(float(scale)) + 1e-300
        resid = Fraction(0)
        for lo, hi, pp in segs:
            diff = [x - y for x, y in zip(pp + [Fraction(0)] * (len(Pn) - len(pp)), Pn + [Fraction(0)] * (len(pp) - len(Pn)))]
            resid += _int_poly(_pmul(diff, diff), lo, hi)
        resid_world = resid * Lw * Fraction(tau)
        assert float(resid_world) <= float((Fraction(tol) * pk) ** 2 * Lw * Fraction(tau)) * (1 + 1e-9)
        assert abs(float(resid_world) - node["r"]) <= 1e-6 * float((Fraction(tol) * pk) ** 2 * Lw * Fraction(tau))


def _solve_exact(G, m):
    """Gaussian elimination in Python fractions (G symmetric positive definite)."""
    n = len(m)
    A = [list(G[i]) + [m[i]] for i in range(n)]
    for c in range(n):
        for r in range(c + 1, n):
            f = A[r][c] / A[c][c]
            for k in range(c, n + 1):
                A[r][k] -= f * A[c][k]
    y = [Fraction(0)] * n
    for r in range(n - 1, -1, -1):
        y[r] = (A[r][n] - sum(A[r][k] * y[k] for k in range(r + 1, n))) / A[r][r]
    return y


def _exact_greedy(pieces, tol, D):
    """The whole-ray greedy merge decided in exact rational arithmetic, by a formulation other
    than the oracle's: the field of each exact piece expanded in powers of x = t - a (a the merged
    interval's start, in quanta), running monomial moments m_k = int F x^k and the energy
    int F^2 added piece by piece, the projection from the Gram system G_jk = L^(j+k+1)/(j+k+1)
    and the residual int F^2 - m.y.  sigma^2 tau is common to the residual and the threshold
    (tol max|a_0|)^2 L, so both are compared without it.  Returns the merged intervals."""
    if not pieces:
        return []
    A0 = max(abs(int(p[2][0])) for p in pieces)
    tol_q = Fraction(tol)

    def piece_terms(p, a):
        ta, tb, c = p[0], p[1], [int(x) for x in p[2]]
        xi, xe = ta - a, tb - a
        # F(x) = sum_d c_d (x - xi)^d = sum_e ce_e x^e
        ce = [sum(c[d] * math.comb(d, e) * (-xi) ** (d - e) for d in range(e, D + 1)) for e in range(D + 1)]
        mom = [sum(Fraction(ce[e] * (xe ** (e + k + 1) - xi ** (e + k + 1)), e + k + 1) for e in range(D + 1))
               for k in range(D + 1)]
        en = sum(Fraction(ce[e] * ce[f] * (xe ** (e + f + 1) - xi ** (e + f + 1)), e + f + 1)
                 for e in range(D + 1) for f in range(D + 1))
        return mom, en

    out = []
    s, n = 0, len(pieces)
    while s < n:
        a = pieces[s][0]
        mom, en = piece_terms(pieces[s], a)
        e = s
        while e + 1 < n:
            m2, e2 = piece_terms(pieces[e + 1], a)
            mom_c = [x + y for x, y in zip(mom, m2)]
            en_c = en + e2
            Lq = pieces[e + 1][1] - a
            G = [[Fraction(Lq ** (j + k + 1), j + k + 1) for k in range(D + 1)] for j in range(D + 1)]
            y = _solve_exact(G, mom_c)
            resid = en_c - sum(mi * yi for mi, yi in zip(mom_c, y))
            if resid <= (tol_q * A0) ** 2 * Lq:
                mom, en, e = mom_c, en_c, e + 1
            else:
                break
        out.append((a, pieces[e][1]))
        s = e + 1
    return out


@pytest.mark.parametrize("seed,tol", [(13, 1e-2), (14, 1e-3), (17, 3e-3)])
def test_merge_equals_exact_rational_greedy(setup, seed, tol):
    """Every decision of the float64 greedy merge (extend while the projection's residual is
    within the tolerance, over the whole ray) is the decision exact rational arithmetic takes, so
    each merged interval is greedy-maximal: all its prefixes pass and adding the next exact piece
    fails."""
    s = setup
    o, v = _ray(seed)
    f = field.ray_field(o, v, -10.0, 10.0, s["xyz"], s["h"], s["val"], s["table"], s["q"], s["K"], s["D"],
                        s["kind"], tol)
    assert f["margin"] > 1e-9, f["margin"]
    got = [(n["a"], n["b"]) for n in f["nodes"]]
    assert len(got) > 3 and len(got) < len(f["pieces"])
    assert got == _exact_greedy(f["pieces"], tol, s["D"])


def test_merge_of_one_polynomial_is_one_piece():
    """Exact pieces that all carry one cubic (split at arbitrary integer points, coefficients by
    the exact Taylor shift) merge into a single piece whose residual is zero and whose coefficients
    are the cubic's, at any tolerance > 0; with tol = 0 nothing merges."""
    D = 3
    tau, sigma = 1e-4, 1e-12
    base = [7 * 10 ** 9, -3 * 10 ** 7, 5 * 10 ** 4, -11]          # polynomial in x = t - 1000 (quanta)
    cuts = [1000, 1013, 1040, 1041, 1100, 1177, 1300]

    def shifted(x0):
        return [sum(base[d] * math.comb(d, e) * (x0 - 1000) ** (d - e) for d in range(e, D + 1)) for e in range(D + 1)]

    pieces = [(a, b, shifted(a), i) for i, (a, b) in enumerate(zip(cuts[:-1], cuts[1:]))]
    nodes, M, _ = field.merge(pieces, 1e-6, tau, sigma, D)
    assert len(nodes) == 1 and nodes[0]["a"] == 1000 and nodes[0]["b"] == 1300
    assert nodes[0]["r"] <= 1e-20 * (sigma * base[0]) ** 2
    L = 300
    want = [sigma * base[d] * L ** d for d in range(D + 1)]
    assert np.allclose(M.to_power(nodes[0]), want, rtol=1e-12, atol=1e-12 * abs(want[0]))
    nodes0, _, _ = field.merge(pieces, 0.0, tau, sigma, D)
    assert [(n["a"], n["b"]) for n in nodes0] == [(a, b) for a, b, _, _ in pieces]


def test_check_merged_catches_planted_mistakes(setup):
    """The validity checker accepts the oracle's own merge and flags each planted mistake: a
    breakpoint off the exact knots, a gap, a piece that exceeds the tolerance, coefficients off
    the projection by 3e-5 of the peak, a missing tail, merging with tol = 0."""
    s = setup
    D = s["D"]
    tau, sigma = s["q"]
    tol = 1e-3
    o, v = _ray(13)
    f = field.ray_field(o, v, -10.0, 10.0, s["xyz"], s["h"], s["val"], s["table"], s["q"], s["K"], D, s["kind"], tol)
    pieces, M = f["pieces"], f["merger"]
    good = [field.node_output_q(n, M) for n in f["nodes"]]
    chk = field.check_merged(pieces, good, tol, tau, sigma, D)
    assert chk["errors"] == [] and chk["n"] == len(good) and chk["max_resid_ratio"] <= 1.0
    i = max(range(len(good) - 1), key=lambda k: good[k][1] - good[k][0])
    a, b, c = good[i]
    off = [list(x) for x in good]
    off[i][1] = b - 1
    off[i + 1][0] = b - 1
    assert field.check_merged(pieces, [tuple(x) for x in off], tol, tau, sigma, D)["errors"]
    gap = good[:i] + good[i + 1:]
    assert field.check_merged(pieces, gap, tol, tau, sigma, D)["errors"]
    # join every pair of neighbours: at least one union exceeds the tolerance
    joined = []
    for k in range(0, len(good) - 1, 2):
        lo = [p for p in range(len(pieces)) if pieces[p][0] == good[k][0]][0]
        hi = [p for p in range(len(pieces)) if pieces[p][1] == good[k + 1][1]][0]
        nd = M.node(lo, hi)
        joined.append(field.node_output_q(nd, M))
    if len(good) % 2:
        joined.append(good[-1])
    assert any("exceeds" in e for e in field.check_merged(pieces, joined, tol, tau, sigma, D)["errors"])
    pert = [list(x) for x in good]
    pert[i][2] = np.array(pert[i][2], dtype=np.float64)
    pert[i][2][0] += 3e-5 * f["peak"]
    assert any("coefficients" in e for e in field.check_merged(pieces, [tuple(x) for x in pert], tol, tau, sigma, D)["errors"])
    assert field.check_merged(pieces, good[:-1], tol, tau, sigma, D)["errors"]
    assert field.check_merged(pieces, good, 0.0, tau, sigma, D)["errors"]
    exact = [field.node_output_q(M.node(k, k), M) for k in range(len(pieces))]
    assert field.check_merged(pieces, exact, 0.0, tau, sigma, D)["errors"] == []


def test_check_merged_on_given_ends(setup):
    """Coefficients given on other ends (float32 roundings of the exact ones): the same polynomial
    re-expressed on those ends passes, the unchanged coefficients evaluated on shifted ends fail."""
    s = setup
    D = s["D"]
    tau, sigma = s["q"]
    tol = 1e-3
    o, v = _ray(13)
    f = field.ray_field(o, v, -10.0, 10.0, s["xyz"], s["h"], s["val"], s["table"], s["q"], s["K"], D, s["kind"], tol)
    pieces, M = f["pieces"], f["merger"]
    good = [field.node_output_q(n, M) for n in f["nodes"]]
    # ends moved by 1 % of each piece: u = al + be u' with al = (ta' - ta) / L, be = (tb' - ta') / L
    moved, recoef, ends = [], [], []
    for qa, qb, c in good:
        ta, tb = qa * tau, qb * tau
        L = tb - ta
        ta2, tb2 = ta + 0.01 * L, tb - 0.01 * L
        al, be = (ta2 - ta) / L, (tb2 - ta2) / L
        comp = np.polynomial.polynomial.polyval(np.polynomial.polynomial.Polynomial([al, be]),
                                                np.asarray(c, dtype=np.float64))
        recoef.append((qa, qb, comp.coef))
        moved.append((qa, qb, c))
        ends.append((ta2, tb2))
    assert field.check_merged(pieces, recoef, tol, tau, sigma, D, ends=ends)["errors"] == []
    assert any("coefficients" in e for e in field.check_merged(pieces, moved, tol, tau, sigma, D, ends=ends)["errors"])
    exact_ends = [(qa * tau, qb * tau) for qa, qb, _ in good]
    chk = field.check_merged(pieces, good, tol, tau, sigma, D, ends=exact_ends)
    assert chk["errors"] == [] and chk["max_coef_err"] < 1e-9


def test_field_close_to_sph_truth(setup):
    """The exact quantized field approximates the true SPH sum along the ray
    (relative L2 error of the order of E_{4,2} ~ 0.8 %, plus the nearest-entry error of a
    32-entry table: 2.2 % measured; 16 % with 8 entries, 1.4 % with 128)."""
    s = setup
    o, v = _ray(15)
    tau, sigma = s["q"]
    f = field.ray_field(o, v, -10.0, 10.0, s["xyz"], s["h"], s["val"], s["table"], s["q"], s["K"], s["D"], s["kind"], 0.0)
    ts = np.linspace(f["pieces"][0][0] * tau, f["pieces"][-1][1] * tau, 4001)
    chi = geometry.widen(s["xyz"])
    z = geometry.widen(s["h"])
    val = geometry.widen(s["val"])
    truth = np.zeros_like(ts)
    for i, t in enumerate(ts):
        r = np.linalg.norm(chi - (o + t * v), axis=1) / z
        truth[i] = np.sum(val / z ** 3 * kernels.w("cubic", r))
    approx = np.zeros_like(ts)
    for (ta, tb, c, _) in f["pieces"]:
        m = (ts >= ta * tau) & (ts < tb * tau)
        x = ts[m] / tau - ta
        approx[m] = sigma * sum(float(c[d]) * x ** d for d in range(len(c)))
    rel = np.sqrt(np.sum((approx - truth) ** 2) / np.sum(truth ** 2))
    assert rel < 0.03


def test_render_special_cases(setup):
    s = setup
    o, v = _ray(16)
    tau, sigma = s["q"]
    f = field.ray_field(o, v, -10.0, 10.0, s["xyz"], s["h"], s["val"], s["table"], s["q"], s["K"], s["D"], s["kind"], 0.0)
    out = [field.node_output(n, f["merger"]) for n in f["nodes"]]
    t0, t1 = out[0][0], out[-1][1]
    # zero emission, constant extinction: alpha = 1 - exp(-sigma * covered length)
    tf = np.zeros((4, 4))
    tf[:, 3] = 0.7
    px = render.composite(out, t0 - 1, t1 + 1, tf, 0.0, 1.0, 1e9)
    assert abs(px[3] - (1 - math.exp(-0.7 * (t1 - t0)))) < 1e-12 and np.all(px[:3] == 0)
    # emission linear in v, no extinction: pixel -> k * integral of F as the step shrinks
    vmax = 2 * f["peak"]
    tf = np.zeros((2, 4))
    tf[1, 0] = 1.0  # red emission = v / vmax
    exact = Fraction(0)
    for (ta, tb, c, _) in f["pieces"]:
        L = tb - ta
        exact += Fraction(sigma) * sum(Fraction(int(c[d])) * Fraction(L) ** (d + 1) / (d + 1) for d in range(len(c))) * Fraction(tau)
    px = render.composite(out, t0 - 1, t1 + 1, tf, 0.0, vmax, (t1 - t0) / 20000)
    assert abs(px[0] - float(exact) / vmax) < 1e-6 * abs(float(exact) / vmax)
    # empty ray
    assert np.all(render.composite([], 0.0, 1.0, tf, 0.0, 1.0, 0.01) == 0)


def test_geometry_against_direct_formula():
    rng = np.random.default_rng(3)
    o, v = synth.random_rays(4, 50)
    xyz, h, _ = synth.random_scene(6, 50)
    for i in range(50):
        oo, vv = o[i].astype(np.float64), v[i].astype(np.float64)
        lam2, tchi = geometry.pair_terms(oo[None], vv[None], geometry.widen(xyz), geometry.widen(h))
        dx = geometry.widen(xyz) - oo
        t_ref = dx @ vv
        perp = dx - np.outer(t_ref, vv)
        lam_ref = np.linalg.norm(perp, axis=1) / geometry.widen(h)
        assert np.allclose(tchi, t_ref, rtol=0, atol=1e-12)
        # float32 directions are unit only to ~1e-7, which both formulas see differently
        assert np.allclose(np.sqrt(lam2), lam_ref, rtol=1e-6, atol=1e-9)


def test_camera_rays_are_unit_and_centered():
    cam = synth.plain_camera(8, 6)
    o, v = geometry.camera_rays(cam)
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0, atol=1e-15)
    c = v.reshape(6, 8, 3)
    mid = 0.25 * (c[2, 3] + c[2, 4] + c[3, 3] + c[3, 4])
    f = np.array([0.0, 0.0, 2.0]) / 2.0
    assert np.allclose(mid / np.linalg.norm(mid), f, atol=1e-12)
    # top row looks up (+y), left column looks towards -x for this right-handed frame
    assert c[0, 3, 1] > 0 and c[5, 3, 1] < 0
    cam2 = synth.tiny_camera(4, 4)
    o2, v2 = geometry.camera_rays(cam2)
    assert np.allclose(v2, [0.0, 0.0, 1.0]) and np.allclose(o2[:, 2], -0.2)


def test_grid_levels_and_morton():
    xyz, h, val = synth.random_scene(7, 500, h_lo=0.005, h_hi=0.08)
    g, codes, perm = grid.morton_order(xyz, h)
    qz = 2.0 * geometry.widen(h)
    c = g["c0"] * 2.0 ** g["level"]
    assert np.all(qz <= c) and np.all((g["level"] == 0) | (qz > c / 2))
    assert math.frexp(g["c0"])[0] == 0.5  # power of two
    # Morton code against a bitwise interleave written differently
    for i in range(0, 500, 37):
        ix, iy, iz = (int(x) for x in g["cell"][i])
        ref = 0
        for b in range(21):
            ref |= ((ix >> b) & 1) << (3 * b) | ((iy >> b) & 1) << (3 * b + 1) | ((iz >> b) & 1) << (3 * b + 2)
        assert int(codes[i]) == ref
    keys = list(zip(g["level"][perm], codes[perm], perm))
    assert keys == sorted(keys)


def test_amax_bounds_the_field():
    kind = "cubic"
    xyz, h, val = synth.random_scene(8, 300, h_lo=0.02, h_hi=0.15, signed=True)
    am = grid.a_max(kind, xyz, h, val)
    chi = geometry.widen(xyz)
    z = geometry.widen(h)
    v = geometry.widen(val)
    rng = np.random.default_rng(0)
    pts = np.concatenate([chi[rng.integers(0, 300, 200)], rng.uniform(-0.1, 1.1, (200, 3))])
    for x in pts:
        r = np.linalg.norm(chi - x, axis=1) / z
        fld = np.sum(np.abs(v) / z ** 3 * kernels.w(kind, r))
        assert fld <= am / grid.AMAX_MARGIN
