"""L2-optimal piecewise polynomial approximation of the ray-restricted kernel.

Sec. 3.2 defines the candidate space S_{K,D}(theta): even, continuous, compactly
supported piecewise polynomials of degree <= D with at most K non-trivial
pieces and positive knots theta_1 < ... < theta_P, P = ceil(K/2).  The error
measure is the L2 distance to B_Lambda(t) = w(sqrt(Lambda^2 + t^2))
(Eq. distance-related-approximation-error).  Sec. 3.3 gives the non-orthogonal
basis A~_kd over the index set J (App. A.1) and states that the orthogonal
projection of B_Lambda onto the space is the unique optimum for fixed knots
(Eq. optimal-approx-for-given-knots, App. A.2).  Any exact solution of the
normal equations G c = b in the basis A~ is that same projection, which is what
``project`` computes (the Gram-Schmidt route of Sec. 3.3 produces an identical
function).  Sec. 3.4 then optimises the knots; ``optimal_knots`` does that with
a gradient method (the gradient of the squared error follows from the
stationarity of the projection) polished by Newton steps, from several starts.

Sec. 2 encodes a piecewise polynomial by knots carrying localized difference
coefficients; ``difference_coefficients`` converts the projection into the
coefficients s^_kd at the knots +theta_k (and at 0 for even K) that the
look-up table of Sec. 3.1 holds.

Inner products are computed by Gauss-Legendre quadrature after substituting
t = Lambda sinh(u), which makes sqrt(Lambda^2 + t^2) = Lambda cosh(u) analytic,
on subintervals split at the knots, at the kernel's breakpoints and at the end
of the support s = sqrt(q^2 - Lambda^2).

Pinned by tests/test_oracle_lut.py: the dimension floor(K D / 2) of the space
(Sec. 3.3), orthogonality of the residual to every basis function (App. A.2),
evenness/continuity/compact support of the result, local optimality of the
knots, the overall approximation errors E_{K,D} printed in Fig. 4, and the line
integral of the approximation against the closed-form kernel column integral.
The storage rounding of the table precision study (round_storage) is pinned by
hand-worked ties, torch's float32 -> bfloat16 and numpy's float32 -> float16
conversions.

Parity unpinned: the knot positions themselves.  The paper prints only the errors E_{K,D} they
reach (Fig. 4), so the positions are pinned through those errors and local optimality, not
against printed values.
"""
from __future__ import annotations

import math

import numpy as np

from . import kernels

_GL_CACHE = {}


def _gauss_legendre(n: int):
    if n not in _GL_CACHE:
        _GL_CACHE[n] = np.polynomial.legendre.leggauss(n)
    return _GL_CACHE[n]


def n_pos_knots(K: int) -> int:
    """P = ceil(K/2) positive knot positions (Sec. 3.3)."""
    return (K + 1) // 2


def index_set(K: int, D: int):
    """J: pairs (k, d), 1 <= k <= P, 1 <= d <= D, without (1, odd d) when K is odd."""
    P = n_pos_knots(K)
    return [(k, d) for k in range(1, P + 1) for d in range(1, D + 1)
            if not (K % 2 == 1 and k == 1 and d % 2 == 1)]


def basis_value(theta, k: int, d: int, t):
    """A~_kd(t) of Sec. 3.3 (theta[0] = 0 is prepended by the caller)."""
    a, b = theta[k - 1], theta[k]
    at = np.abs(t)
    z = (at - a) / (b - a)
    out = np.where(at <= a, 1.0, 1.0 - np.clip(z, 0.0, 1.0) ** d)
    return np.where(at >= b, 0.0, out)


def basis_dtheta(theta, k: int, d: int, t, j: int):
    """Derivative of A~_kd(t) with respect to theta_j (j >= 1).

    On [theta_{k-1}, theta_k], with z = (|t| - theta_{k-1}) / Delta:
    d/dtheta_k = (d / Delta) z^d and d/dtheta_{k-1} = (d / Delta) z^(d-1) (1 - z);
    zero elsewhere (A~ is continuous, so moving a boundary adds nothing).
    """
    a, b = theta[k - 1], theta[k]
    at = np.abs(t)
    inside = (at > a) & (at < b)
    z = np.where(inside, (at - a) / (b - a), 0.0)
    if j == k:
        v = d / (b - a) * z ** d
    elif j == k - 1:
        v = d / (b - a) * z ** (d - 1) * (1.0 - z)
    else:
        return np.zeros_like(t)
    return np.where(inside, v, 0.0)


def _quadrature(kind: str, lam: float, theta, n_gl: int = 16, max_du: float = 0.5):
    """Nodes t >= 0 and weights on [0, max(theta_P, s)] with the splits described above.

    Returns (t, w_t, B) with B = B_Lambda(t) evaluated accurately near the support end.
    """
    q = kernels.support(kind)
    s2 = (q - lam) * (q + lam)
    s = math.sqrt(s2)
    cuts = {0.0, s}
    for th in theta[1:]:
        cuts.add(float(th))
    for rb in kernels.breakpoints(kind):
        if rb > lam:
            cuts.add(math.sqrt((rb - lam) * (rb + lam)))
    edges = sorted(c for c in cuts if c >= 0.0)
    xg, wg = _gauss_legendre(n_gl)
    ts, ws = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        if b <= a:
            continue
        if b <= s and lam > 0.0:
            ua, ub = math.asinh(a / lam), math.asinh(b / lam)
            m = max(1, int(math.ceil((ub - ua) / max_du)))
            us = np.linspace(ua, ub, m + 1)
            for u0, u1 in zip(us[:-1], us[1:]):
                u = 0.5 * (u1 - u0) * xg + 0.5 * (u1 + u0)
                t = lam * np.sinh(u)
                ts.append(t)
                ws.append(0.5 * (u1 - u0) * wg * lam * np.cosh(u))
        else:
            t = 0.5 * (b - a) * xg + 0.5 * (b + a)
            ts.append(t)
            ws.append(0.5 * (b - a) * wg)
    t = np.concatenate(ts)
    wt = np.concatenate(ws)
    r = np.sqrt(lam * lam + t * t)
    inside = t < s
    e = np.where(inside, (s - t) * (s + t) / (q + r), 0.0)  # q - r without cancellation
    B = np.where(inside, kernels.w_near_edge(kind, r, e), 0.0)
    return t, wt, B


def project(kind: str, lam: float, theta_pos, K: int, D: int, want_grad: bool = False):
    """Optimal approximation for fixed knots (Eq. optimal-approx-for-given-knots).

    Returns a dict with the basis coefficients c (over ``index_set``), the squared
    error E^2 = ||S - B_Lambda||^2, ||B_Lambda||^2, and optionally dE^2/dtheta.
    """
    theta = np.concatenate([[0.0], np.asarray(theta_pos, dtype=np.float64)])
    J = index_set(K, D)
    t, wt, B = _quadrature(kind, lam, theta)
    A = np.stack([basis_value(theta, k, d, t) for (k, d) in J])
    # both sides of the even functions: factor 2
    G = 2.0 * (A * wt) @ A.T
    b = 2.0 * (A * wt) @ B
    try:
        c = np.linalg.solve(G, b)
    except np.linalg.LinAlgError:  # knots collapsed: no longer a basis
        return {"c": None, "J": J, "E2": math.inf, "B2": float(2.0 * np.sum(wt * B * B)), "theta": theta,
                "grad": np.zeros(len(theta) - 1)}
    S = c @ A
    R = B - S
    out = {"c": c, "J": J, "E2": float(2.0 * np.sum(wt * R * R)), "B2": float(2.0 * np.sum(wt * B * B)),
           "theta": theta}
    if want_grad:
        g = np.zeros(len(theta) - 1)
        for j in range(1, len(theta)):
            dS = np.zeros_like(t)
            for ci, (k, d) in zip(c, J):
                if k == j or k - 1 == j:
                    dS += ci * basis_dtheta(theta, k, d, t, j)
            g[j - 1] = -2.0 * 2.0 * np.sum(wt * R * dS)
        out["grad"] = g
    return out


def _y_from_p(p):
    return np.cumsum(np.exp(p))


def _p_from_y(y):
    y = np.asarray(y, dtype=np.float64)
    return np.log(np.diff(np.concatenate([[0.0], y])))


def _local_opt(kind, lam, K, D, y0, s):
    """Minimise E^2 over knots y = theta / s from y0.

    Damped Newton on the analytic gradient (central-difference Hessian) in the
    coordinates p with y_1 = exp(p_1), y_k = y_{k-1} + exp(p_k), which keeps the
    knots ordered; falls back to BFGS when the Hessian is not positive definite.
    """
    from scipy import optimize

    scale = project(kind, lam, s * np.asarray(y0), K, D)["B2"]

    def fg(p):
        y = _y_from_p(p)
        r = project(kind, lam, s * y, K, D, want_grad=True)
        # chain rule: dE2/dp_i = sum_{j>=i} dE2/dy_j * exp(p_i), and dy = s dtheta
        gy = r["grad"] * s
        gp = np.cumsum(gy[::-1])[::-1] * np.exp(p)
        return r["E2"] / scale, gp / scale

    def hess(p, hstep=1e-5):
        n = len(p)
        H = np.zeros((n, n))
        for i in range(n):
            e = np.zeros(n)
            e[i] = hstep
            H[:, i] = (fg(p + e)[1] - fg(p - e)[1]) / (2 * hstep)
        return 0.5 * (H + H.T)

    p = _p_from_y(y0)
    f0, g0 = fg(p)
    converged = False
    for _ in range(60):
        H = hess(p)
        try:
            np.linalg.cholesky(H)
            step = np.linalg.solve(H, g0)
        except np.linalg.LinAlgError:
            break
        lam_ls = min(1.0, 1.0 / max(1e-300, float(np.max(np.abs(step)))))
        while lam_ls > 1e-4:
            p_new = p - lam_ls * step
            f1, g1 = fg(p_new)
            if f1 <= f0 + 1e-15 * abs(f0):
                break
            lam_ls *= 0.5
        else:
            break
        p, f0, g0 = p_new, f1, g1
        if np.max(np.abs(lam_ls * step)) < 1e-12:
            converged = True
            break
    if not converged:
        res = optimize.minimize(fg, p, jac=True, method="BFGS", options={"gtol": 1e-13, "maxiter": 500})
        p = res.x
        for _ in range(8):
            f0, g0 = fg(p)
            H = hess(p)
            try:
                np.linalg.cholesky(H)
                step = np.linalg.solve(H, g0)
            except np.linalg.LinAlgError:
                break
            if fg(p - step)[0] > f0 * (1 + 1e-14):
                break
            p = p - step
            if np.max(np.abs(step)) < 1e-12:
                break
    y = _y_from_p(p)
    return y, project(kind, lam, s * y, K, D)["E2"]


def default_starts(P: int):
    """Fixed grid of starting shapes y = theta / s for the multistart (Sec. 3.4 asks for a
    global optimum; neighbouring local optima can differ by ~1 % in E^2, so the
    starts cover the plausible region rather than a few guesses)."""
    if P == 1:
        return [[0.3 + 0.1 * i] for i in range(9)]
    if P == 2:
        return [[y1, y2] for y1 in (0.2, 0.3, 0.4, 0.5, 0.6) for y2 in (0.7, 0.8, 0.9, 1.0, 1.1)]
    if P == 3:
        return [[y1, y2, y3] for y1 in (0.15, 0.3, 0.45) for y2 in (0.5, 0.65, 0.8) for y3 in (0.9, 1.0, 1.1)]
    raise ValueError("K <= 6 supported")


def optimal_knots(kind: str, lam: float, K: int, D: int, extra_starts=()):
    """Optimal positive knots theta_1..theta_P for B_Lambda (Sec. 3.4).

    Multistart local optimisation in s-normalised coordinates y = theta / s,
    s = sqrt(q^2 - Lambda^2); the best local optimum is returned.
    """
    q = kernels.support(kind)
    s = math.sqrt((q - lam) * (q + lam))
    best = None
    for y0 in list(default_starts(n_pos_knots(K))) + [list(e) for e in extra_starts]:
        y, e2 = _local_opt(kind, lam, K, D, y0, s)
        # a start whose local search leaves the admissible shapes (non-finite E^2) is no optimum
        if np.isfinite(e2) and np.all(np.isfinite(y)) and (best is None or e2 < best[1]):
            best = (y, e2)
    return s * best[0], best[1]


def lambda_midpoints(kind: str, n: int):
    """Table abscissae Lambda_i = (i + 1/2) q / n (equidistant, Sec. 3.1)."""
    q = kernels.support(kind)
    return (np.arange(n) + 0.5) * q / n


def lut_index(kind: str, lam: float, n: int) -> int:
    """Nearest table entry for distance parameter Lambda (Sec. 4.3: 'closest').

    With midpoints, the closest entry is floor(Lambda * n / q), clamped.
    """
    q = kernels.support(kind)
    i = int(math.floor(lam * n / q))
    return min(max(i, 0), n - 1)


def _best_from(kind, lam, K, D, starts):
    q = kernels.support(kind)
    s = math.sqrt((q - lam) * (q + lam))
    best = None
    for y0 in starts:
        if not np.all(np.isfinite(y0)):
            continue
        y, e2 = _local_opt(kind, lam, K, D, list(y0), s)
        if np.isfinite(e2) and np.all(np.isfinite(y)) and (best is None or e2 < best[1]):
            best = (y, e2)
    return best


def knot_table(kind: str, K: int, D: int, n: int, pool=None):
    """Optimal knots theta[i] for every table abscissa Lambda_i (Sec. 3.4).

    Pass 1: best local optimum from the fixed starts ``default_starts``.
    Pass 2: entry i also tries the pass-1 optima of entries i-1 and i+1 (in
    s-normalised form) as starts and keeps the best.  Every entry depends only on
    pass-1 results, so the table does not depend on evaluation order.
    Returns (Lambda, theta [n, P], E^2 [n]).
    """
    lams = lambda_midpoints(kind, n)
    P = n_pos_knots(K)
    starts = default_starts(P)
    mapper = map if pool is None else pool.map
    p1 = list(mapper(_pass1, [(kind, float(l), K, D, starts) for l in lams]))
    jobs = []
    for i, l in enumerate(lams):
        cand = [p1[i][0]]
        if i > 0:
            cand.append(p1[i - 1][0])
        if i + 1 < n:
            cand.append(p1[i + 1][0])
        jobs.append((kind, float(l), K, D, cand))
    p2 = list(mapper(_pass1, jobs))
    q = kernels.support(kind)
    out = np.zeros((n, P))
    e2 = np.zeros(n)
    for i, l in enumerate(lams):
        y, err = p2[i] if p2[i][1] <= p1[i][1] else p1[i]
        out[i] = math.sqrt((q - l) * (q + l)) * np.asarray(y)
        e2[i] = err
    return lams, out, e2


def _pass1(args):
    kind, lam, K, D, starts = args
    y, e2 = _best_from(kind, lam, K, D, starts)
    return list(y), e2


def piece_polynomials(kind: str, lam: float, theta_pos, K: int, D: int):
    """Polynomials p_1..p_P of the projection on the positive pieces, in global t.

    p_m applies on [theta_{m-1}, theta_m]; A~_kd is 1 for k > m, 1 - z^d for k = m
    and 0 for k < m there.
    """
    from numpy.polynomial import Polynomial as Poly

    r = project(kind, lam, theta_pos, K, D)
    theta = r["theta"]
    P = n_pos_knots(K)
    polys = []
    for m in range(1, P + 1):
        a, b = theta[m - 1], theta[m]
        z = Poly([-a / (b - a), 1.0 / (b - a)])
        p = Poly([0.0])
        for ci, (k, d) in zip(r["c"], r["J"]):
            if k > m:
                p = p + ci
            elif k == m:
                p = p + ci * (1.0 - z ** d)
        polys.append(p)
    return polys, r


def _localized(poly, at, D):
    """Coefficients of poly(at + v) in powers of v (Sec. 2, localized coefficients)."""
    from numpy.polynomial import Polynomial as Poly

    shifted = poly(Poly([at, 1.0]))
    c = np.zeros(D + 1)
    cc = shifted.coef
    c[: min(len(cc), D + 1)] = cc[: D + 1]
    return c


def difference_coefficients(kind: str, lam: float, theta_pos, K: int, D: int):
    """Localized difference coefficients of the projection (Sec. 2 knot encoding).

    Returns (s_hat, s_mid): s_hat[k-1, d] for the knot at +theta_k, k = 1..P, the
    change p_{k+1} - p_k (p_{P+1} = 0) written in powers of (t - theta_k); and
    s_mid[d], the change at t = 0 for even K (p_1(t) - p_1(-t): twice the odd
    coefficients of p_1), all zeros for odd K.
    """
    from numpy.polynomial import Polynomial as Poly

    polys, _ = piece_polynomials(kind, lam, theta_pos, K, D)
    P = n_pos_knots(K)
    theta = np.concatenate([[0.0], np.asarray(theta_pos, dtype=np.float64)])
    s_hat = np.zeros((P, D + 1))
    for k in range(1, P + 1):
        nxt = polys[k] if k < P else Poly([0.0])
        s_hat[k - 1] = _localized(nxt - polys[k - 1], theta[k], D)
    s_hat[:, 0] = 0.0  # continuity: the value jump is zero by construction
    s_mid = np.zeros(D + 1)
    if K % 2 == 0:
        c0 = _localized(polys[0], 0.0, D)
        for d in range(1, D + 1, 2):
            s_mid[d] = 2.0 * c0[d]
    return s_hat, s_mid


def lut_entries(kind: str, K: int, D: int, thetas):
    """(s_hat[n, P, D+1], s_mid[n, D+1]) for every row of a knot table."""
    lams = lambda_midpoints(kind, len(thetas))
    P = n_pos_knots(K)
    sh = np.zeros((len(thetas), P, D + 1))
    sm = np.zeros((len(thetas), D + 1))
    for i, (lam, th) in enumerate(zip(lams, thetas)):
        sh[i], sm[i] = difference_coefficients(kind, float(lam), th, K, D)
    return sh, sm


def overall_error(kind: str, K: int, D: int, n: int, thetas=None):
    """E_{K,D} of Sec. 5.2: (1/kappa) (2 pi int_0^q Lambda E_Lambda^2 dLambda)^(1/2).

    Approximated, as in the paper, by a Riemann sum (midpoints of n intervals).
    """
    q = kernels.support(kind)
    lams = lambda_midpoints(kind, n)
    if thetas is None:
        _, thetas, e2 = knot_table(kind, K, D, n)
    else:
        e2 = np.array([project(kind, float(l), th, K, D)["E2"] for l, th in zip(lams, thetas)])
    integral = np.sum(lams * e2) * (q / n)
    return math.sqrt(2.0 * math.pi * integral) / kernels.kappa(kind), thetas, e2


def round_storage(values, fmt: str):
    """Table values as a float table stored in `fmt` holds them, returned as float64 (the table
    precision study; the table is that of Sec. 3.1).

    fp64: unchanged.  fp32: the nearest float32.  bf16: the nearest float32, then the nearest
    number with 8 significant bits, ties to even: with f = m 2^e, 1/2 <= |m| < 1 (frexp), the
    result is rint(256 m) / 256 * 2^e (rint rounds half to even; every step is exact in float64).
    fp16: the nearest float32, then the nearest IEEE binary16: 11 significant bits for
    |f| >= 2^-14 (rint(2048 m) / 2048 * 2^e), multiples of 2^-24 below (subnormals), infinity
    beyond the largest finite value 65504."""
    a = np.asarray(values, dtype=np.float64)
    if fmt == "fp64":
        return a.copy()
    f = a.astype(np.float32).astype(np.float64)
    if fmt == "fp32":
        return f
    m, e = np.frexp(f)
    if fmt == "bf16":
        return np.ldexp(np.rint(m * 256.0) / 256.0, e)
    if fmt != "fp16":
        raise ValueError(fmt)
    normal = np.ldexp(np.rint(m * 2048.0) / 2048.0, e)
    sub = np.rint(f * 2.0 ** 24) * 2.0 ** -24
    r = np.where(np.abs(f) >= 2.0 ** -14, normal, sub)
    return np.where(np.abs(r) > 65504.0, np.copysign(np.inf, f), r)
