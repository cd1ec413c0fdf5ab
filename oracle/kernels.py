"""SPH kernel functions and the kernel constants used by the error analysis.

Follows the paper's introduction (Eq. cubic-kernel: the cubic B-spline with
support bound q = 2), Sec. 3.1 (the normalized ray-restricted kernel
B_Lambda(t) = w(sqrt(Lambda^2 + t^2))) and Sec. 4.4 / App. A.4 (the constants
kappa and kappa').  The Wendland kernels are not in the paper (it allows any
piecewise polynomial kernel); they are the standard 3-D forms with support 2h:
  C2: (21/16pi)   (1 - r/2)^4 (1 + 2r),
  C4: (495/256pi) (1 - r/2)^6 (1 + 3r + 35/12 r^2),
  C6: (1365/512pi)(1 - r/2)^8 (1 + 4r + 25/4 r^2 + 4 r^3)  on [0, 2).

Gradient fields (Sec. 6 says the procedure carries over to other features that the particles
generate additively, gradients among them): with y = (x - chi)/h a particle's gradient is
h^-4 w'(r) y / r.  On a ray its part across the ray is a field of the radial function
g(r) = -w'(r)/r, which for the Wendland kernels is again (1 - r/2)^m times a polynomial:
  C2: (21/16pi) 5 (1 - r/2)^3,
  C4: (495/256pi) (14/3) (1 - r/2)^5 (1 + 5r/2),
  C6: (1365/512pi) (11/2) (1 - r/2)^7 (1 + 7r/2 + 4r^2)
(kinds "<kernel>_grad"; pinned against difference quotients of w and by
4 pi int r^2 g dr = 4 pi int_0^2 w dr, which integration by parts gives).

Every kernel here is a piecewise polynomial in r, stored as
(r_lo, r_hi, ascending coefficients) times a constant factor, so that the
integrals below can be written out in closed form.

Pinned by tests/test_oracle_kernels.py: kappa and kappa' against the values
printed in App. A.4, unit volume integral, the column integral against an
independent high-precision quadrature and against 2*int_0^q w and the
normalisation 2*pi*int Lambda*Sigma(Lambda) dLambda = 1.
"""
from __future__ import annotations

import functools
import math

import numpy as np
from numpy.polynomial import polynomial as P
from fractions import Fraction

CUBIC = "cubic"
WENDLAND = "wendland"        # Wendland C2
WENDLAND_C4 = "wendland_c4"
WENDLAND_C6 = "wendland_c6"
WENDLAND_GRAD = "wendland_grad"
WENDLAND_C4_GRAD = "wendland_c4_grad"
WENDLAND_C6_GRAD = "wendland_c6_grad"
GRAD_OF = {WENDLAND: WENDLAND_GRAD, WENDLAND_C4: WENDLAND_C4_GRAD, WENDLAND_C6: WENDLAND_C6_GRAD}
KINDS = (CUBIC, WENDLAND, WENDLAND_C4, WENDLAND_C6, WENDLAND_GRAD, WENDLAND_C4_GRAD, WENDLAND_C6_GRAD)

# Wendland kernels as (factor, power n of (1 - r/2), polynomial p ascending in r, exact)
_WENDLAND = {
    WENDLAND: (21.0 / (16.0 * math.pi), 4, [Fraction(1), Fraction(2)]),
    WENDLAND_C4: (495.0 / (256.0 * math.pi), 6, [Fraction(1), Fraction(3), Fraction(35, 12)]),
    WENDLAND_C6: (1365.0 / (512.0 * math.pi), 8, [Fraction(1), Fraction(4), Fraction(25, 4), Fraction(4)]),
    # g = -w'/r (module docstring)
    WENDLAND_GRAD: (21.0 / (16.0 * math.pi) * 5.0, 3, [Fraction(1)]),
    WENDLAND_C4_GRAD: (495.0 / (256.0 * math.pi) * (14.0 / 3.0), 5, [Fraction(1), Fraction(5, 2)]),
    WENDLAND_C6_GRAD: (1365.0 / (512.0 * math.pi) * 5.5, 7, [Fraction(1), Fraction(7, 2), Fraction(4)]),
}


def _pmul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def pieces_exact(kind: str):
    """Kernel pieces [(r_lo, r_hi, exact rational coefficients ascending in r)] and the
    constant factor (the only irrational part)."""
    if kind == CUBIC:
        # (2-r)^3 - 4(1-r)^3 = 4 - 6r^2 + 3r^3 on [0,1); (2-r)^3 on [1,2)
        return ([(0.0, 1.0, [Fraction(4), Fraction(0), Fraction(-6), Fraction(3)]),
                 (1.0, 2.0, [Fraction(8), Fraction(-12), Fraction(6), Fraction(-1)])], 1.0 / (4.0 * math.pi))
    if kind in _WENDLAND:
        fac, n, p = _WENDLAND[kind]
        poly = [Fraction(1)]
        for _ in range(n):
            poly = _pmul(poly, [Fraction(1), Fraction(-1, 2)])
        return [(0.0, 2.0, _pmul(poly, p))], fac
    raise ValueError(kind)

Q_SUPPORT = 2.0  # both kernels vanish for r >= 2


def support(kind: str) -> float:
    """Upper bound q of the kernel's support (Fig. 1 caption)."""
    if kind not in KINDS:
        raise ValueError(kind)
    return Q_SUPPORT


def pieces(kind: str):
    """Kernel as [(r_lo, r_hi, coeffs ascending in r)], and its constant factor.

    cubic (Eq. cubic-kernel):  (1/4pi)[(2-r)^3 - 4(1-r)^3] on [0,1) which expands
    to (1/4pi)(4 - 6r^2 + 3r^3), and (1/4pi)(2-r)^3 on [1,2).
    Wendland: factor (1-r/2)^n p(r) on [0,2) (module docstring).
    """
    if kind == CUBIC:
        inner = P.polysub(P.polypow([2.0, -1.0], 3), 4.0 * P.polypow([1.0, -1.0], 3))
        outer = P.polypow([2.0, -1.0], 3)
        return [(0.0, 1.0, inner), (1.0, 2.0, outer)], 1.0 / (4.0 * math.pi)
    if kind in _WENDLAND:
        pcs, fac = pieces_exact(kind)
        return [(lo, hi, np.array([float(c) for c in co])) for lo, hi, co in pcs], fac
    raise ValueError(kind)


def w(kind: str, r):
    """Kernel value w(r) for r >= 0 (zero outside the support); Wendland kernels are evaluated
    in their factored form, which has no cancellation near r = 2."""
    r = np.asarray(r, dtype=np.float64)
    if kind in _WENDLAND:
        return w_near_edge(kind, r, np.maximum(2.0 - r, 0.0) * (r >= 0))
    out = np.zeros_like(r)
    pcs, fac = pieces(kind)
    for lo, hi, c in pcs:
        m = (r >= lo) & (r < hi)
        out[m] = P.polyval(r[m], c)
    return fac * out


def w_near_edge(kind: str, r, two_minus_r):
    """w(r) evaluated with 2 - r supplied separately (accurate near r -> 2).

    Only the outermost piece uses the supplied 2 - r; every kernel is written as
    a polynomial in (2 - r) there: cubic (2-r)^3, Wendland ((2-r)/2)^n p(r).
    """
    r = np.asarray(r, dtype=np.float64)
    e = np.asarray(two_minus_r, dtype=np.float64)
    out = np.zeros_like(r)
    if kind == CUBIC:
        m_in = r < 1.0
        m_out = (r >= 1.0) & (e > 0.0)
        out[m_in] = (4.0 - 6.0 * r[m_in] ** 2 + 3.0 * r[m_in] ** 3) / (4.0 * math.pi)
        out[m_out] = e[m_out] ** 3 / (4.0 * math.pi)
        return out
    if kind in _WENDLAND:
        fac, n, p = _WENDLAND[kind]
        m = e > 0.0
        out[m] = fac * (0.5 * e[m]) ** n * P.polyval(r[m], [float(c) for c in p])
        return out
    raise ValueError(kind)


def breakpoints(kind: str):
    """Interior radii where the kernel's polynomial changes (excluding 0 and q)."""
    return [1.0] if kind == CUBIC else []


def w0(kind: str) -> float:
    """Kernel peak w(0): the cubic kernel gives 1/pi, Wendland C2 21/(16 pi)."""
    return float(w(kind, np.array([0.0]))[0])


def _int_exact(coefs, lo, hi, shift):
    """int_lo^hi sum_i c_i r^(i + shift) dr in exact rational arithmetic."""
    a, b = Fraction(lo), Fraction(hi)
    return sum(c * (b ** (i + shift + 1) - a ** (i + shift + 1)) / (i + shift + 1) for i, c in enumerate(coefs))


def volume_integral(kind: str) -> float:
    """4 pi int_0^q r^2 w(r) dr (must be 1 for a normalised SPH kernel); the polynomial part is
    integrated exactly."""
    pcs, fac = pieces_exact(kind)
    tot = sum(_int_exact(c, lo, hi, 2) for lo, hi, c in pcs)
    return 4.0 * math.pi * fac * float(tot)


def kappa(kind: str) -> float:
    """kappa = (4 pi int_0^inf [t w(t)]^2 dt)^(1/2)  (Sec. 4.4; App. A.4).

    The L2 norm of a normalized particle's contribution; the paper prints
    roughly 0.352 for the cubic kernel.
    """
    pcs, fac = pieces_exact(kind)
    tot = sum(_int_exact(_pmul(c, c), lo, hi, 2) for lo, hi, c in pcs)
    return math.sqrt(4.0 * math.pi * fac * fac * float(tot))


def dB_dt(kind: str, lam: float, t):
    """d/dt of B_Lambda(t) = w(sqrt(Lambda^2 + t^2)) (Sec. 3.1): w'(r) t / r."""
    t = np.asarray(t, dtype=np.float64)
    r = np.sqrt(lam * lam + t * t)
    pcs, fac = pieces(kind)
    out = np.zeros_like(t)
    for lo, hi, c in pcs:
        m = (r >= lo) & (r < hi) & (r > 0)
        out[m] = P.polyval(r[m], P.polyder(c)) * t[m] / r[m]
    return fac * out


@functools.lru_cache(maxsize=None)
def kappa_prime(kind: str) -> float:
    """kappa' = (int_0^q Lambda int_R [d/dt B_Lambda(t)]^2 dt dLambda)^(1/2).

    Evaluated from this definition (App. A.4) by nested adaptive quadrature that
    splits at the kernel's breakpoints.  The paper prints sqrt(14)/(7 pi) ~ 0.170
    for the cubic kernel.
    """
    from scipy import integrate

    q = support(kind)
    bps = breakpoints(kind)

    def inner(lam):
        s = math.sqrt(max(q * q - lam * lam, 0.0))
        pts = [math.sqrt(b * b - lam * lam) for b in bps if b > lam]
        edges = [0.0] + sorted(pts) + [s]
        tot = 0.0
        for a, b in zip(edges[:-1], edges[1:]):
            if b > a:
                v, _ = integrate.quad(lambda t: dB_dt(kind, lam, np.array([t]))[0] ** 2, a, b,
                                      epsabs=0.0, epsrel=1e-12, limit=200)
                tot += v
        return 2.0 * tot  # the integrand is even in t

    outer_pts = sorted(set(bps))
    edges = [0.0] + outer_pts + [q]
    tot = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        v, _ = integrate.quad(lambda lam: lam * inner(lam), a, b, epsabs=0.0, epsrel=1e-12, limit=200)
        tot += v
    return math.sqrt(tot)


def _power_antiderivative(n: int, lam, t):
    """Antiderivative in t of r^n with r = sqrt(lam^2 + t^2), lam > 0 (mpmath numbers).

    Even n: expand (lam^2 + t^2)^(n/2) binomially.  Odd n: the reduction
    K_n = (t r^n + n lam^2 K_{n-2}) / (n + 1) with K_{-1} = asinh(t / lam).
    """
    import mpmath

    if n % 2 == 0:
        m = n // 2
        return sum(math.comb(m, j) * lam ** (2 * (m - j)) * t ** (2 * j + 1) / (2 * j + 1)
                   for j in range(m + 1))
    r = mpmath.sqrt(lam * lam + t * t)
    k = mpmath.asinh(t / lam)  # K_{-1}
    for p in range(1, n + 1, 2):
        k = (t * r ** p + p * lam * lam * k) / (p + 1)
    return k


def column_integral(kind: str, lam: float, digits: int = 60) -> float:
    """Sigma(Lambda) = int_R B_Lambda(t) dt, the line integral of the kernel.

    Closed form: on each kernel piece r in [r_lo, r_hi) the integrand is a
    polynomial in r, and each power r^n has the antiderivative above; the
    t-range of a piece is sqrt(max(r_lo^2 - Lambda^2, 0)) .. sqrt(r_hi^2 - Lambda^2).
    The antiderivatives cancel heavily for grazing rays (Lambda -> q), so they
    are evaluated with ``digits`` significant digits (mpmath) and rounded once.
    """
    import mpmath

    q = support(kind)
    if lam >= q:
        return 0.0
    pcs, fac = pieces(kind)
    with mpmath.workdps(digits):
        L = mpmath.mpf(lam)
        tot = mpmath.mpf(0)
        for lo, hi, c in pcs:
            if hi <= lam:
                continue
            ta = mpmath.sqrt(max(mpmath.mpf(lo) ** 2 - L * L, 0))
            tb = mpmath.sqrt(mpmath.mpf(hi) ** 2 - L * L)
            for n, cn in enumerate(c):
                if cn == 0.0:
                    continue
                cm = mpmath.mpf(cn)
                if lam == 0.0:
                    tot += cm * (tb ** (n + 1) - ta ** (n + 1)) / (n + 1)
                else:
                    tot += cm * (_power_antiderivative(n, L, tb) - _power_antiderivative(n, L, ta))
        return float(2 * mpmath.mpf(fac) * tot)
