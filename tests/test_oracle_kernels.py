"""Pins of oracle.kernels against the paper's printed constants and independent quadrature."""
import math

import mpmath
import numpy as np
import pytest

from oracle import kernels as K


BASE_OF = {g: b for b, g in K.GRAD_OF.items()}


def expected_volume(kind):
    """1 for an SPH kernel; for g = -w'/r integration by parts gives
    4 pi int_0^2 r^2 g dr = -4 pi int_0^2 r w' dr = 4 pi int_0^2 w dr (w(2) = 0), taken here by
    adaptive quadrature of the base kernel."""
    if kind not in BASE_OF:
        return 1.0
    from scipy import integrate

    v, _ = integrate.quad(lambda r: K.w(BASE_OF[kind], np.array([r]))[0], 0, 2, epsabs=0, epsrel=2e-14)
    return 4 * math.pi * v


@pytest.mark.parametrize("kind", K.KINDS)
def test_unit_volume(kind):
    # an SPH kernel integrates to one over R^3; a gradient kernel to the by-parts value
    assert abs(K.volume_integral(kind) - expected_volume(kind)) < 1e-13 * max(1.0, expected_volume(kind))


@pytest.mark.parametrize("grad", sorted(BASE_OF))
def test_gradient_kernel_is_minus_dw_over_r(grad):
    # g(r) = -w'(r)/r against central difference quotients of the base kernel
    base = BASE_OF[grad]
    r = np.linspace(0.02, 1.98, 50)
    e = 1e-5
    dw = (K.w(base, r + e) - K.w(base, r - e)) / (2 * e)
    g = K.w(grad, r)
    assert np.max(np.abs(g + dw / r)) < 1e-8 * np.max(np.abs(g))
    # the gradient of a particle is w'(r) y / r: compare with difference quotients of w(|y|) in 3-D
    rng = np.random.default_rng(3)
    for _ in range(5):
        y = rng.uniform(-1.1, 1.1, 3)
        rr = np.linalg.norm(y)
        num = np.array([(K.w(base, np.array([np.linalg.norm(y + e * ax)]))[0]
                         - K.w(base, np.array([np.linalg.norm(y - e * ax)]))[0]) / (2 * e) for ax in np.eye(3)])
        ana = -K.w(grad, np.array([rr]))[0] * y
        assert np.max(np.abs(num - ana)) < 1e-8 * max(1e-3, np.max(np.abs(ana)))


def test_cubic_peak_and_pieces():
    # Eq. cubic-kernel: w(0) = (8 - 4) / 4pi, w(1) = 1/4pi, w(2) = 0, continuous at 1
    assert abs(K.w0("cubic") - 1.0 / math.pi) < 1e-15
    assert abs(K.w("cubic", np.array([1.0 - 1e-12]))[0] - 1 / (4 * math.pi)) < 1e-11
    assert abs(K.w("cubic", np.array([1.0]))[0] - 1 / (4 * math.pi)) < 1e-15
    assert K.w("cubic", np.array([2.0]))[0] == 0.0


def test_kappa_printed_cubic():
    # App. A.4 prints kappa ~ 0.352 for the cubic kernel
    assert abs(K.kappa("cubic") - 0.352) < 5e-4


def test_kappa_prime_printed_cubic():
    # App. A.4 prints kappa' = sqrt(14) / (7 pi) for the cubic kernel
    assert abs(K.kappa_prime("cubic") - math.sqrt(14) / (7 * math.pi)) < 1e-11


@pytest.mark.parametrize("kind", K.KINDS)
def test_kappa_against_mpmath(kind):
    mpmath.mp.dps = 30
    pcs, fac = K.pieces(kind)

    def wm(r):
        for lo, hi, c in pcs:
            if lo <= r < hi:
                return fac * sum(mpmath.mpf(cc) * r ** i for i, cc in enumerate(c))
        return mpmath.mpf(0)

    v = mpmath.quad(lambda t: (t * wm(t)) ** 2, [0, 1, 2])
    assert abs(float(mpmath.sqrt(4 * mpmath.pi * v)) - K.kappa(kind)) < 1e-12


@pytest.mark.parametrize("kind", K.KINDS)
@pytest.mark.parametrize("lam", [0.0, 1e-4, 0.3, 0.99, 1.0, 1.01, 1.7, 1.999])
def test_column_integral_against_mpmath(kind, lam):
    # 60 digits: near the support edge the power-basis integrand cancels to ~1e-27 of its terms
    mpmath.mp.dps = 60
    pcs, fac = K.pieces(kind)

    def B(t):
        r = mpmath.sqrt(mpmath.mpf(lam) ** 2 + t * t)
        for lo, hi, c in pcs:
            if lo <= r < hi:
                return fac * sum(mpmath.mpf(cc) * r ** i for i, cc in enumerate(c))
        return mpmath.mpf(0)

    s = math.sqrt(4 - lam * lam)
    pts = [0]
    if lam < 1:
        pts.append(math.sqrt(1 - lam * lam))
    pts.append(s)
    ref = 2 * mpmath.quad(B, pts)
    got = K.column_integral(kind, lam)
    assert abs(got - float(ref)) <= 1e-12 * max(1e-30, abs(float(ref))) + 1e-300


@pytest.mark.parametrize("kind", K.KINDS)
def test_column_integral_identities(kind):
    from scipy import integrate

    # Sigma(0) = 2 int_0^q w(r) dr
    pcs, fac = K.pieces(kind)
    tot = 0.0
    for lo, hi, c in pcs:
        ci = np.polynomial.polynomial.polyint(c)
        tot += np.polynomial.polynomial.polyval(hi, ci) - np.polynomial.polynomial.polyval(lo, ci)
    assert abs(K.column_integral(kind, 0.0) - 2 * fac * tot) < 1e-14 * max(1.0, 8 * abs(2 * fac * tot))
    if kind == "cubic":
        assert abs(K.column_integral(kind, 0.0) - 3 / (2 * math.pi)) < 1e-14
    # summing the line integrals over all rays of one direction gives the volume integral (= 1
    # for an SPH kernel)
    v, _ = integrate.quad(lambda l: l * K.column_integral(kind, l), 0, 2, points=[1.0], epsabs=0, epsrel=1e-13)
    assert abs(2 * math.pi * v - expected_volume(kind)) < 1e-11 * max(1.0, expected_volume(kind))
