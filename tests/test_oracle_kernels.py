"""Pins of oracle.kernels against the paper's printed constants and independent quadrature."""
import math

import mpmath
import numpy as np
import pytest

from oracle import kernels as K


@pytest.mark.parametrize("kind", K.KINDS)
def test_unit_volume(kind):
    # an SPH kernel integrates to one over R^3
    assert abs(K.volume_integral(kind) - 1.0) < 1e-13


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
    assert abs(K.column_integral(kind, 0.0) - 2 * fac * tot) < 1e-14
    if kind == "cubic":
        assert abs(K.column_integral(kind, 0.0) - 3 / (2 * math.pi)) < 1e-14
    # summing the line integrals over all rays of one direction gives the volume integral (= 1)
    v, _ = integrate.quad(lambda l: l * K.column_integral(kind, l), 0, 2, points=[1.0], epsabs=0, epsrel=1e-13)
    assert abs(2 * math.pi * v - 1.0) < 1e-11
