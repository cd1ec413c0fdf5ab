"""Quantization error estimate and the choice of the two quanta.

Sec. 4.2 fixes the coefficient quanta sigma_d = sigma / tau^d, leaving a length
quantum tau and a value quantum sigma.  Sec. 4.4 (derived in App. A.4) gives the
relative quantization error estimate

    Q_D(tau, sigma) = 1/(4 kappa) * sqrt( kappa'^2 tau^2
                       + sum_{d=0..D} 2 q^(2d+3) / ((2d+1)(2d+3)) * sigma^2 / tau^(2d) ),

sets sigma = a_max / INT_MAX, and chooses tau as the minimiser of
Q_D(tau / h_repr, sigma / phi_repr), which App. A.5 shows to be the unique root
of dQ^2/dtau (a strictly increasing function of tau).

Pinned by tests/test_oracle_quanta.py against the grey bars of Fig. 4
(Q_2 .. Q_6 for 64-bit integers and a data-variance ratio of 1e5) and against
the stationarity of Q at the returned tau.
"""
from __future__ import annotations

import math

from . import kernels


def int_max(bits: int) -> int:
    """Largest representable signed integer of the given bit length (Sec. 4.4)."""
    return (1 << (bits - 1)) - 1


def _terms(kind: str, D: int):
    q = kernels.support(kind)
    return [2.0 * q ** (2 * d + 3) / ((2 * d + 1) * (2 * d + 3)) for d in range(D + 1)]


def Q(kind: str, D: int, tau: float, sigma: float, kap=None, kapp=None) -> float:
    """Quantization error estimate Q_D(tau, sigma) of a normalized particle."""
    kap = kernels.kappa(kind) if kap is None else kap
    kapp = kernels.kappa_prime(kind) if kapp is None else kapp
    s = kapp * kapp * tau * tau
    for d, c in enumerate(_terms(kind, D)):
        s += c * sigma * sigma / tau ** (2 * d)
    return math.sqrt(s) / (4.0 * kap)


def dQ2_dtau(kind: str, D: int, tau: float, sigma: float, kap: float, kapp: float) -> float:
    """First derivative of Q_D^2 with respect to tau (App. A.5)."""
    q = kernels.support(kind)
    v = kapp * kapp * tau / (8.0 * kap * kap)
    for d in range(1, D + 1):
        v -= d * q ** (2 * d + 3) / (4.0 * kap * kap * (2 * d + 1) * (2 * d + 3)) * sigma * sigma / tau ** (2 * d + 1)
    return v


def optimal_tau(kind: str, D: int, sigma: float, kap=None, kapp=None) -> float:
    """Minimiser of Q_D(., sigma): the root of dQ^2/dtau, by bisection on log(tau).

    App. A.5: dQ^2/dtau is negative for tau -> 0, positive for tau -> inf and
    strictly increasing, so the root is unique; bisection to the last bit.
    """
    if D < 1:
        raise ValueError("the length quantum is only determined for D >= 1")
    kap = kernels.kappa(kind) if kap is None else kap
    kapp = kernels.kappa_prime(kind) if kapp is None else kapp
    lo, hi = 1e-300, 1.0
    while dQ2_dtau(kind, D, hi, sigma, kap, kapp) <= 0.0:
        hi *= 2.0
    lo = hi
    while dQ2_dtau(kind, D, lo, sigma, kap, kapp) > 0.0:
        lo *= 0.5
    # lo < root <= hi; bisect until the interval no longer shrinks
    while True:
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if dQ2_dtau(kind, D, mid, sigma, kap, kapp) > 0.0:
            hi = mid
        else:
            lo = mid
    return hi


def sigma_from_amax(a_max: float, bits: int = 64) -> float:
    """sigma = a_max / INT_MAX (Sec. 4.4)."""
    return a_max / float(int_max(bits))


def choose_quanta(kind: str, D: int, a_max: float, h_repr: float, phi_repr: float, bits: int = 64):
    """(tau, sigma) for a data set (Sec. 4.4).

    sigma = a_max / INT_MAX; tau = h_repr * argmin_x Q_D(x, sigma / phi_repr),
    i.e. tau minimises Q_D(tau / h_repr, sigma / phi_repr).
    """
    sigma = sigma_from_amax(a_max, bits)
    x = optimal_tau(kind, D, sigma / phi_repr)
    return h_repr * x, sigma


def fig4_sigma_ratio(kind: str, bits: int = 64, variance_ratio: float = 1e5) -> float:
    """sigma / phi_repr for the Fig. 4 setting.

    Reading of "a_max / phi_repr = 1e5" (Sec. 5.2, Fig. 4 caption): the ratio is
    taken relative to the peak of the representative contribution,
    phi_repr * w(0), so sigma / phi_repr = 1e5 * w(0) / INT_MAX.  This reading
    reproduces the printed grey bars to all printed digits.
    """
    return variance_ratio * kernels.w0(kind) / float(int_max(bits))
