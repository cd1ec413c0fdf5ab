"""Pins of oracle.knots: the integer closure of Sec. 4.3 / App. A.3."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import knots, lut, quanta


def _random_row(rng, K, D):
    P = lut.n_pos_knots(K)
    theta = np.sort(rng.uniform(0.1, 2.0, P))
    shat = rng.normal(0, 1.0, (P, D + 1))
    shat[:, 0] = 0.0
    return theta, shat


def _eval_exact(kn, x):
    """Value of the encoded function at integer position x (quanta units, exact):
    sum over knots at positions <= x of the jump polynomial (Sec. 2 encoding)."""
    v = 0
    for t, _, a in kn:
        if t <= x:
            v += sum(a[d] * (x - t) ** d for d in range(len(a)))
    return v


@pytest.mark.parametrize("K", range(1, 7))
@pytest.mark.parametrize("D", range(1, 7))
def test_closure_zero_tail_and_shifted_evenness(K, D):
    """App. A.3: every particle's quantized knots cancel exactly (compact support)
    and encode a function that is even about t0."""
    if (K * D) // 2 == 0:
        pytest.skip("empty candidate space")
    rng = np.random.default_rng(100 * K + D)
    for trial in range(40):
        theta, shat = _random_row(rng, K, D)
        tchi = rng.uniform(-3, 3)
        zeta = rng.uniform(0.001, 0.1)
        value = rng.lognormal(0, 2) * rng.choice([-1, 1])
        tau = 10 ** rng.uniform(-6, -3)
        sigma = 10 ** rng.uniform(-14, -8)
        kn = knots.pair_knots(tchi, zeta, value, theta, shat, tau, sigma, K, D)
        assert len(kn) == K + 1
        assert all(a[0] == 0 for _, _, a in kn)                 # value jumps vanish
        pos = sorted(kn, key=lambda e: (e[0], e[1]))
        acc = knots.accumulate(pos)
        assert acc[-1][1] == [0] * (D + 1)                      # exact zero tail
        t0 = int(np.rint(np.float64(tchi) / np.float64(tau)))
        ts = [t for t, _, _ in kn]
        assert sorted(ts) == sorted(2 * t0 - t for t in ts)     # symmetric positions
        span = max(ts) - min(ts)
        for u in rng.integers(0, span + 2, 12):
            assert _eval_exact(kn, t0 + int(u)) == _eval_exact(kn, t0 - int(u))


def test_quantized_close_to_table_function():
    """The quantized particle function stays close to the scaled, shifted table
    approximation (the quantization error of Sec. 4.4 is small for small quanta)."""
    kind, K, D, lam = "cubic", 4, 3, 0.7
    th, _ = lut.optimal_knots(kind, lam, K, D)
    sh, sm = lut.difference_coefficients(kind, lam, th, K, D)
    polys, r = lut.piece_polynomials(kind, lam, th, K, D)
    tchi, zeta, value = 0.4321, 0.03, 2.5
    # quanta chosen as in Sec. 4.4 for a data-variance ratio of 1e5 with this particle as representative
    phi = value / zeta ** 3
    ratio = quanta.fig4_sigma_ratio(kind)
    sigma = ratio * phi
    tau = zeta * quanta.optimal_tau(kind, D, ratio)
    kn = knots.pair_knots(tchi, zeta, value, th, sh, tau, sigma, K, D)
    theta = np.concatenate([[0.0], th])

    def S(x):  # unquantized approximation of the particle
        y = abs((x - tchi) / zeta)
        for m in range(1, len(theta)):
            if y <= theta[m]:
                return value / zeta ** 3 * polys[m - 1](y)
        return 0.0

    peak = value / zeta ** 3 * polys[0](0.0)
    for x in np.linspace(tchi - 2.1 * zeta, tchi + 2.1 * zeta, 301):
        xi = int(np.rint(x / tau))
        got = float(Fraction(_eval_exact(kn, xi)) * Fraction(sigma))
        # knots move by up to tau/2 = 3e-4 zeta: pointwise deviations of a few 1e-4 of the peak
        assert abs(got - S(xi * tau)) < 1e-3 * peak


def test_rint_ties_to_even():
    assert knots.rint(2.5) == 2 and knots.rint(3.5) == 4 and knots.rint(-2.5) == -2


def test_wrapped_accumulation_hand_case():
    """Sec. 5.1 study, worked by hand: D = 1, one table entry (distance 3, jump 1 + 2 x), four
    knots at 0, 3, 6, 9.  At the last knot the encoded function is sum_s (1 + 2 (x - t_s)): value
    4 + 2 (9 + 6 + 3 + 0) = 40, slope 8; in 4-bit arithmetic 8 and 8."""
    assert knots.accumulate_wrapped([3], [[1, 2]], 0, 4, 32) == [40, 8]
    assert knots.accumulate_wrapped([3], [[1, 2]], 0, 4, 4) == [8, 8]
    # two entries: knot s of accumulator 1 takes entry (1 + s mod 4) mod 2 = 1, 0, 1, 0
    # with distances 7 (entry 0) and 5 (entry 1): positions 0, 7, 12, 19; jumps x, 1, x, 1
    got = knots.accumulate_wrapped([7, 5], [[1, 0], [0, 1]], 1, 4, 64)
    assert got == [(19 - 0) + 1 + (19 - 12) + 1, 2]


@pytest.mark.parametrize("bits", [32, 64, 96, 128])
@pytest.mark.parametrize("D", [1, 3, 6])
def test_wrapped_accumulation_equals_encoded_function(bits, D):
    """The rule's state at the last knot is the encoded function re-expanded about that knot: its
    polynomial at x = t_last + u equals the sum of every knot's jump polynomial at x (the encoding
    of Sec. 2, evaluated directly), modulo 2^bits."""
    import synth

    dist, jumps = synth.bit_tables(seed=10 + D, n_table=5, degree=D, bits=bits)
    table = [[synth.limbs_to_int(jumps[k, d]) for d in range(D + 1)] for k in range(5)]
    m = 1 << bits
    for g in (0, 3, 7):
        steps = 12
        got = knots.accumulate_wrapped(dist, table, g, steps, bits)
        kn, t = [], 0
        for s in range(steps):
            k = (g + s % 4) % 5
            t += int(dist[k]) if s > 0 else 0
            kn.append((t, k, table[k]))
        for u in (0, 1, 2, 1000, 1 << 33):
            x = t + u
            assert sum(c * u ** d for d, c in enumerate(got)) % m == _eval_exact(kn, x) % m
