"""The hit test's short cut (the kernels' contribution test, Sec. 2's relevant pairs) against the
oracle's full test: a pair with Lambda^2 < q^2 whose centre t_chi lies strictly inside
(t_min, t_max) passes both end checks fl(t_chi + s zeta) > t_min and fl(t_chi - s zeta) < t_max
whatever s >= 0 is, because rounding is monotone and t_chi itself is a float64.  The device
skips the square root for such pairs; here the implication is checked on random and adversarial
float64 values (centres one ulp inside the interval, tiny and huge s zeta, signed zeros).
"""
import numpy as np

from oracle import geometry

Q = 2.0


def _shortcut(lam2, tchi, t_min, t_max):
    return (lam2 < Q * Q) & (tchi > t_min) & (tchi < t_max)


def _check(lam2, tchi, zeta, t_min, t_max):
    full = geometry.hit_mask(lam2, tchi, zeta, Q, t_min, t_max)
    short = _shortcut(lam2, tchi, t_min, t_max)
    # the short cut never accepts a pair the full test rejects ...
    assert not np.any(short & ~full)
    # ... and pairs it leaves undecided are exactly those the device still tests in full
    undecided = (lam2 < Q * Q) & ~short
    assert np.array_equal(full, short | (undecided & full))
    return int(short.sum()), int(full.sum())


def test_random_pairs():
    rng = np.random.default_rng(20240106)
    n = 400_000
    for scale in (1e-3, 1.0, 1e3, 1e7):
        t_min = rng.uniform(-scale, scale, n)
        t_max = t_min + rng.exponential(scale, n)
        tchi = rng.uniform(t_min - scale, t_max + scale)
        zeta = rng.exponential(scale * 0.1, n) + 1e-300
        lam2 = rng.uniform(0.0, 1.2 * Q * Q, n)
        s, f = _check(lam2, tchi, zeta, t_min, t_max)
        assert 0 < s <= f


def test_adversarial_pairs():
    t_min = np.array([0.0, -0.0, 1.0, -1e300, 5e-324, 1e16, -3.5, 0.1])
    t_max = np.array([1.0, 1e-300, 1.0 + 2 ** -52, 1e300, 1e-323, 1e16 + 2.0, -3.5 + 1e-15, 0.3])
    cases = []
    for a, b in zip(t_min, t_max):
        inside = [np.nextafter(a, np.inf), np.nextafter(b, -np.inf), 0.5 * (a + b)]
        edge = [a, b, np.nextafter(a, -np.inf), np.nextafter(b, np.inf)]
        for tc in inside + edge:
            for zeta in (5e-324, 1e-300, 1e-16, 1.0, 1e16, 1e300):
                for lam2 in (0.0, np.nextafter(Q * Q, 0.0), 0.5 * Q * Q, Q * Q):
                    cases.append((lam2, tc, zeta, a, b))
    c = np.array(cases, dtype=np.float64)
    with np.errstate(over="ignore"):
        _check(c[:, 0], c[:, 1], c[:, 2], c[:, 3], c[:, 4])
