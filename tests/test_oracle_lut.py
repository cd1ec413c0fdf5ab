"""Pins of oracle.lut: the candidate space (Sec. 3.2/3.3, App. A.1/A.2), the knot
optimisation (Sec. 3.4) and Fig. 4's approximation errors."""
import math
from multiprocessing import Pool

import mpmath
import numpy as np
import pytest

from oracle import kernels, lut
from tests import fig4

F = fig4.load()


@pytest.mark.parametrize("K", range(1, 7))
@pytest.mark.parametrize("D", range(1, 7))
def test_dimension(K, D):
    # Sec. 3.3: the space has dimension floor(K D / 2)
    assert len(lut.index_set(K, D)) == (K * D) // 2


@pytest.mark.parametrize("K,D", [(3, 4), (4, 3), (6, 4), (5, 3)])
def test_basis_shape(K, D):
    theta = np.concatenate([[0.0], np.cumsum(np.linspace(0.3, 0.5, lut.n_pos_knots(K)))])
    t = np.linspace(-3, 3, 2001)
    mats = []
    for (k, d) in lut.index_set(K, D):
        f = lut.basis_value(theta, k, d, t)
        assert np.allclose(f, f[::-1])                       # even
        assert np.all(f[np.abs(t) >= theta[-1]] == 0.0)      # compact support
        for th in theta[1:]:                                 # continuous at the knots
            assert abs(lut.basis_value(theta, k, d, np.array([th - 1e-12]))[0]
                       - lut.basis_value(theta, k, d, np.array([th + 1e-12]))[0]) < 1e-9
        if K % 2 == 1:                                       # no change at 0 for odd K
            h = 1e-6
            g = lut.basis_value(theta, k, d, np.array([-h, 0.0, h]))
            assert abs(g[0] - 2 * g[1] + g[2]) / h < 1e-3 or d % 2 == 0
        mats.append(f)
    # linear independence (App. A.1)
    assert np.linalg.matrix_rank(np.array(mats), tol=1e-9) == len(mats)


def _mp_inner(fa, fb, pts):
    return 2 * mpmath.quad(lambda x: fa(x) * fb(x), pts)


@pytest.mark.parametrize("kind,lam,K,D", [("cubic", 0.37, 4, 3), ("wendland", 1.3, 3, 2), ("cubic", 1.9, 4, 2)])
def test_projection_is_orthogonal(kind, lam, K, D):
    """App. A.2: the residual B - S is orthogonal to every basis function (independent quadrature)."""
    mpmath.mp.dps = 25
    s = math.sqrt(4 - lam * lam)
    theta_pos = s * np.array([0.5, 0.95][: lut.n_pos_knots(K)])
    r = lut.project(kind, lam, theta_pos, K, D)
    theta = r["theta"]

    def B(x):
        return mpmath.mpf(float(kernels.w(kind, np.array([math.sqrt(lam * lam + float(x) ** 2)]))[0]))

    def S(x):
        return sum(ci * float(lut.basis_value(theta, k, d, np.array([float(x)]))[0]) for ci, (k, d) in zip(r["c"], r["J"]))

    pts = sorted({0.0, s, *[float(v) for v in theta[1:]]} | ({math.sqrt(1 - lam * lam)} if kind == "cubic" and lam < 1 else set()))
    pts = [p for p in pts if p <= max(s, theta[-1])]
    nb = math.sqrt(float(_mp_inner(B, B, pts)))
    for (k, d) in r["J"]:
        def A(x, k=k, d=d):
            return float(lut.basis_value(theta, k, d, np.array([float(x)]))[0])
        ip = _mp_inner(lambda x: B(x) - S(x), A, pts)
        na = math.sqrt(float(_mp_inner(A, A, pts)))
        assert abs(float(ip)) < 1e-10 * nb * na
    e2 = float(_mp_inner(lambda x: B(x) - S(x), lambda x: B(x) - S(x), pts))
    assert abs(e2 - r["E2"]) < 1e-9 * e2 + 1e-30


@pytest.mark.parametrize("kind,lam,K,D", [("cubic", 0.5, 4, 3), ("cubic", 1.5, 4, 2), ("wendland", 0.9, 4, 3),
                                          ("cubic", 1.2, 3, 3)])
def test_knots_are_local_optimum(kind, lam, K, D):
    th, e2 = lut.optimal_knots(kind, lam, K, D)
    for j in range(len(th)):
        for f in (1 - 1e-3, 1 + 1e-3):
            t2 = th.copy()
            t2[j] *= f
            assert lut.project(kind, lam, t2, K, D)["E2"] >= e2
    for j in range(len(th)):
        for f in (1 - 1e-6, 1 + 1e-6):
            t2 = th.copy()
            t2[j] *= f
            assert lut.project(kind, lam, t2, K, D)["E2"] >= e2 * (1 - 1e-12)


@pytest.mark.parametrize("K", range(1, 7))
@pytest.mark.parametrize("D", [1, 2, 3])
def test_difference_coefficients_reencode_projection(K, D):
    """Sec. 2 knot encoding: summing localized jumps from the left reproduces S."""
    if (K * D) // 2 == 0:
        pytest.skip("K = D = 1 leaves only the zero function (dimension floor(K D / 2) = 0)")
    kind, lam = "cubic", 0.8
    s = math.sqrt(4 - lam * lam)
    P = lut.n_pos_knots(K)
    theta_pos = s * np.linspace(0.35, 0.97, P)
    r = lut.project(kind, lam, theta_pos, K, D)
    sh, sm = lut.difference_coefficients(kind, lam, theta_pos, K, D)
    knots = []
    for k in range(P, 0, -1):
        knots.append((-theta_pos[k - 1], [(-1) ** (d + 1) * sh[k - 1][d] for d in range(D + 1)]))
    if K % 2 == 0:
        knots.append((0.0, list(sm)))
    for k in range(1, P + 1):
        knots.append((theta_pos[k - 1], list(sh[k - 1])))
    if K % 2 == 1:
        # the odd-order jumps at +-theta_1 come from the left/right of the even central piece
        pass
    rng = np.random.default_rng(K * 10 + D)
    for x in rng.uniform(-s, s, 50):
        v = sum(sum(c[d] * (x - kp) ** d for d in range(D + 1)) for kp, c in knots if kp <= x)
        ref = sum(ci * float(lut.basis_value(r["theta"], k, d, np.array([x]))[0]) for ci, (k, d) in zip(r["c"], r["J"]))
        assert abs(v - ref) < 1e-10


def test_line_integral_of_projection():
    """The approximation's line integral is within Cauchy-Schwarz of the closed-form column integral."""
    for kind, K, D in [("cubic", 4, 2), ("wendland", 4, 3)]:
        for lam in (0.05, 0.6, 1.1, 1.8):
            th, e2 = lut.optimal_knots(kind, lam, K, D)
            polys, _ = lut.piece_polynomials(kind, lam, th, K, D)
            theta = np.concatenate([[0.0], th])
            integ = 0.0
            for m, p in enumerate(polys, start=1):
                ip = p.integ()
                integ += 2 * (ip(theta[m]) - ip(theta[m - 1]))
            sig = kernels.column_integral(kind, lam)
            bound = math.sqrt(e2) * math.sqrt(2 * max(th[-1], math.sqrt(4 - lam * lam)))
            assert abs(integ - sig) <= bound
            assert abs(integ - sig) <= 0.01 * sig


def _overall(args):
    K, D = args
    return K, D, lut.overall_error("cubic", K, D, 48)[0]


def test_fig4_approximation_errors():
    """Fig. 4 (left panel): E_{K,D} by a 48-point midpoint Riemann sum over Lambda.

    The midpoint rule converges as 1/n^2; at n = 48 its own error is below 4e-4
    relative for these entries (it is 1e-3 at n = 24 and 3e-4 at n = 50).
    """
    cases = [(4, 3), (4, 2), (3, 2), (2, 1), (1, 2), (2, 2)]
    with Pool(min(6, len(cases))) as p:
        res = p.map(_overall, cases)
    for K, D, E in res:
        assert abs(E / F["E"][(K, D)] - 1) < 4e-4, (K, D, E)


def test_storage_rounding_hand_cases():
    """bf16 keeps 8 significant bits: the spacing just above 1 is 2^-7.  1 + 2^-8 lies halfway
    between 1 and 1 + 2^-7 and goes to the even one (1); 1 + 3 2^-8 lies halfway between
    1 + 2^-7 (odd last bit) and 1 + 2^-6, and goes to 1 + 2^-6; just above a tie rounds up."""
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -20, -(1 + 3 * 2.0 ** -8),
                  0.0, 3.0, 255.5, 256.5, 2.0 ** -130])
    want = np.array([1.0, 1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7, -(1 + 2.0 ** -6), 0.0, 3.0, 256.0, 256.0,
                     2.0 ** -130])
    assert np.array_equal(lut.round_storage(x, "bf16"), want)
    # fp32: 1 + 2^-30 is not a float32 and rounds to 1; 1/3 rounds to the float32 nearest it
    assert lut.round_storage(np.array([1 + 2.0 ** -30]), "fp32")[0] == 1.0
    assert lut.round_storage(np.array([1.0 / 3.0]), "fp32")[0] == float(np.float32(1.0 / 3.0))
    assert np.array_equal(lut.round_storage(x, "fp64"), x)


def test_storage_rounding_matches_torch_bfloat16():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.normal(0, 1, 20000) * 10.0 ** rng.uniform(-12, 12, 20000),
                        rng.uniform(-1, 1, 20000)])
    f32 = torch.from_numpy(x.astype(np.float32))
    ref = f32.to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(lut.round_storage(x, "bf16"), ref)


def test_storage_rounding_fp16_hand_cases_and_numpy():
    """binary16 keeps 11 significant bits: 1 + 2^-11 is a tie between 1 and 1 + 2^-10 (even: 1);
    below 2^-14 the spacing is 2^-24 (2^-25 is a tie between 0 and 2^-24: 0); 65504 is the
    largest finite value, 65520 (a tie with the next binade's 65536) overflows."""
    x = np.array([1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11, 2.0 ** -25, 3e-8, 65504.0, 65520.0, -65520.0])
    want = np.array([1.0, 1 + 2.0 ** -9, 0.0, 2.0 ** -24, 65504.0, np.inf, -np.inf])
    assert np.array_equal(lut.round_storage(x, "fp16"), want)
    rng = np.random.default_rng(9)
    y = np.concatenate([rng.normal(0, 1, 20000) * 10.0 ** rng.uniform(-10, 4.5, 20000), rng.uniform(-1, 1, 2000)])
    with np.errstate(over="ignore"):
        ref = y.astype(np.float32).astype(np.float16).astype(np.float64)
    assert np.array_equal(lut.round_storage(y, "fp16"), ref)
