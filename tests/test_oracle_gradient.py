"""Pins of oracle.gradient (gradient fields, Sec. 6) by plain calculus: difference quotients of
the field, the closest-point construction of the pair factor, and the decomposition of the
gradient into the value field's derivative and three transverse fields."""
import numpy as np
import pytest

import synth
from oracle import gradient as G
from oracle import kernels

KINDS = sorted(kernels.GRAD_OF)


def _scene(seed=7, n=60):
    return synth.random_scene(seed, n, lo=0.3, hi=0.7, h_lo=0.05, h_hi=0.15, signed=True)


@pytest.mark.parametrize("kind", KINDS)
def test_gradient_against_difference_quotients(kind):
    xyz, h, val = _scene()
    rng = np.random.default_rng(1)
    e = 1e-6
    for _ in range(6):
        x = rng.uniform(0.35, 0.65, 3)
        num = np.array([(G.field_value(x + e * ax, xyz, h, val, kind) - G.field_value(x - e * ax, xyz, h, val, kind))
                        / (2 * e) for ax in np.eye(3)])
        got = G.gradient(x, xyz, h, val, kind)
        assert np.max(np.abs(got - num)) <= 1e-6 * np.max(np.abs(num)), (x, got, num)


def test_pair_factor_from_closest_points():
    # m h is the offset of the ray's point closest to chi from chi, along the axis: perpendicular to
    # the ray, of length Lambda h, found here by minimising the distance along the ray numerically
    rng = np.random.default_rng(2)
    for _ in range(50):
        o = rng.uniform(-2, 2, 3)
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        chi = rng.uniform(-1, 1, 3)
        h = rng.uniform(0.01, 0.2)
        ts = np.linspace(-6.0, 6.0, 240001)
        d2 = np.sum((o[None, :] + ts[:, None] * v[None, :] - chi[None, :]) ** 2, axis=1)
        t_best = ts[int(np.argmin(d2))]
        closest = o + t_best * v
        m = np.array([G.pair_factor(o, v, chi, h, a) for a in range(3)])
        assert np.max(np.abs(m * h - (closest - chi))) < 1e-4
        assert abs((m * h) @ v) < 1e-12
        lam = np.linalg.norm(np.cross(chi - o, v)) / h
        assert abs(np.linalg.norm(m) - lam) < 1e-9 * max(1.0, lam)


@pytest.mark.parametrize("kind", KINDS)
def test_decomposition_with_exact_fields(kind):
    """e.grad f = (v.e) F' - sum_a e_a T_a, every field taken exactly (F' by a difference quotient
    along the ray, the T's as fields of -w'/r with values c/h and the pair factors)."""
    xyz, h, val = _scene(11)
    tv = G.transverse_values(xyz, h, val, dtype=np.float64)
    gk = kernels.GRAD_OF[kind]
    rng = np.random.default_rng(4)
    o, v = synth.random_rays(9, 4, box=(0.3, 0.7))
    for r in range(4):
        ov, vv = o[r].astype(np.float64), v[r].astype(np.float64)
        vv /= np.linalg.norm(vv)
        for t in rng.uniform(0.8, 1.6, 5):
            x = ov + t * vv
            eps = 1e-6
            dF = (G.field_value(x + eps * vv, xyz, h, val, kind) - G.field_value(x - eps * vv, xyz, h, val, kind)) / (2 * eps)
            T = [G.transverse_field(x, ov, vv, xyz, h, tv, gk, a) for a in range(3)]
            grad = G.gradient(x, xyz, h, val, kind)
            scale = max(np.max(np.abs(grad)), 1e-300)
            for e in list(np.eye(3)) + [rng.standard_normal(3)]:
                e = e / np.linalg.norm(e)
                got = G.assemble(vv, e, dF, T)
                assert abs(got - grad @ e) <= 1e-6 * scale, (r, t, got, grad @ e)


def test_approximated_gradient_on_rays():
    """The same decomposition with the method's approximated fields (exact integer pieces of the
    value field, K = 4, D = 3, and of the three transverse fields): within the method's error.  The
    along-ray part is the derivative of an L2-optimal value approximation (a few per cent of the
    largest gradient on these rays), the transverse part an approximation of its own (about 1 %)."""
    from tests import gpu_helpers as H

    xyz, h, val = synth.random_scene(41, 200, h_lo=0.05, h_hi=0.12)
    o, v = synth.random_rays(5, 2)
    tv = G.transverse_values(xyz, h, val)
    scF = H.Scene("wendland", 4, 3, 4096, xyz, h, val, 0.0)
    scT = [H.Scene("wendland_grad", 4, 3, 1024, xyz, h, tv, 0.0, transverse=a) for a in range(3)]
    for r in range(2):
        fF = scF.oracle_ray(o[r], v[r], 0.0, 3.0)
        fT = [s.oracle_ray(o[r], v[r], 0.0, 3.0) for s in scT]
        assert fF["pieces"]
        lo, hi = fF["pieces"][0][0] * scF.tau, fF["pieces"][-1][1] * scF.tau
        ts = np.random.default_rng(r).uniform(lo, hi, 100)
        dF = H.eval_exact_pieces(fF["pieces"], scF.tau, scF.sigma, ts, deriv=True)
        T = [H.eval_exact_pieces(f["pieces"], s.tau, s.sigma, ts) for f, s in zip(fT, scT)]
        ov, vv = o[r].astype(np.float64), v[r].astype(np.float64)
        grads = np.array([G.gradient(ov + t * vv, xyz, h, val, "wendland") for t in ts])
        for e in np.eye(3):
            got = G.assemble(vv, e, dF, T)
            ref = grads @ e
            assert np.max(np.abs(got - ref)) <= 0.08 * np.max(np.abs(ref)), (r, e)
