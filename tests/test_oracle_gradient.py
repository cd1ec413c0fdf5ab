"""Pins of oracle.gradient (gradient fields, Sec. 6) by plain calculus: difference quotients of
the field, the closest-point construction of the ray constants, and the decomposition of the
gradient into the value field's derivative and four fields of the transverse kernel."""
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


def test_ray_constants_from_closest_points():
    # h (y_perp . e) is (o + t_chi v - chi) . e with t_chi = (chi - o) . v
    rng = np.random.default_rng(2)
    for _ in range(50):
        o = rng.uniform(-2, 2, 3)
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        e = rng.standard_normal(3)
        e /= np.linalg.norm(e)
        chi = rng.uniform(-1, 1, 3)
        alpha, beta = G.ray_constants(o, v, e)
        t_chi = (chi - o) @ v
        perp = o + t_chi * v - chi
        assert abs(perp @ v) < 1e-12
        assert abs(alpha + beta @ chi - perp @ e) < 1e-12


@pytest.mark.parametrize("kind", KINDS)
def test_decomposition_with_exact_fields(kind):
    """e.grad f = (v.e) F' - alpha G_0 - beta.(G_x, G_y, G_z), every field taken exactly (F' by a
    difference quotient along the ray, the G's as fields of -w'/r with float64 values)."""
    xyz, h, val = _scene(11)
    gvals = G.transverse_values(xyz, h, val, dtype=np.float64)
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
            Gs = [G.field_value(x, xyz, h, gv, gk) for gv in gvals]
            grad = G.gradient(x, xyz, h, val, kind)
            scale = max(np.max(np.abs(grad)), 1e-300)
            for e in list(np.eye(3)) + [rng.standard_normal(3)]:
                e = e / np.linalg.norm(e)
                got = G.assemble(vv, e, ov, dF, Gs[0], Gs[1:])
                assert abs(got - grad @ e) <= 1e-6 * scale, (r, t, got, grad @ e)


def test_approximated_gradient_on_rays():
    """The same decomposition with the method's approximated fields (exact integer pieces of the
    value field, K = 4, D = 3, and of the four transverse fields): within the method's error.  The
    along-ray part is the derivative of an L2-optimal value approximation (a few per cent of the
    largest gradient on these rays), the transverse part an approximation of its own (about 1 %)."""
    from tests import gpu_helpers as H

    xyz, h, val = synth.random_scene(41, 200, h_lo=0.05, h_hi=0.12)
    o, v = synth.random_rays(5, 2)
    scF = H.Scene("wendland", 4, 3, 4096, xyz, h, val, 0.0)
    scG = [H.Scene("wendland_grad", 4, 3, 1024, xyz, h, gv, 0.0) for gv in G.transverse_values(xyz, h, val)]
    for r in range(2):
        fF = scF.oracle_ray(o[r], v[r], 0.0, 3.0)
        fG = [s.oracle_ray(o[r], v[r], 0.0, 3.0) for s in scG]
        assert fF["pieces"]
        lo, hi = fF["pieces"][0][0] * scF.tau, fF["pieces"][-1][1] * scF.tau
        ts = np.random.default_rng(r).uniform(lo, hi, 100)
        dF = H.eval_exact_pieces(fF["pieces"], scF.tau, scF.sigma, ts, deriv=True)
        Gs = [H.eval_exact_pieces(f["pieces"], s.tau, s.sigma, ts) for f, s in zip(fG, scG)]
        ov, vv = o[r].astype(np.float64), v[r].astype(np.float64)
        grads = np.array([G.gradient(ov + t * vv, xyz, h, val, "wendland") for t in ts])
        for e in np.eye(3):
            got = G.assemble(vv, e, ov, dF, Gs[0], Gs[1:])
            ref = grads @ e
            assert np.max(np.abs(got - ref)) <= 0.08 * np.max(np.abs(ref)), (r, e)
