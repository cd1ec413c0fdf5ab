"""Gradient fields along rays (Sec. 6: the method carries over to any feature that the particles
generate additively, gradients among them).  Test infrastructure: a plain, slow reference.

Definitions (plain calculus; how the gradient is split into fields the method can encode is this
implementation's reading of that remark):
  field       f(x) = sum_j c_j h_j^-3 w(r_j),  y_j = (x - chi_j) / h_j,  r_j = |y_j|
  gradient    grad f(x) = sum_j c_j h_j^-4 w'(r_j) y_j / r_j = -sum_j c_j h_j^-4 g(r_j) y_j
              with g = -w'/r (the kinds "<kernel>_grad" of oracle.kernels).
On a ray x = o + t v (|v| = 1), y_j = y_perp_j + s_j v with s_j = (t - t_chi_j) / h_j and
t_chi_j = (chi_j - o).v, so for a unit axis e
  e.grad f = (v.e) dF/dt - sum_j c_j h_j^-5 g(r_j) h_j (y_perp_j.e),
F the field on the ray, and h_j (y_perp_j.e) = (o + t_chi_j v - chi_j).e = alpha + beta.chi_j with
the ray constants alpha = o.e - (o.v)(v.e) and beta = (v.e) v - e.  Hence
  e.grad f(o + t v) = (v.e) F'(t) - alpha G_0(t) - beta.(G_x, G_y, G_z)(t),
where G_0 and G_a are ordinary fields of g with particle values c/h^2 and c chi_a/h^2: four fields
of the transverse kernel serve every axis, and each is approximated, quantized and accumulated
exactly like the value field.

Pinned by tests/test_oracle_gradient.py: the gradient against difference quotients of the field,
alpha + beta.chi against the closest-point construction, and the decomposition (with the exact
column functions) against the gradient.
"""
from __future__ import annotations

import numpy as np

from . import kernels


def field_value(x, xyz, h, val, kind):
    """f(x) = sum_j c_j h_j^-3 w(|x - chi_j| / h_j) at one point (float64)."""
    x = np.asarray(x, dtype=np.float64)
    chi = np.asarray(xyz, dtype=np.float64)
    hh = np.asarray(h, dtype=np.float64)
    c = np.asarray(val, dtype=np.float64)
    r = np.linalg.norm(x[None, :] - chi, axis=1) / hh
    return float(np.sum(c * kernels.w(kind, r) / hh ** 3))


def gradient(x, xyz, h, val, kind):
    """grad f(x) = -sum_j c_j h_j^-4 g(r_j) y_j at one point (float64 3-vector)."""
    x = np.asarray(x, dtype=np.float64)
    chi = np.asarray(xyz, dtype=np.float64)
    hh = np.asarray(h, dtype=np.float64)
    c = np.asarray(val, dtype=np.float64)
    y = (x[None, :] - chi) / hh[:, None]
    r = np.linalg.norm(y, axis=1)
    g = kernels.w(kernels.GRAD_OF[kind], r)
    return -np.sum((c * g / hh ** 4)[:, None] * y, axis=0)


def ray_constants(o, v, e):
    """(alpha, beta) with h_j (y_perp_j.e) = alpha + beta.chi_j on the ray o + t v."""
    o = np.asarray(o, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    ve = float(v @ e)
    return float(o @ e - (o @ v) * ve), ve * v - e


def transverse_values(xyz, h, val, dtype=np.float32):
    """Particle values of the four transverse fields G_0, G_x, G_y, G_z: c/h^2 and c chi_a/h^2,
    rounded to `dtype` (float32: the precision in which particle values are given)."""
    chi = np.asarray(xyz, dtype=np.float64)
    hh = np.asarray(h, dtype=np.float64)
    c = np.asarray(val, dtype=np.float64)
    base = c / (hh * hh)
    return [base.astype(dtype)] + [(base * chi[:, a]).astype(dtype) for a in range(3)]


def assemble(v, e, o, dF, G0, Gxyz):
    """e.grad f on the ray from the value field's t-derivative and the four transverse fields
    (scalars or arrays over sample points; Gxyz a sequence of three)."""
    alpha, beta = ray_constants(o, v, e)
    ve = float(np.asarray(v, dtype=np.float64) @ np.asarray(e, dtype=np.float64))
    return ve * np.asarray(dF) - alpha * np.asarray(G0) - sum(beta[a] * np.asarray(Gxyz[a]) for a in range(3))
