"""Gradient fields along rays (Sec. 6: the method carries over to any feature that the particles
generate additively, gradients among them).  Test infrastructure: a plain, slow reference.

Definitions (plain calculus; how the gradient is split into fields the method can encode is this
implementation's reading of that remark):
  field       f(x) = sum_j c_j h_j^-3 w(r_j),  y_j = (x - chi_j) / h_j,  r_j = |y_j|
  gradient    grad f(x) = sum_j c_j h_j^-4 w'(r_j) y_j / r_j = -sum_j c_j h_j^-4 g(r_j) y_j
              with g = -w'/r (the kinds "<kernel>_grad" of oracle.kernels).
On a ray x = o + t v (|v| = 1), y_j = y_perp_j + s_j v with s_j = (t - t_chi_j) / h_j,
t_chi_j = (chi_j - o).v, and y_perp_j = (o + t_chi_j v - chi_j) / h_j constant along the ray, so
for a unit axis e
  e.grad f(o + t v) = (v.e) F'(t) - sum_a e_a T_a(t),
F the value field on the ray and T_a (a = x, y, z) the field of the transverse kernel g in which
particle j contributes with amplitude (c_j / h_j) m_ja, where m_ja = y_perp_j . e_a is a per-pair
factor (|m| <= Lambda < q).  Each T_a is approximated, quantized and accumulated exactly like the
value field, with the pair's amplitude in place of the particle's value.  The per-pair factor keeps
every term of the order of the gradient itself: writing the transverse part with fixed particle
values (c/h^2 and c chi/h^2 against ray constants) instead would make the terms |chi| / h times
larger than their sum, and every field's error would be magnified by that factor.

Pinned by tests/test_oracle_gradient.py: the gradient against difference quotients of the field,
the pair factor against the closest-point construction, and the decomposition (with exact column
functions) against the gradient.
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


def pair_factor(o, v, chi, zeta, axis):
    """m = ((o + t_chi v - chi) . e_axis) / zeta for a ray o, v (float64) and particles chi, zeta,
    in the operation order both implementations use: dx = chi - o, t_chi = dx.x v.x + dx.y v.y +
    dx.z v.z (left to right), m = (t_chi v_axis - dx_axis) / zeta.  Broadcasts over particles."""
    o = np.asarray(o, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    chi = np.asarray(chi, dtype=np.float64)
    zeta = np.asarray(zeta, dtype=np.float64)
    dx = [chi[..., k] - o[k] for k in range(3)]
    tchi = dx[0] * v[0] + dx[1] * v[1] + dx[2] * v[2]
    return (tchi * v[axis] - dx[axis]) / zeta


def transverse_values(xyz, h, val, dtype=np.float32):
    """Particle values c/h of the transverse fields T_x, T_y, T_z (their pairs carry the factor
    m_ja on top), rounded to `dtype` (float32: the precision in which particle values are given)."""
    return (np.asarray(val, dtype=np.float64) / np.asarray(h, dtype=np.float64)).astype(dtype)


def transverse_field(x, o, v, xyz, h, tvals, kind_grad, axis):
    """T_axis at the point x of the ray o + t v, exactly: sum_j tv_j m_j,axis h_j^-3 g(r_j)."""
    x = np.asarray(x, dtype=np.float64)
    chi = np.asarray(xyz, dtype=np.float64)
    hh = np.asarray(h, dtype=np.float64)
    tv = np.asarray(tvals, dtype=np.float64)
    r = np.linalg.norm(x[None, :] - chi, axis=1) / hh
    m = pair_factor(o, v, chi, hh, axis)
    return float(np.sum(tv * m * kernels.w(kind_grad, r) / hh ** 3))


def assemble(v, e, dF, T):
    """e.grad f on the ray from the value field's t-derivative and the three transverse fields
    (scalars or arrays over sample points; T a sequence of three)."""
    v = np.asarray(v, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    return float(v @ e) * np.asarray(dF) - sum(e[a] * np.asarray(T[a]) for a in range(3))
