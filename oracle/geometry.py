"""Ray / particle geometry (Sec. 3.1, Fig. 1) and viewing-ray generation.

A ray is x(t) = b + t v with unit v.  For a particle at chi with smoothing
length zeta, t_chi = (chi - b) . v is the parameter of the closest point and
Lambda = |chi - x(t_chi)| / zeta = |(chi - b) x v| / zeta the normalized
distance; the particle contributes along the ray as its amplitude times
zeta^-3 B_Lambda((t - t_chi) / zeta), and only if Lambda < q.

A (particle, ray) pair counts as a contribution when Lambda < q and the
support interval [t_chi - s zeta, t_chi + s zeta], s = sqrt(q^2 - Lambda^2),
overlaps the ray segment [t_min, t_max] (the paper does not bound rays; the
segment is this implementation's reading).

Every quantity that decides an integer later (the hit test, the table index,
the quantized knot positions) is computed here in float64 from float32 inputs
widened exactly, in the operation order written below and without fused
multiply-adds, so that any other IEEE implementation of the same sequence
obtains the same bits.
"""
from __future__ import annotations

import math

import numpy as np

f64 = np.float64


def widen(a):
    """float32 inputs widened exactly to float64."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def pair_terms(o, v, chi, zeta):
    """(Lambda^2, t_chi) for rays o, v (float64 [..., 3]) and particles chi, zeta.

    dx = chi - o; c = dx x v; Lambda^2 = (cx*cx + cy*cy + cz*cz) / (zeta*zeta);
    t_chi = dx.x*v.x + dx.y*v.y + dx.z*v.z; sums left to right.
    Broadcasts over leading dimensions.
    """
    dxx = chi[..., 0] - o[..., 0]
    dxy = chi[..., 1] - o[..., 1]
    dxz = chi[..., 2] - o[..., 2]
    cx = dxy * v[..., 2] - dxz * v[..., 1]
    cy = dxz * v[..., 0] - dxx * v[..., 2]
    cz = dxx * v[..., 1] - dxy * v[..., 0]
    lam2 = (cx * cx + cy * cy + cz * cz) / (zeta * zeta)
    tchi = dxx * v[..., 0] + dxy * v[..., 1] + dxz * v[..., 2]
    return lam2, tchi


def hit_mask(lam2, tchi, zeta, q, t_min, t_max):
    """Contribution test: Lambda^2 < q^2 and the support overlaps [t_min, t_max].

    s = sqrt(q*q - Lambda^2); sz = s * zeta; (t_chi + sz > t_min) and (t_chi - sz < t_max).
    """
    inside = lam2 < q * q
    s = np.sqrt(np.where(inside, q * q - lam2, 0.0))
    sz = s * zeta
    return inside & (tchi + sz > t_min) & (tchi - sz < t_max)


def ray_hits(o, v, t_min, t_max, xyz, zeta, q):
    """Indices (ascending) of all particles contributing to one ray, by brute force."""
    chi = widen(xyz)
    z = widen(zeta)
    lam2, tchi = pair_terms(np.asarray(o, f64)[None, :], np.asarray(v, f64)[None, :], chi, z)
    m = hit_mask(lam2, tchi, z, q, f64(t_min), f64(t_max))
    return np.nonzero(m)[0]


def normalize3(x, y, z):
    n = math.sqrt(x * x + y * y + z * z)
    return x / n, y / n, z / n


def camera_frame(eye, look_at, up):
    """Forward, right and up unit vectors of a camera, float64 from float32 inputs.

    f = normalize(look_at - eye); r = normalize(f x up); u = r x f.
    """
    e = widen(eye)
    la = widen(look_at)
    upv = widen(up)
    fx, fy, fz = normalize3(la[0] - e[0], la[1] - e[1], la[2] - e[2])
    rx = fy * upv[2] - fz * upv[1]
    ry = fz * upv[0] - fx * upv[2]
    rz = fx * upv[1] - fy * upv[0]
    rx, ry, rz = normalize3(rx, ry, rz)
    ux = ry * fz - rz * fy
    uy = rz * fx - rx * fz
    uz = rx * fy - ry * fx
    return (fx, fy, fz), (rx, ry, rz), (ux, uy, uz)


def camera_rays(cam, pixels=None):
    """Origins and unit directions (float64) of the camera's pixel-centre rays.

    cam keys: eye, look_at, up (3 floats each, taken as float32), fov_y_deg,
    ortho (0/1), ortho_half_extent, width, height.  Ray index = row * width + col,
    row 0 at the top.  Per pixel (col i, row j):
      a = (2 i + 1) / W - 1;  b = 1 - (2 j + 1) / H;  aspect = W / H
      perspective: g = tan(fov_y_deg * pi / 180 / 2) (evaluated once, in double);
                   d = f + (a * g * aspect) r + (b * g) u;  v = d / |d|;  origin = eye
      orthographic: h = ortho_half_extent;
                   origin = eye + (a * h * aspect) r + (b * h) u;  v = f
    (products left to right, sums in the order written).
    """
    W, H = int(cam["width"]), int(cam["height"])
    f, r, u = camera_frame(cam["eye"], cam["look_at"], cam["up"])
    eye = widen(cam["eye"])
    aspect = f64(W) / f64(H)
    if pixels is None:
        pixels = np.arange(W * H, dtype=np.int64)
    pixels = np.asarray(pixels, dtype=np.int64)
    col = (pixels % W).astype(np.float64)
    row = (pixels // W).astype(np.float64)
    a = (2.0 * col + 1.0) / f64(W) - 1.0
    b = 1.0 - (2.0 * row + 1.0) / f64(H)
    n = len(pixels)
    o = np.zeros((n, 3))
    v = np.zeros((n, 3))
    if int(cam.get("ortho", 0)):
        h = f64(np.float32(cam["ortho_half_extent"]))
        sa = a * h * aspect
        sb = b * h
        for k in range(3):
            o[:, k] = eye[k] + sa * r[k] + sb * u[k]
            v[:, k] = f[k]
    else:
        fov = f64(np.float32(cam["fov_y_deg"]))
        g = math.tan(fov * math.pi / 180.0 / 2.0)
        sa = a * g * aspect
        sb = b * g
        dx = f[0] + sa * r[0] + sb * u[0]
        dy = f[1] + sa * r[1] + sb * u[1]
        dz = f[2] + sa * r[2] + sb * u[2]
        nrm = np.sqrt(dx * dx + dy * dy + dz * dz)
        v[:, 0], v[:, 1], v[:, 2] = dx / nrm, dy / nrm, dz / nrm
        o[:, 0], o[:, 1], o[:, 2] = eye[0], eye[1], eye[2]
    return o, v
