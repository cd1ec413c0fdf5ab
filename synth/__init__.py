"""Seeded synthetic SPH-like scenes, rays, cameras and transfer functions.

Shared by the tests, the benchmark and the oracle checks.  This module holds
none of the method's arithmetic: it only draws inputs.  The paper's own data
set (an unnamed SPH simulation rendered in its Fig. 2) is not available, so
these generators stand in for it with the shapes below.

tiny   : 4,096 particles uniform in the unit cube, h ~ U[0.02, 0.05],
         amplitude ~ lognormal(0, 1); 64 x 64 orthographic rays along +z from
         z = -0.2 through pixel centres of the unit square, t in [0, 1.4].
plain  : N particles (default 1,000,000): 90 % from 16 isotropic Gaussian
         clusters (centres U[0.2, 0.8]^3, sigma U[0.02, 0.1], equal weights,
         samples outside the unit cube redrawn), 10 % uniform; support radius
         q h = distance to the 32nd nearest neighbour (h = r32 / 2); amplitude
         m alpha / rho with alpha = rho (the field is the SPH density) and equal
         masses m = 1 / N, i.e. amplitude 1 / N; 512 x 512 perspective camera at
         (0.5, 0.5, -1.5) looking at the cube centre, fov_y 30 deg, t in [1, 3].
"""
from __future__ import annotations

import numpy as np


def tiny_particles(seed: int = 1, n: int = 4096):
    rng = np.random.default_rng(seed)
    xyz = rng.random((n, 3)).astype(np.float32)
    h = rng.uniform(0.02, 0.05, n).astype(np.float32)
    val = rng.lognormal(0.0, 1.0, n).astype(np.float32)
    return xyz, h, val


def ortho_rays(width: int = 64, height: int = 64, z0: float = -0.2):
    """Rays with origin ((i + 1/2) / W, (j + 1/2) / H, z0), direction +z; index j * W + i."""
    j, i = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    o = np.zeros((height * width, 3), dtype=np.float32)
    o[:, 0] = ((i.reshape(-1) + 0.5) / width).astype(np.float32)
    o[:, 1] = ((j.reshape(-1) + 0.5) / height).astype(np.float32)
    o[:, 2] = np.float32(z0)
    d = np.zeros_like(o)
    d[:, 2] = 1.0
    return o, d


def clustered_particles(seed: int = 2, n: int = 1_000_000, clusters: int = 16, background: float = 0.1,
                        k_neigh: int = 32):
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    n_bg = int(round(background * n))
    n_cl = n - n_bg
    centres = rng.uniform(0.2, 0.8, (clusters, 3))
    sig = rng.uniform(0.02, 0.1, clusters)
    which = rng.integers(0, clusters, n_cl)
    pts = centres[which] + rng.standard_normal((n_cl, 3)) * sig[which, None]
    while True:
        bad = np.any((pts < 0.0) | (pts > 1.0), axis=1)
        nb = int(bad.sum())
        if nb == 0:
            break
        pts[bad] = centres[which[bad]] + rng.standard_normal((nb, 3)) * sig[which[bad], None]
    bg = rng.random((n_bg, 3))
    xyz = np.concatenate([pts, bg]).astype(np.float32)
    perm = rng.permutation(n)
    xyz = xyz[perm]
    pts64 = xyz.astype(np.float64)
    tree = cKDTree(pts64)
    h = np.empty(n, dtype=np.float32)
    chunk = 1 << 20  # bounded memory for large sets (the query's k + 1 distances and indices per point)
    for a in range(0, n, chunk):
        dist, _ = tree.query(pts64[a:a + chunk], k=k_neigh + 1, workers=-1)
        h[a:a + chunk] = (0.5 * dist[:, k_neigh]).astype(np.float32)
    val = np.full(n, 1.0 / n, dtype=np.float32)
    return xyz, h, val


def cluster_centres(seed: int = 2, clusters: int = 16):
    """The Gaussian centres clustered_particles(seed, ..., clusters) draws first."""
    return np.random.default_rng(seed).uniform(0.2, 0.8, (clusters, 3))


def batch_cameras(seed: int = 4, n: int = 256, centres=None, core_fraction: float = 0.5):
    """Ray bundles of the batching workload: square images of side 2^k, k uniform in 5..9
    (32..512, log-uniform), eyes uniform on the sphere of radius 2 about the cube centre, t in
    [1, 3].  A fraction of the bundles look at a cluster centre with a narrow field of view, so
    their rays run through the dense cores (the heavy tail of hits per ray); the others see the
    whole cube."""
    rng = np.random.default_rng(seed)
    cams = []
    for _ in range(n):
        side = int(2 ** int(rng.integers(5, 10)))
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        eye = 0.5 + 2.0 * d
        core = centres is not None and rng.random() < core_fraction
        target = centres[int(rng.integers(len(centres)))] if core else np.array([0.5, 0.5, 0.5])
        fwd = target - eye
        fwd /= np.linalg.norm(fwd)
        up = [0.0, 1.0, 0.0] if abs(fwd[1]) < 0.9 else [1.0, 0.0, 0.0]
        cams.append({"eye": [float(x) for x in eye], "look_at": [float(x) for x in target], "up": up,
                     "fov_y_deg": 6.0 if core else 30.0, "ortho": 0, "ortho_half_extent": 0.0,
                     "width": side, "height": side, "t_min": 1.0, "t_max": 3.0})
    return cams


def plain_camera(width: int = 512, height: int = 512):
    return {"eye": [0.5, 0.5, -1.5], "look_at": [0.5, 0.5, 0.5], "up": [0.0, 1.0, 0.0], "fov_y_deg": 30.0,
            "ortho": 0, "ortho_half_extent": 0.0, "width": width, "height": height, "t_min": 1.0, "t_max": 3.0}


def tiny_camera(width: int = 64, height: int = 64):
    return {"eye": [0.5, 0.5, -0.2], "look_at": [0.5, 0.5, 1.0], "up": [0.0, 1.0, 0.0], "fov_y_deg": 0.0,
            "ortho": 1, "ortho_half_extent": 0.5, "width": width, "height": height, "t_min": 0.0, "t_max": 1.4}


def transfer_function(n: int = 256, seed: int = 3, opacity: float = 1.0):
    """Smooth RGBA control points: emission r, g, b in [0, 1] and extinction a >= 0."""
    rng = np.random.default_rng(seed)
    x = np.linspace(0.0, 1.0, n)
    ph = rng.uniform(0, 2 * np.pi, 3)
    rgb = 0.5 + 0.5 * np.sin(2 * np.pi * x[:, None] * np.array([1.0, 1.7, 2.3]) + ph[None, :])
    a = opacity * x ** 1.5
    return np.concatenate([rgb, a[:, None]], axis=1).astype(np.float32)


def random_scene(seed: int, n: int, lo=0.0, hi=1.0, h_lo=0.02, h_hi=0.08, signed=False):
    """Small uniform scene for edge-case tests."""
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(lo, hi, (n, 3)).astype(np.float32)
    h = rng.uniform(h_lo, h_hi, n).astype(np.float32)
    val = rng.lognormal(0.0, 1.0, n).astype(np.float32)
    if signed:
        val *= rng.choice(np.array([-1.0, 1.0], dtype=np.float32), n)
    return xyz, h, val


def random_rays(seed: int, n: int, box=(0.0, 1.0)):
    """Rays from points on a sphere around the box towards random points inside it."""
    rng = np.random.default_rng(seed)
    c = 0.5 * (box[0] + box[1])
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = c - 1.5 * d * (box[1] - box[0])
    tgt = rng.uniform(box[0], box[1], (n, 3))
    v = tgt - o
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return o.astype(np.float32), v.astype(np.float32)


def bit_tables(seed: int = 6, n_table: int = 37, degree: int = 3, bits: int = 64):
    """Knot table of the integer bit-length study: distances uint32 [n_table] and jump limbs
    uint32 [n_table, degree + 1, bits // 32] (low limb first), uniform over the full 32-bit range
    except entry 0, which is all ones (every carry propagates) with distance 2^32 - 1."""
    rng = np.random.default_rng(seed)
    L = bits // 32
    dist = rng.integers(0, 1 << 32, n_table, dtype=np.uint64).astype(np.uint32)
    jumps = rng.integers(0, 1 << 32, (n_table, degree + 1, L), dtype=np.uint64).astype(np.uint32)
    dist[0] = 0xFFFFFFFF
    jumps[0] = 0xFFFFFFFF
    return dist, jumps


def limbs_to_int(limbs) -> int:
    """Unsigned integer of little-endian uint32 limbs."""
    v = 0
    for i, x in enumerate(limbs):
        v |= int(x) << (32 * i)
    return v
