"""Shared setup of the GPU parity tests: one scene, its oracle quanta and table,
the library index built with the same table and quanta, and oracle runs per ray.

The knot table (optimal knots, Sec. 3.4) is the one written by
tests/golden/make_knot_tables.py from the oracle; the quanta are the oracle's.
Both are passed to the library so that every discrete key (hit test, table
index, quantized positions) must agree bit for bit; the projection
coefficients are recomputed independently on each side.
"""
from __future__ import annotations

import functools

import numpy as np

import synth
from oracle import field, geometry, grid, lut, quanta, render
from tests.golden.make_knot_tables import load as load_knots

KIND_ID = {"cubic": 0, "wendland": 1, "wendland_c4": 2, "wendland_c6": 3, "wendland_grad": 4,
           "wendland_c4_grad": 5, "wendland_c6_grad": 6}


class Scene:
    def __init__(self, kind, K, D, n_lut, xyz, h, val, tol, tau_scale=1.0, lut_precision="fp64"):
        self.kind, self.K, self.D, self.n_lut, self.tol = kind, K, D, n_lut, tol
        self.xyz, self.h, self.val = xyz, h, val
        self.lut_precision = lut_precision
        self.theta = load_knots(kind, K, D, n_lut)
        # the table as stored (precision study): knots and projection rows rounded once
        self.theta_stored = lut.round_storage(self.theta, lut_precision)
        self._shat = None
        self.a_max = grid.a_max(kind, xyz, h, val)
        self.h_repr, self.phi_repr = grid.representatives(h, val)
        self.tau, self.sigma = quanta.choose_quanta(kind, D, self.a_max, self.h_repr, self.phi_repr)
        self.tau *= tau_scale
        self._index = None

    @property
    def shat(self):
        if self._shat is None:
            self._shat = LazyRows(self)
        return self._shat

    def table(self):
        return {"theta": self.theta_stored, "shat": self.shat}

    def index(self):
        import paper_2401_02896_amd as L

        if self._index is None:
            self._index = L.sph_hoa_build_index(self.xyz, self.h, self.val, kernel=KIND_ID[self.kind], degree=self.D,
                                                pieces=self.K, lut_entries=self.n_lut, merge_tol=self.tol,
                                                a_max=self.a_max, h_repr=self.h_repr, phi_repr=self.phi_repr,
                                                tau=self.tau, knot_table=self.theta,
                                                lut_precision=self.lut_precision)
        return self._index

    def oracle_ray(self, o, v, t_min, t_max, tol=None):
        return field.ray_field(np.asarray(o, np.float64), np.asarray(v, np.float64), t_min, t_max, self.xyz, self.h,
                               self.val, self.table(), (self.tau, self.sigma), self.K, self.D, self.kind,
                               self.tol if tol is None else tol)


class LazyRows:
    """Oracle jump coefficients of table rows, computed when first used."""

    def __init__(self, sc):
        self.sc = sc
        self.rows = {}
        self.lams = lut.lambda_midpoints(sc.kind, sc.n_lut)

    def __getitem__(self, i):
        i = int(i)
        if i not in self.rows:
            rows, _ = lut.difference_coefficients(self.sc.kind, float(self.lams[i]), self.sc.theta[i],
                                                  self.sc.K, self.sc.D)
            self.rows[i] = lut.round_storage(rows, self.sc.lut_precision)
        return self.rows[i]




@functools.lru_cache(maxsize=None)
def tiny_scene(tol=1e-3):
    xyz, h, val = synth.tiny_particles()
    return Scene("cubic", 4, 2, 4096, xyz, h, val, tol)


def field_of_ray(out, r, D):
    """(t_start, t_end, coef) arrays of ray r from an approx_rays result (host numpy)."""
    offs = out["ray_offsets"].cpu().numpy()
    a, b = offs[r], offs[r + 1]
    return (out["t_start"][a:b].cpu().numpy(), out["t_end"][a:b].cpu().numpy(),
            out["coef"][a:b].cpu().numpy().astype(np.float64))


def eval_pieces(t0, t1, coef, ts):
    """Evaluate a piecewise polynomial in the u-power form at points ts (0 outside)."""
    out = np.zeros_like(ts)
    for a, b, c in zip(t0, t1, coef):
        m = (ts >= a) & (ts < b)
        u = (ts[m] - a) / (b - a)
        out[m] = np.polyval(c[::-1], u)
    return out


def eval_exact_pieces(pieces, tau, sigma, ts, deriv=False):
    """Value (or t-derivative) at world positions ts of exact integer pieces
    [(t_start, t_end, coefficients, _)] in length quanta (0 outside the pieces), float64."""
    out = np.zeros_like(ts)
    for a, b, c, *_ in pieces:
        m = (ts >= a * tau) & (ts < b * tau)
        x = ts[m] / tau - a
        cf = [float(q) for q in c]
        if deriv:
            out[m] = sigma / tau * sum(d * cf[d] * x ** (d - 1) for d in range(1, len(cf)))
        else:
            out[m] = sigma * sum(cf[d] * x ** d for d in range(len(cf)))
    return out


def oracle_pixel(sc, f, t_min, t_max, tf, vmin, vmax, step):
    outn = [field.node_output(n, f["merger"]) for n in f["nodes"]]
    return render.composite(outn, t_min, t_max, tf, vmin, vmax, step)
