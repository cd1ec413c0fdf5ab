"""Pins of oracle.floatpath: the float accumulation variant of Sec. 4.1 (reinitialization knots)."""
import math
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import floatpath as fp
from oracle import geometry, lut
from tests.golden.make_knot_tables import load as load_knots


class Table:
    """Table rows (theta, s-hat, s-mid) of one golden knot table, projected when first used."""

    def __init__(self, kind, K, D, n):
        self.kind, self.K, self.D, self.n = kind, K, D, n
        self.theta = load_knots(kind, K, D, n)
        self.lams = lut.lambda_midpoints(kind, n)
        self.rows = {}

    def row(self, i):
        if i not in self.rows:
            self.rows[i] = lut.difference_coefficients(self.kind, float(self.lams[i]), self.theta[i], self.K, self.D)
        return self.rows[i]

    def as_dict(self):
        t = self

        class Col:
            def __init__(self, j):
                self.j = j

            def __getitem__(self, i):
                return t.row(int(i))[self.j]

        return {"theta": self.theta, "shat": Col(0), "smid": Col(1)}


def _direct(knot_lists, x):
    """Sum of every knot's jump polynomial at x over knots at positions <= x (exact)."""
    v = Fraction(0)
    for kn in knot_lists:
        for t, _, c in kn:
            if t <= x:
                v += sum(cd * (x - t) ** d for d, cd in enumerate(c))
    return v


def _per_particle(o, v, t_min, t_max, xyz, h, val, tab, num):
    hits = geometry.ray_hits(o, v, t_min, t_max, xyz, h, 2.0)
    chi, z, va = geometry.widen(xyz), geometry.widen(h), geometry.widen(val)
    out = {}
    for pid in sorted(int(p) for p in hits):
        lam2, tchi = geometry.pair_terms(np.asarray(o, np.float64), np.asarray(v, np.float64), chi[pid], z[pid])
        li = lut.lut_index(tab.kind, math.sqrt(float(lam2)), tab.n)
        sh, sm = tab.row(li)
        out[pid] = fp.particle_knots(float(tchi), z[pid], va[pid], tab.theta[li], sh, sm, tab.K, tab.D, num)
    return out


@pytest.mark.parametrize("spec", [("wendland", 2, 2, 256), ("cubic", 3, 3, 256)])
@pytest.mark.parametrize("n_reinit", [0, 4])
def test_exact_sweep_equals_direct_sum(spec, n_reinit):
    """In exact arithmetic the sweep's piece at [a, b) equals, at any x in it, the direct sum of the
    jump polynomials of all knots <= a of the particles not finished by the last reinitialization
    knot T <= a (last knot > T; all particles when there is none), and the sweep's tail is that
    sum past every knot."""
    tab = Table(*spec)
    xyz, h, val = synth.random_scene(seed=31, n=40, h_lo=0.05, h_hi=0.15)
    o, v = synth.random_rays(seed=32, n=3)
    for r in range(3):
        per = _per_particle(o[r], v[r], 0.0, 3.0, xyz, h, val, tab, fp.Exact)
        pieces = fp.ray_pieces(o[r], v[r], 0.0, 3.0, xyz, h, val, tab.as_dict(), tab.K, tab.D, tab.kind,
                               n_reinit=n_reinit, num=fp.Exact)
        assert pieces
        Ts = fp.reinit_positions(0.0, 3.0, n_reinit, fp.Exact)
        for a, b, c in pieces:
            assert a < b
            prior = [T for T in Ts if T <= a]
            alive = [kn for kn in per.values() if not prior or kn[-1][0] > prior[-1]]
            for x in (a, (a + b) / 2, b - (b - a) / 7):
                got = sum(cd * (x - a) ** d for d, cd in enumerate(c))
                assert got == _direct(alive, x)


def test_particle_encodes_the_scaled_table_function():
    """One hit's knots and jumps (exact sums of its float32-rounded inputs) reproduce
    vf / zf^3 * f((t - tc) / zf), f the table's even piecewise polynomial (Sec. 3.2), to the
    float32 rounding of the inputs."""
    for spec in [("wendland", 2, 2, 256), ("cubic", 3, 3, 256), ("wendland", 4, 1, 256)]:
        tab = Table(*spec)
        rng = np.random.default_rng(3)
        for li in rng.integers(0, tab.n, 4):
            sh, sm = tab.row(int(li))
            tchi, zeta, value = 1.3, 0.07, 2.5
            kn = fp.particle_knots(tchi, zeta, value, tab.theta[li], sh, sm, tab.K, tab.D, fp.Exact)
            polys, r = lut.piece_polynomials(tab.kind, float(tab.lams[li]), tab.theta[li], tab.K, tab.D)
            th = r["theta"]
            zf, tc, vf = float(np.float32(zeta)), float(np.float32(tchi)), float(np.float32(value))
            span = th[-1] * zf
            for x in np.linspace(tc - 1.2 * span, tc + 1.2 * span, 57):
                u = abs(x - tc) / zf
                want = 0.0
                if u < th[-1]:
                    m = max(1, int(np.searchsorted(th, u, side="right")))
                    want = vf / zf ** 3 * polys[m - 1](u)
                got = float(_direct([kn], Fraction(float(x))))
                assert abs(got - want) <= 2e-6 * vf / zf ** 3, (spec, int(li), x, got, want)


def test_float32_sweep_sprinkles_behind_the_particles():
    """Behind the particles the float32 field does not return to zero (Sec. 4.1: measured 1e-5 to
    5e-4 of the ray's peak on these rays through a cluster core), and reinitialization knots
    remove that residue there (the last one lies behind the cluster)."""
    tab = Table("wendland", 4, 3, 4096)
    xyz, h, val = synth.clustered_particles(seed=7, n=3000, clusters=1)
    o = np.array([0.5, 0.5, -1.0])
    tails = {0: [], 10: []}
    rng = np.random.default_rng(8)
    for _ in range(3):
        tgt = np.array([0.5, 0.5, 0.5]) + rng.normal(0, 0.01, 3)
        v = (tgt - o) / np.linalg.norm(tgt - o)
        for n_re in (0, 10):
            pcs = fp.ray_pieces(o, v, 0.5, 3.0, xyz, h, val, tab.as_dict(), 4, 3, "wendland", n_reinit=n_re)
            peak = max(abs(float(c[0])) for _, _, c in pcs)
            a, b, c = pcs[-1]
            L = float(b) - float(a)
            tail = max(abs(sum(float(cd) * (L * s) ** d for d, cd in enumerate(c))) for s in (0.0, 0.5, 1.0))
            tails[n_re].append(tail / peak)
    assert max(tails[0]) > 1e-6            # no exact return to zero behind the particles
    assert np.mean(tails[10]) < np.mean(tails[0])
