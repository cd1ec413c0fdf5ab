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
import os

import numpy as np

import synth
from oracle import field, geometry, grid, lut, render
from oracle import quanta as quanta_mod
from tests.golden.make_knot_tables import load as load_knots

KIND_ID = {"cubic": 0, "wendland": 1, "wendland_c4": 2, "wendland_c6": 3, "wendland_grad": 4,
           "wendland_c4_grad": 5, "wendland_c6_grad": 6}


class Scene:
    """quanta: (a_max, h_repr, phi_repr, tau, sigma) when already known (skips the data analysis)."""

    def __init__(self, kind, K, D, n_lut, xyz, h, val, tol, tau_scale=1.0, lut_precision="fp64", quanta=None,
                 transverse=None):
        self.kind, self.K, self.D, self.n_lut, self.tol = kind, K, D, n_lut, tol
        self.xyz, self.h, self.val = xyz, h, val
        self.lut_precision = lut_precision
        self.transverse = transverse  # transverse gradient field along this axis (pair amplitude value * m)
        self.tau_scale = tau_scale
        self.theta = load_knots(kind, K, D, n_lut)
        # the table as stored (precision study): knots and projection rows rounded once
        self.theta_stored = lut.round_storage(self.theta, lut_precision)
        self._shat = None
        if quanta is None:
            self.a_max = grid.a_max(kind, xyz, h, val)
            if transverse is not None:
                self.a_max *= 2.0  # |value * m| <= 2 |value|
            self.h_repr, self.phi_repr = grid.representatives(h, val)
            self.tau, self.sigma = quanta_mod.choose_quanta(kind, D, self.a_max, self.h_repr, self.phi_repr)
            self.tau *= tau_scale
        else:
            self.a_max, self.h_repr, self.phi_repr, self.tau, self.sigma = quanta
        self._index = None

    def spec(self):
        """Constructor arguments of an equal scene (for worker processes)."""
        return dict(kind=self.kind, K=self.K, D=self.D, n_lut=self.n_lut, xyz=self.xyz, h=self.h, val=self.val,
                    tol=self.tol, lut_precision=self.lut_precision, transverse=self.transverse,
                    quanta=(self.a_max, self.h_repr, self.phi_repr, self.tau, self.sigma))

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
                                                lut_precision=self.lut_precision, transverse=self.transverse)
        return self._index

    def oracle_ray(self, o, v, t_min, t_max, tol=None):
        return field.ray_field(np.asarray(o, np.float64), np.asarray(v, np.float64), t_min, t_max, self.xyz, self.h,
                               self.val, self.table(), (self.tau, self.sigma), self.K, self.D, self.kind,
                               self.tol if tol is None else tol, transverse=self.transverse)


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


# ---------------------------------------------------------------- per-ray comparison with the oracle

_OUT_KEYS = ("ray_offsets", "t_start", "t_end", "coef", "ray_peak", "knot_offsets", "knot_t", "knot_pid", "knot_kidx",
             "exact_offsets", "exact_t", "exact_end", "exact_coef")


def host_out(out):
    """Host (numpy) copies of the arrays of an approx_rays / approx_camera result."""
    return {k: out[k].cpu().numpy() for k in _OUT_KEYS if k in out}


def ray_data(h, r):
    """Ray r of a host_out result (the form compare_ray takes)."""
    a, b = int(h["ray_offsets"][r]), int(h["ray_offsets"][r + 1])
    g = {"t0": h["t_start"][a:b], "t1": h["t_end"][a:b], "coef": h["coef"][a:b], "peak": float(h["ray_peak"][r])}
    if "knot_offsets" in h:
        ka, kb = int(h["knot_offsets"][r]), int(h["knot_offsets"][r + 1])
        g["knots"] = (h["knot_t"][ka:kb], h["knot_pid"][ka:kb], h["knot_kidx"][ka:kb])
        ea, eb = int(h["exact_offsets"][r]), int(h["exact_offsets"][r + 1])
        g["exact"] = (h["exact_t"][ea:eb], h["exact_end"][ea:eb], h["exact_coef"][ea:eb])
    return g


def library_merged(pcs, t0, t1, coef, tau):
    """The library's merged pieces of one ray as check_merged input: each float32 end mapped to the
    exact piece boundary (integer position) it is the rounding of, plus the float32 ends the
    coefficients refer to.  Returns (merged, ends, errors)."""
    errors = []
    bounds = ([p[0] for p in pcs] + [pcs[-1][1]]) if pcs else []
    cand = {}
    for q in bounds:
        cand.setdefault(float(np.float32(np.float64(q) * tau)), []).append(int(q))
    merged, ends = [], []
    prev = None
    for a, b, c in zip(t0.tolist(), t1.tolist(), coef):
        ca, cb = cand.get(float(a)), cand.get(float(b))
        if not ca or not cb:
            errors.append(f"merged end {a} / {b} is not the float32 of an exact piece boundary")
            continue
        qa = prev if (prev is not None and prev in ca) else ca[0]
        later = [q for q in cb if q > qa]
        qb = later[0] if later else cb[-1]
        merged.append((qa, qb, np.asarray(c, dtype=np.float64)))
        ends.append((float(a), float(b)))
        prev = qb
    return merged, ends, errors


def compare_ray(sc, f, g, coef_tol=1e-8, field_tol=1e-5, vtol=None, pixel=None):
    """Compare one ray of the library (g, from ray_data, optionally with "hits": the ray's hit ids)
    with the oracle's ray field f.  Returns (errors, stats).

    Bars: hit set, knot list (position, particle, kidx) and exact-piece boundaries bit-exact;
    integer coefficients per order within coef_tol * 100 of the order's largest value on the ray
    (plus one unit), exact-piece values within vtol of the ray peak (default 1e-9 for D <= 3, 1e-6
    for D >= 4: the projections are computed independently on both sides and the Gram system of
    Sec. 3.3 conditions worse with D), the float32 peak within its rounding plus vtol; the merged
    field valid by oracle.field.check_merged with its coefficients, evaluated on the library's own
    float32 ends, within field_tol of the peak; pixel = (rgba, t_min, t_max, tf, vmin, vmax, step):
    the library's pixel within 1e-4 of the oracle's compositing of the projections on the library's
    (validated) partition."""
    D = sc.D
    errors = []
    stats = {}
    if vtol is None:
        vtol = 1e-9 if D <= 3 else 1e-6
    if "hits" in g:
        got = np.sort(np.asarray(g["hits"], dtype=np.int64))
        want = np.sort(np.asarray(f["hits"], dtype=np.int64))
        if not np.array_equal(got, want):
            errors.append(f"hit set differs ({len(got)} vs {len(want)})")
        stats["hits"] = len(want)
    if "knots" in g:
        kt, kp, kk = g["knots"]
        ref = f["knots"]
        if len(kt) != len(ref) or list(zip(kt.tolist(), kp.tolist(), kk.tolist())) != \
                [(t, p, k) for (t, p, k, _) in ref]:
            errors.append(f"knot list differs ({len(kt)} vs {len(ref)} knots)")
    pcs = f["pieces"]
    if "exact" in g:
        et, ee, ec = g["exact"]
        if et.tolist() != [p[0] for p in pcs] or ee.tolist() != [p[1] for p in pcs]:
            errors.append("exact piece boundaries differ")
        elif pcs:
            oc = np.array([[float(x) for x in p[2]] for p in pcs])
            scale = np.maximum(np.abs(oc).max(axis=0), 1.0)
            if not np.all(np.abs(ec.astype(np.float64) - oc) <= coef_tol * 100 * scale + 1.0):
                errors.append("integer coefficients differ")
            L = (ee - et).astype(np.float64)
            for x in (0.0, 0.5, 1.0):
                xs = x * L
                vg = sum(ec[:, d].astype(np.float64) * xs ** d for d in range(D + 1))
                vo = sum(oc[:, d] * xs ** d for d in range(D + 1))
                err = np.max(np.abs(vg - vo)) * sc.sigma
                if err > vtol * max(f["peak"], 1e-300) + 4 * sc.sigma:
                    errors.append(f"exact-piece values differ by {err / max(f['peak'], 1e-300):.3g} of the peak")
                    break
    pk = g["peak"]
    if abs(pk - f["peak"]) > (vtol + 6e-8) * f["peak"]:
        errors.append(f"peak {pk} vs {f['peak']}")
    merged, ends, merr = library_merged(pcs, g["t0"], g["t1"], g["coef"], sc.tau)
    errors.extend(merr)
    stats["n_lib"] = len(g["t0"])
    stats["n_greedy"] = len(f["nodes"])
    if not merr:
        chk = field.check_merged(pcs, merged, sc.tol, sc.tau, sc.sigma, D, coef_tol=field_tol, ends=ends)
        errors.extend(chk["errors"])
        stats["max_coef_err"] = chk["max_coef_err"]
        stats["max_resid_ratio"] = chk["max_resid_ratio"]
        if pixel is not None and not chk["errors"]:
            rgba, t_min, t_max, tf, vmin, vmax, step = pixel
            M = f["merger"]
            lo_of = {int(s): i for i, s in enumerate(M.start)}
            hi_of = {int(e): i for i, e in enumerate(M.end)}
            outn = [field.node_output(M.node(lo_of[qa], hi_of[qb]), M) for qa, qb, _ in merged]
            px = render.composite(outn, t_min, t_max, tf, vmin, vmax, step)
            d = float(np.max(np.abs(np.asarray(rgba, dtype=np.float64) - px)))
            stats["pixel_diff"] = d
            if d > 1e-4:
                errors.append(f"pixel {list(rgba)} vs {list(px)} ({d:.3g})")
    elif pixel is not None:
        errors.append("pixel not checked: the partition is invalid")
    return errors, stats


_POOL_SCENE = None


def _pool_init(spec):
    global _POOL_SCENE
    _POOL_SCENE = Scene(**spec)


def _pool_task(task):
    r, o, v, t_min, t_max, g, kw = task
    f = _POOL_SCENE.oracle_ray(o, v, t_min, t_max)
    errs, st = compare_ray(_POOL_SCENE, f, g, **kw)
    return r, errs, st


def pool_workers():
    return max(1, min(16, os.cpu_count() or 1))


def compare_rays_parallel(sc, tasks, workers=None, progress=None):
    """compare_ray over many rays in a pool of CPU processes (spawned: they never touch the GPU).
    tasks: [(r, o, v, t_min, t_max, g, kwargs)].  Returns {r: (errors, stats)}; progress(done) is
    called after every finished ray."""
    import multiprocessing as mp

    workers = workers or pool_workers()
    ctx = mp.get_context("spawn")
    res = {}
    with ctx.Pool(workers, initializer=_pool_init, initargs=(sc.spec(),)) as pool:
        for r, errs, st in pool.imap_unordered(_pool_task, tasks, chunksize=max(1, min(8, len(tasks) // (8 * workers)))):
            res[r] = (errs, st)
            if progress is not None:
                progress(len(res))
    return res


def summarize(res):
    """Failures and merge statistics of compare_rays_parallel results."""
    bad = {r: e for r, (e, _) in res.items() if e}
    n_lib = sum(st.get("n_lib", 0) for _, st in res.values())
    n_gr = sum(st.get("n_greedy", 0) for _, st in res.values())
    coef = max([st.get("max_coef_err", 0.0) for _, st in res.values()] or [0.0])
    pix = max([st.get("pixel_diff", 0.0) for _, st in res.values()] or [0.0])
    return {"bad": bad, "pieces_library": n_lib, "pieces_plain_greedy": n_gr, "max_coef_err": coef,
            "max_pixel_diff": pix}


def _pool_hits(task):
    r, o, v, t_min, t_max, got = task
    want = geometry.ray_hits(np.asarray(o, np.float64), np.asarray(v, np.float64), t_min, t_max, _POOL_SCENE.xyz,
                             _POOL_SCENE.h, 2.0)
    same = np.array_equal(np.sort(np.asarray(got, np.int64)), np.sort(np.asarray(want, np.int64)))
    return r, same, len(want)


def compare_hits_parallel(sc, tasks, workers=None):
    """Hit sets of many rays against oracle.geometry.ray_hits (brute force over all particles) in a
    pool of CPU processes.  tasks: [(r, o, v, t_min, t_max, library hit ids)].  Returns
    {r: (same, oracle hit count)}."""
    import multiprocessing as mp

    workers = workers or pool_workers()
    ctx = mp.get_context("spawn")
    res = {}
    with ctx.Pool(workers, initializer=_pool_init, initargs=(sc.spec(),)) as pool:
        for r, same, n in pool.imap_unordered(_pool_hits, tasks, chunksize=max(1, len(tasks) // (8 * workers))):
            res[r] = (same, n)
    return res


def hit_lists(offs, ids, rays):
    """{r: hit ids of ray r} from sph_hoa_camera_hits / sph_hoa_ray_hits outputs (device tensors)."""
    o = offs.cpu().numpy()
    i = ids.cpu().numpy()
    return {int(r): i[o[r]:o[r + 1]] for r in rays}
