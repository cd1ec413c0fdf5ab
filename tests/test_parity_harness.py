"""The GPU parity harness (tests/gpu_helpers.compare_ray) on the CPU: a library output written from
the oracle's own results in the library's format (float32 ends, coefficients re-expressed on them)
passes, and each planted mistake is reported; the process-pool path gives the same verdicts."""
import numpy as np
import pytest

import synth
from oracle import field, geometry, render
from tests import gpu_helpers as H


def _scene():
    xyz, h, val = synth.random_scene(41, 300, h_lo=0.04, h_hi=0.1)
    return H.Scene("cubic", 4, 2, 4096, xyz, h, val, 1e-3)


def _as_library(sc, f):
    """f's greedy merge in the library's output format (as the field kernel writes it)."""
    M = f["merger"]
    t0, t1, coef = [], [], []
    for n in f["nodes"]:
        ta, tb = n["a"] * sc.tau, n["b"] * sc.tau
        fa, fb = np.float32(ta), np.float32(tb)
        c = M.to_power(n)
        L = (n["b"] - n["a"]) * sc.tau
        al, be = (float(fa) - ta) / L, (float(fb) - float(fa)) / L
        comp = np.polynomial.polynomial.polyval(np.polynomial.polynomial.Polynomial([al, be]), c).coef
        comp = np.pad(comp, (0, sc.D + 1 - len(comp)))
        t0.append(fa)
        t1.append(fb)
        coef.append(comp.astype(np.float32))
    pcs = f["pieces"]
    g = {"t0": np.array(t0, np.float32), "t1": np.array(t1, np.float32),
         "coef": np.array(coef, np.float32).reshape(-1, sc.D + 1), "peak": float(np.float32(f["peak"])),
         "hits": np.array(f["hits"], np.int32),
         "knots": (np.array([k[0] for k in f["knots"]], np.int64), np.array([k[1] for k in f["knots"]], np.int32),
                   np.array([k[2] for k in f["knots"]], np.int32)),
         "exact": (np.array([p[0] for p in pcs], np.int64), np.array([p[1] for p in pcs], np.int64),
                   np.array([[int(x) for x in p[2]] for p in pcs], np.int64).reshape(-1, sc.D + 1))}
    return g


def _rays():
    o, v = synth.random_rays(8, 6)
    return [(o[i].astype(np.float64), v[i].astype(np.float64)) for i in range(6)]


def test_compare_ray_accepts_the_oracle_and_flags_mistakes():
    sc = _scene()
    tf = synth.transfer_function().astype(np.float64)
    seen = 0
    for o, v in _rays():
        f = sc.oracle_ray(o, v, -0.5, 3.5)
        if len(f["nodes"]) < 2:
            continue
        seen += 1
        g = _as_library(sc, f)
        px = H.oracle_pixel(sc, f, -0.5, 3.5, tf, 0.0, 3e3, 4.0 / 256)
        errs, st = H.compare_ray(sc, f, g, pixel=(px, -0.5, 3.5, tf, 0.0, 3e3, 4.0 / 256))
        assert errs == [], errs
        assert st["n_lib"] == st["n_greedy"] and st["pixel_diff"] < 1e-6 and st["max_coef_err"] < 1e-6
        bad = dict(g, hits=g["hits"][1:])
        assert any("hit set" in e for e in H.compare_ray(sc, f, bad)[0])
        kt, kp, kk = g["knots"]
        bad = dict(g, knots=(kt, kp[::-1].copy(), kk))
        assert any("knot list" in e for e in H.compare_ray(sc, f, bad)[0])
        et, ee, ec = g["exact"]
        ec2 = ec.copy()
        ec2[len(ec2) // 2, 0] += max(1, abs(int(ec2[:, 0].max())) // 1000)
        assert H.compare_ray(sc, f, dict(g, exact=(et, ee, ec2)))[0]
        c2 = g["coef"].copy()
        c2[0, 0] += np.float32(3e-5 * f["peak"])
        assert any("coefficients" in e for e in H.compare_ray(sc, f, dict(g, coef=c2))[0])
        t2 = g["t0"].copy()
        t2[1] = np.nextafter(t2[1], np.float32(10))
        assert H.compare_ray(sc, f, dict(g, t0=t2))[0]
        wrong_px = np.asarray(px) + np.array([0, 0, 2e-4, 0])
        assert any("pixel" in e for e in H.compare_ray(sc, f, g, pixel=(wrong_px, -0.5, 3.5, tf, 0.0, 3e3,
                                                                        4.0 / 256))[0])
    assert seen >= 3


def test_pool_gives_the_same_verdicts():
    sc = _scene()
    tasks = []
    for i, (o, v) in enumerate(_rays()):
        f = sc.oracle_ray(o, v, -0.5, 3.5)
        g = _as_library(sc, f)
        if i % 2:
            g = dict(g, hits=g["hits"][:-1])
        tasks.append((i, o, v, -0.5, 3.5, g, {}))
    res = H.compare_rays_parallel(sc, tasks, workers=2)
    assert sorted(res) == list(range(6))
    for i, (errs, st) in res.items():
        if i % 2 and len(tasks[i][5]["hits"]) + 1 > 0 and st.get("hits", 0) > 0:
            assert any("hit set" in e for e in errs)
        elif not i % 2:
            assert errs == [], errs
    s = H.summarize(res)
    assert s["pieces_library"] == s["pieces_plain_greedy"]
