"""Benchmark: particle-ray contributions per second of the rendering path on one MI355X.

Workload (default): the plain GPU configuration - 1,000,000 particles from a
16-cluster Gaussian mixture plus 10 % uniform background, h = r32 / 2, values
= SPH density (amplitude 1/N), Wendland C2, K = 4, D = 3, merge tolerance
1e-3, 512 x 512 perspective rays, t in [1, 3].  One step = one full frame:
camera rays, hit gathering, knot generation, sort, exact accumulation, merge,
classification and compositing (sph_hoa_render).  The index (grid, tables,
quanta) is built once before the timed region, as a viewer would keep it
resident.

Prints one JSON line.  `value` = contributions (particle, ray pairs) over the
timed frames divided by the timed wall time; p50/p99 are per-frame wall
latencies.  `roofline` covers the per-ray field kernel, timed with hipEvents
inside the library on the rendering stream; `cpu_baseline` times the oracle on
a bounded sample of the same frame's rays on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X unit counts and clock, and the integer arithmetic rate used for the ALU roofline
# (256 CUs x 4 SIMD x 16 lanes x 2.4 GHz).  On gfx950 the 32-bit integer multiplies
# (v_mul_lo_u32, v_mad_u64_u32) issue at the full VALU rate: the 32-bit loop of the bit-length
# workload below sustains more than twice a quarter-rate bound.
N_CU, CLOCK_HZ = 256, 2.4e9
LANES_PER_CLK = N_CU * 64                   # 32-bit VALU lanes per clock
INT32_MUL_PER_S = LANES_PER_CLK * CLOCK_HZ  # 3.93e13 32-bit multiplies / s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--particles", type=int, default=1_000_000)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--parity-rays", type=int, default=2621,
                    help="rays of the seeded subsample checked against the oracle (and timed as the CPU baseline)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--rates", default="1,2,200", help="serve workload: Poisson arrival rates (requests/s), one "
                    "run each")
    ap.add_argument("--requests", type=int, default=16, help="serve workload: requests per rate")
    ap.add_argument("--sides", default="128,256,512,1024,2048", help="serve workload: image sides (uniform choice)")
    ap.add_argument("--serve-sets", default="2000000,8000000,32000000", help="serve workload: resident set sizes")
    ap.add_argument("--batch-sets", default="500000,2000000,4000000,16000000", help="batch workload: set sizes")
    ap.add_argument("--lanes", type=int, default=2, help="batch and serve workloads: server lanes")
    ap.add_argument("--precision-rays", type=int, default=48, help="precision workload: oracle rays per format")
    ap.add_argument("--budget-gib", type=int, default=96, help="batch and serve workloads: server HBM budget")
    ap.add_argument("--workload", choices=("plain", "batch", "serve", "bitlength", "precision", "sprinkle",
                                           "gradient"),
                    default="plain",
                    help="plain: the 1M-particle 512x512 frame (the reported metric); batch: camera bundles "
                         "of 32^2..512^2 rendered with one sph_hoa_render_batch call; serve: Poisson render "
                         "requests to the native render server; bitlength: the accumulation rule in 32/64/96/"
                         "128-bit integers (the cost study of Sec. 5.1); precision: the plain frame with the "
                         "float table stored in fp64 / fp32 / bf16, timed, with pixel errors against the "
                         "float64 oracle; sprinkle: the float32 accumulation variant with and without "
                         "reinitialization knots (Sec. 4.1), its residue behind the particles and its time; "
                         "gradient: the value field and the four transverse gradient fields (Sec. 6) on the "
                         "plain frame's rays")
    ap.add_argument("--batch-cams", type=int, default=256, help="ray bundles per step (batch workload)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="instead of the benchmark, run 5 plain device copies of MIB MiB each (the "
                         "reference kernel for scaling the HBM byte counters) and exit")
    return ap.parse_args()


def _build(L, xyz, h, val, D, tables):
    """Index of a clustered set (Wendland C2, K = 4, degree D) with the oracle-written knot table."""
    from tests.golden.make_knot_tables import load as load_knots

    if D not in tables:
        tables[D] = load_knots("wendland", 4, D, 4096)
    return L.sph_hoa_build_index(xyz, h, val, kernel=L.KERNEL_WENDLAND_C2, degree=D, pieces=4, lut_entries=4096,
                                 merge_tol=1e-3, knot_table=tables[D])


def _served(srv, reqs):
    """Submit every (slot, camera, tf, vmin, vmax, step) at once, wait for all; (outputs, latencies ms)."""
    subs = [srv.submit(*r) for r in reqs]
    outs, lat = [], []
    for rid, out in subs:
        done, ms = srv.wait(rid)
        assert done
        outs.append(out)
        lat.append(ms)
    return outs, lat


def camera_oracle_leg(L, jobs, workers=None):
    """Sampled pixels of rendered images against the oracle (bench's CPU-baseline leg of the batch
    and serve workloads).  jobs: [(scene spec (index info, xyz, h, val, D), index, camera, image
    (host [n][4]), sampled pixel rays, tf, vmin, vmax, step)].  Per ray, as for the plain frame: the
    render's hit set equals the oracle's, its merged partition passes the oracle's checker, and the
    pixel agrees with the oracle's compositing of those projections within 1e-4.  Returns
    (cpu_baseline, parity)."""
    from oracle import geometry
    from tests import gpu_helpers as H

    tasks_by_scene, scenes = [], []
    for spec, idx, cam, img, rays, tf, vmin, vmax, step in jobs:
        info, xyz, h, val, D = spec[:5]
        prec = spec[5] if len(spec) > 5 else "fp64"
        sc = H.Scene("wendland", 4, D, 4096, xyz, h, val, 1e-3, lut_precision=prec,
                     quanta=(info["a_max"], info["h_repr"], info["phi_repr"], info["tau"], info["sigma"]))
        oo, vv = geometry.camera_rays(cam)
        fo = L.sph_hoa_approx_camera(idx, cam)
        hout = H.host_out(fo)
        del fo
        offs, ids = L.sph_hoa_camera_hits(idx, cam)
        hits = H.hit_lists(offs, ids, rays)
        del offs, ids
        tf64 = np.asarray(tf, dtype=np.float64)
        tasks = []
        for r in rays:
            r = int(r)
            g = H.ray_data(hout, r)
            g["hits"] = hits[r]
            tasks.append((r, oo[r], vv[r], float(cam["t_min"]), float(cam["t_max"]), g,
                          {"pixel": (img[r], float(cam["t_min"]), float(cam["t_max"]), tf64, vmin, vmax, step)}))
        scenes.append(sc)
        tasks_by_scene.append(tasks)
    workers = workers or H.pool_workers()
    t0 = time.perf_counter()
    res_all, n_hits = {}, 0
    for j, (sc, tasks) in enumerate(zip(scenes, tasks_by_scene)):
        res = H.compare_rays_parallel(sc, tasks, workers=workers)
        for r, v in res.items():
            res_all[(j, r)] = v
            n_hits += v[1].get("hits", 0)
        print(f"oracle leg: image {j + 1}/{len(scenes)} checked ({time.perf_counter() - t0:.0f} s)", file=sys.stderr,
              flush=True)
    elapsed = time.perf_counter() - t0
    s = H.summarize(res_all)
    base = {"value": n_hits / elapsed, "unit": "contributions/s", "cores": workers, "kind": "oracle",
            "nproc": os.cpu_count() or 1,
            "sample": f"{len(res_all)} sampled pixel rays of {len(scenes)} of the rendered images ({n_hits} "
                      f"contributions): FP64 oracle with Python-integer accumulation plus the parity checks, "
                      f"{workers} worker processes, {elapsed:.1f} s wall"}
    parity = {"rays": len(res_all), "rays_failed": len(s["bad"]),
              "failures": {str(r): e[:2] for r, e in list(s["bad"].items())[:5]},
              "field_max_coef_err_rel_peak": s["max_coef_err"], "field_tol": 1e-5,
              "max_abs_rgba": s["max_pixel_diff"], "rgba_tol": 1e-4}
    return base, parity


def _lane_summary(st, st0):
    return {"batches": st["batches"] - st0["batches"], "lanes": st["lanes"],
            "overlapped_batches": st["overlapped_batches"] - st0["overlapped_batches"],
            "max_in_flight": st["max_in_flight"], "lane_busy_s": st["busy_s"] - st0["busy_s"]}


def run_batch(a, torch, L, synth):
    """Batch workload (many ray bundles over several resident sets): four clustered sets of 0.5M,
    2M, 4M and 16M particles (Wendland C2, K = 4, tol 1e-3), a.batch_cams bundles with square sides
    2^k, k uniform in 5..9 (32^2..512^2), eyes on the radius-2 sphere about the cube centre, half
    of them narrow views through cluster cores (the heavy tail of hits per ray), each bundle on a
    random set with a random degree D in {2, 3, 4} (one index per set and degree).  One step = every
    bundle rendered: all are submitted to the native server at once, which groups them per index
    into batched launch chains and runs a.lanes of them at a time on their own streams.  Also
    timed: the same bundles as one sph_hoa_render_batch call per index, one after the other."""
    sizes = [int(x) for x in a.batch_sets.split(",")]
    tf = torch.as_tensor(synth.transfer_function(), device="cuda")
    vmin, vmax, step = 0.0, 300.0, 2.0 / 512
    rng = np.random.default_rng(4)
    n_b = a.batch_cams
    set_of = rng.integers(0, len(sizes), n_b)
    deg_of = rng.choice([2, 3, 4], n_b)
    t_gen = time.time()
    sets = []
    for i, n in enumerate(sizes):
        sets.append(synth.clustered_particles(seed=40 + i, n=n))
        print(f"batch: set {i} ({n} particles) generated ({time.time() - t_gen:.0f} s)", file=sys.stderr, flush=True)
    gen_s = time.time() - t_gen
    cams_by_set = [synth.batch_cameras(seed=400 + i, n=n_b, centres=synth.cluster_centres(seed=40 + i))
                   for i in range(len(sizes))]
    cams = [cams_by_set[set_of[j]][j] for j in range(n_b)]
    tables, idx = {}, {}
    t_idx = time.time()
    for j in range(n_b):
        key = (int(set_of[j]), int(deg_of[j]))
        if key not in idx:
            xyz, h, val = sets[key[0]]
            idx[key] = _build(L, xyz, h, val, key[1], tables)
    torch.cuda.synchronize()
    index_s = time.time() - t_idx
    print(f"batch: {len(idx)} indices built ({time.time() - t_gen:.0f} s)", file=sys.stderr, flush=True)
    keys = sorted(idx)
    srv = L.Server(hbm_budget_bytes=a.budget_gib << 30, max_batch_rays=1 << 24, lanes=a.lanes)
    slots = {k: srv.add_index(idx[k]) for k in keys}
    reqs = [(slots[(int(set_of[j]), int(deg_of[j]))], cams[j], tf, vmin, vmax, step) for j in range(n_b)]
    for _ in range(a.warmup):
        _served(srv, reqs)
        print(f"batch: warm-up step done ({time.time() - t_gen:.0f} s)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    st0 = srv.stats()
    lat_steps, step_lat = [], []
    t0 = time.perf_counter()
    outs = None
    for _ in range(a.steps):
        ts = time.perf_counter()
        outs, lat = _served(srv, reqs)
        torch.cuda.synchronize()
        step_lat.append(time.perf_counter() - ts)
        lat_steps.extend(lat)
        print(f"batch: timed step done ({time.time() - t_gen:.0f} s)", file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t0
    st = srv.stats()
    pairs = st["n_pairs"] - st0["n_pairs"]
    imgs = [o.cpu().numpy().reshape(-1, 4) for o in outs]
    srv.close()
    # the same bundles as one render_batch call per index, sequentially (per-index kernel times and
    # ray layouts from the library's timing), and as one sph_hoa_render call per bundle (the plain
    # path on the same work)
    groups = {k: [j for j in range(n_b) if (int(set_of[j]), int(deg_of[j])) == k] for k in keys}
    for k in keys:
        L.sph_hoa_render_batch(idx[k], [cams[j] for j in groups[k]], tf, vmin, vmax, step)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    seq_pairs = 0
    per_index = {}
    for k in keys:
        idx[k].set_timing(True)
        L.sph_hoa_render_batch(idx[k], [cams[j] for j in groups[k]], tf, vmin, vmax, step)
        st_k = idx[k].stats()
        print(f"batch: set {k[0]} D={k[1]} by one render_batch call ({time.time() - t_gen:.0f} s)", file=sys.stderr,
              flush=True)
        idx[k].set_timing(False)
        seq_pairs += st_k["n_pairs"]
        per_index[f"set{k[0]}_D{k[1]}"] = {
            "bundles": len(groups[k]), "rays": st_k["n_rays"], "pairs": st_k["n_pairs"],
            "max_hits_per_ray": st_k["max_hits"], "field_ms": st_k["ms_field"], "gather_ms": st_k["ms_gather"],
            "rays_jump_rows_in_hbm": st_k["rays_jumps_device"],
            "rays_jump_rows_and_sort_scratch_in_hbm": st_k["rays_scratch_device"],
            "rays_all_in_hbm": st_k["rays_global"]}
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - ts
    for j in range(n_b):
        L.sph_hoa_render(idx[(int(set_of[j]), int(deg_of[j]))], cams[j], tf, vmin, vmax, step)
        if j % 32 == 31:
            print(f"batch: single-call warm-up {j + 1}/{n_b} ({time.time() - t_gen:.0f} s)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    single_pairs = 0
    for j in range(n_b):
        ix = idx[(int(set_of[j]), int(deg_of[j]))]
        L.sph_hoa_render(ix, cams[j], tf, vmin, vmax, step)
        single_pairs += ix.stats()["n_pairs"]
        if j % 32 == 31:
            print(f"batch: single calls {j + 1}/{n_b} ({time.time() - t_gen:.0f} s)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    single_s = time.perf_counter() - ts
    n_rays = sum(c["width"] * c["height"] for c in cams)
    step_ms = np.array(step_lat) * 1e3
    result = {
        "metric": "particle-ray contributions/s at rel err <=1e-5; p50/p99 frame latency",
        "value": pairs / elapsed, "unit": "contributions/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": elapsed / a.steps * 1e3, "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"batch: {n_b} ray bundles (32^2..512^2, half through cluster cores) over resident "
                               f"clustered sets of {sizes} particles, Wendland C2, K=4, D in {{2,3,4}} per bundle, "
                               f"tol 1e-3; all bundles submitted at once to the native server ({a.lanes} lanes)",
                   "indices": len(keys), "rays_per_step": n_rays, "pairs_per_step": pairs // max(1, a.steps),
                   "bundle_latency_p50_ms": float(np.percentile(lat_steps, 50)),
                   "bundle_latency_p99_ms": float(np.percentile(lat_steps, 99)),
                   "server": _lane_summary(st, st0),
                   "sequential_render_batch_per_index_s": seq_s,
                   "sequential_contributions_per_s": seq_pairs / seq_s,
                   "single_render_calls_s": single_s,
                   "single_render_calls_contributions_per_s": single_pairs / single_s,
                   "per_index": per_index,
                   "generate_s": gen_s, "index_build_s": index_s},
        "cpu_baseline": None,
    }
    if not a.no_cpu:
        prng = np.random.default_rng(44)
        pick = prng.choice(n_b, size=min(8, n_b), replace=False)
        jobs = []
        for j in pick:
            k = (int(set_of[j]), int(deg_of[j]))
            xyz, h, val = sets[k[0]]
            n = cams[j]["width"] * cams[j]["height"]
            rays = np.sort(prng.choice(n, size=min(4, n), replace=False))
            jobs.append(((idx[k].info(), xyz, h, val, k[1]), idx[k], cams[j], imgs[j], rays,
                         synth.transfer_function(), vmin, vmax, step))
        result["cpu_baseline"], result["parity"] = camera_oracle_leg(L, jobs)
    for k in keys:
        idx[k].free()
    print(json.dumps(result), flush=True)


def run_serve(a, torch, L, synth):
    """Serving workload: render requests arrive as Poisson streams at the native render server, which
    holds three resident clustered sets (default 2M, 8M and 32M particles, Wendland C2, K = 4,
    D = 3, tol 1e-3).  Each request is one random camera on the radius-2 sphere (half of them narrow
    views through cluster cores) with a square image of a side drawn uniformly from a.sides, on a
    uniformly drawn set.  For each offered rate in a.rates, a.requests requests arrive at that
    Poisson rate; the run reports latency (submit to completion) against the offered load and the
    served contribution rate (the headline line is the last rate)."""
    sizes = [int(x) for x in a.serve_sets.split(",")]
    sides = [int(x) for x in a.sides.split(",")]
    rates = [float(x) for x in a.rates.split(",")]
    tf = torch.as_tensor(synth.transfer_function(), device="cuda")
    vmin, vmax, step = 0.0, 300.0, 2.0 / 512
    t_gen = time.time()
    sets, tables, idxs = [], {}, []
    for i, n in enumerate(sizes):
        sets.append(synth.clustered_particles(seed=50 + i, n=n))
        idxs.append(_build(L, *sets[-1], 3, tables))
        torch.cuda.synchronize()
        print(f"serve: set {i} ({n} particles) ready ({time.time() - t_gen:.0f} s)", file=sys.stderr, flush=True)
    setup_s = time.time() - t_gen
    srv = L.Server(hbm_budget_bytes=a.budget_gib << 30, max_batch_rays=max(sides) ** 2, lanes=a.lanes)
    slots = [srv.add_index(ix) for ix in idxs]
    rng = np.random.default_rng(5)
    # warm-up: every set at every side once (hit estimates, lane buffers), not counted
    warm = []
    for i in range(len(sizes)):
        cam = synth.batch_cameras(seed=500 + i, n=1, centres=synth.cluster_centres(seed=50 + i))[0]
        for sd in sides:
            warm.append((slots[i], dict(cam, width=sd, height=sd), tf, vmin, vmax, step))
    _served(srv, warm)
    table, last = [], None
    sample = []
    for rate in rates:
        n_req = a.requests
        arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
        which = rng.integers(0, len(sizes), n_req)
        cams = []
        for q in range(n_req):
            c = synth.batch_cameras(seed=int(rng.integers(1 << 30)), n=1,
                                    centres=synth.cluster_centres(seed=50 + int(which[q])))[0]
            sd = int(sides[int(rng.integers(len(sides)))])
            cams.append(dict(c, width=sd, height=sd))
        st0 = srv.stats()
        subs = []
        t0 = time.perf_counter()
        for q in range(n_req):
            dt = arrivals[q] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            subs.append(srv.submit(slots[int(which[q])], cams[q], tf, vmin, vmax, step))
        lat = []
        for rid, _ in subs:
            lat.append(srv.wait(rid)[1])
        wall = time.perf_counter() - t0
        st = srv.stats()
        pairs = st["n_pairs"] - st0["n_pairs"]
        lat = np.array(lat)
        row = {"offered_requests_per_s": rate, "requests": n_req, "arrival_span_s": float(arrivals[-1]),
               "wall_s": wall, "served_requests_per_s": n_req / wall, "contributions_per_s": pairs / wall,
               "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "max_ms": float(lat.max()), "offered_rays_per_s": sum(c["width"] * c["height"] for c in cams) / max(
                   1e-9, float(arrivals[-1])),
               "served_rays": st["n_rays"] - st0["n_rays"], "pairs": pairs}
        row.update(_lane_summary(st, st0))
        table.append(row)
        print(f"serve: rate {rate}/s done: {json.dumps(row)}", file=sys.stderr, flush=True)
        last = row
        if not sample:
            # one served image per set for the oracle leg (the smallest side drawn at this rate)
            for i in range(len(sizes)):
                qs = [q for q in range(n_req) if int(which[q]) == i]
                if qs:
                    q = min(qs, key=lambda q: cams[q]["width"])
                    sample.append((i, cams[q], subs[q][1].cpu().numpy().reshape(-1, 4)))
    srv.close()
    result = {
        "metric": "particle-ray contributions/s at rel err <=1e-5; p50/p99 frame latency",
        "value": last["contributions_per_s"], "unit": "contributions/s", "n_gpus": 1, "steps": last["requests"],
        "warmup": len(warm), "ms_per_step": last["wall_s"] / last["requests"] * 1e3, "p50_ms": last["p50_ms"],
        "p99_ms": last["p99_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"serve: Poisson render requests at {rates} per s ({a.requests} each), sides {sides}, "
                               f"resident clustered sets of {sizes} particles, Wendland C2, K=4, D=3, tol 1e-3, "
                               f"native server with {a.lanes} lanes, HBM budget {a.budget_gib} GiB",
                   "latency_vs_offered_load": table, "setup_s": setup_s},
        "cpu_baseline": None,
    }
    if not a.no_cpu and sample:
        prng = np.random.default_rng(55)
        jobs = []
        for i, cam, img in sample:
            n = cam["width"] * cam["height"]
            rays = np.sort(prng.choice(n, size=min(4, n), replace=False))
            xyz, h, val = sets[i]
            jobs.append(((idxs[i].info(), xyz, h, val, 3), idxs[i], cam, img, rays, synth.transfer_function(),
                         vmin, vmax, step))
        result["cpu_baseline"], result["parity"] = camera_oracle_leg(L, jobs)
    for ix in idxs:
        ix.free()
    print(json.dumps(result), flush=True)


def run_bitlength(a, torch, L, synth):
    """Integer bit-length study (Sec. 5.1): the accumulation rule (Taylor shift by a 32-bit knot
    distance, then the jump added) in wrap-around 32, 64, 96 and 128-bit integers, 2^20
    independent accumulators x 1024 knots per launch, degrees 2, 3 and 4.  Reports knots/s per
    width and the cost of each width relative to 32 bits (the paper puts emulated 64/96/128-bit
    operations at about 9x/24x/45x a 32-bit one on the GPUs it used).  value = knots/s at 64 bits,
    D = 3 (the width and degree of the field kernel)."""
    n, steps = 1 << 20, 1024
    widths, degrees = (32, 64, 96, 128), (2, 3, 4)
    ms = {}
    for D in degrees:
        for bits in widths:
            dist, jumps = synth.bit_tables(seed=6, n_table=37, degree=D, bits=bits)
            for _ in range(max(1, a.warmup)):
                L.sph_hoa_accumulate_bits(bits, D, dist, jumps, n, steps, want_out=False)
            t = [L.sph_hoa_accumulate_bits(bits, D, dist, jumps, n, steps, want_out=False)[1]
                 for _ in range(a.steps)]
            ms[(D, bits)] = float(np.median(t))
    knots = float(n) * steps
    rate = {f"D{D}_w{b}": knots / (ms[(D, b)] * 1e-3) for D in degrees for b in widths}
    cost = {f"D{D}_w{b}": ms[(D, b)] / ms[(D, 32)] for D in degrees for b in widths}
    mul32 = 3 * 4 / 2 * knots / (ms[(3, 32)] * 1e-3)   # D (D + 1) / 2 32-bit multiplies per knot
    result = {
        "metric": "accumulation-rule knots/s by integer width (64-bit, D=3); cost relative to 32-bit",
        "value": rate["D3_w64"], "unit": "knots/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms[(3, 64)], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"bitlength: {n} accumulators x {steps} knots per launch (4-knot cycle in "
                               "registers), full-range 32-bit distances and W-bit jumps, widths 32/64/96/128, "
                               "D = 2, 3, 4",
                   "ms_per_launch": {f"D{D}_w{b}": ms[(D, b)] for D in degrees for b in widths},
                   "knots_per_s": rate, "cost_vs_32bit": cost,
                   "paper_cost_vs_32bit": {"w64": 9, "w96": 24, "w128": 45}},
        "roofline": {"bound": "alu", "achieved": mul32, "peak": INT32_MUL_PER_S, "unit": "int32 mul/s",
                     "frac": mul32 / INT32_MUL_PER_S, "traffic": None,
                     "note": "32-bit, D=3 launch: the rule's 6 multiplies per knot against the full-rate "
                             "32-bit multiply peak"},
        "cpu_baseline": None,
    }
    print(json.dumps(result), flush=True)


def run_precision(a, torch, L, synth):
    """Table storage precision at the precision configuration: 8M particles from the clustered
    generator with 64 clusters (seed 3), Wendland C2, K = 4, D = 3, tol 1e-3, the plain camera at
    1024^2, rendered with the float table of Sec. 3.1 stored (and read by the field kernel) in fp64,
    fp32, bf16 and fp16.  Reports each format's frame time and its pixel differences against the
    fp64-table frame and, on a sample of rays, against the float64 oracle run with the same stored
    table (hit sets, merged partition and pixels).  value = contributions/s with the bf16 table."""
    n = a.particles if a.particles != 1_000_000 else 8_000_000
    size = a.size if a.size != 512 else 1024
    xyz, h, val = synth.clustered_particles(seed=3, n=n, clusters=64)
    kind, K, D, tol = "wendland", 4, 3, 1e-3
    cam = synth.plain_camera(size, size)
    tf = synth.transfer_function()
    vmin, vmax, step = 0.0, 300.0, 2.0 / 512
    from tests.golden.make_knot_tables import load as load_knots

    theta = load_knots(kind, K, D, 4096)
    res, imgs, jobs = {}, {}, []
    prng = np.random.default_rng(33)
    rays = np.sort(prng.choice(size * size, size=a.precision_rays, replace=False))
    for fmt in ("fp64", "fp32", "bf16", "fp16"):
        idx = L.sph_hoa_build_index(xyz, h, val, kernel=L.KERNEL_WENDLAND_C2, degree=D, pieces=K, lut_entries=4096,
                                    merge_tol=tol, lut_precision=fmt, knot_table=theta)
        out = torch.empty((cam["height"], cam["width"], 4), dtype=torch.float32, device="cuda")
        for _ in range(max(1, a.warmup)):
            L.sph_hoa_render(idx, cam, tf, vmin, vmax, step, out=out)
        torch.cuda.synchronize()
        lat, pairs = [], 0
        for _ in range(a.steps):
            ts = time.perf_counter()
            L.sph_hoa_render(idx, cam, tf, vmin, vmax, step, out=out)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - ts)
            pairs += idx.stats()["n_pairs"]
        imgs[fmt] = out.reshape(-1, 4).cpu().numpy()
        res[fmt] = {"p50_ms": float(np.percentile(np.array(lat) * 1e3, 50)),
                    "contributions_per_s": pairs / sum(lat), "pairs_per_frame": pairs // max(1, a.steps)}
        print(f"precision: {fmt} table rendered ({res[fmt]['p50_ms']:.1f} ms)", file=sys.stderr, flush=True)
        if not a.no_cpu:
            leg_base, leg_par = camera_oracle_leg(L, [((idx.info(), xyz, h, val, D, fmt), idx, cam, imgs[fmt], rays,
                                                       tf, vmin, vmax, step)])
            res[fmt]["oracle_same_table"] = leg_par
            res[fmt]["oracle_contributions_per_s"] = leg_base["value"]
        idx.free()
    for fmt in ("fp32", "bf16", "fp16"):
        d = np.abs(imgs[fmt].astype(np.float64) - imgs["fp64"].astype(np.float64))
        res[fmt]["max_abs_rgba_vs_fp64_table"] = float(d.max())
        res[fmt]["mean_abs_rgba_vs_fp64_table"] = float(d.mean())
        if "oracle_same_table" in res["fp64"]:
            # the fp64-table frame meets the float64 oracle (max_abs_rgba); a narrow format's error
            # against that oracle is at most its difference from the fp64-table frame plus that
            res[fmt]["max_abs_rgba_vs_fp64_oracle_bound"] = float(
                d.max() + res["fp64"]["oracle_same_table"]["max_abs_rgba"])
            res[fmt]["meets_1e-4_vs_fp64_oracle"] = bool(res[fmt]["max_abs_rgba_vs_fp64_oracle_bound"] <= 1e-4)
    result = {
        "metric": "particle-ray contributions/s with the bf16 table; pixel error vs fp64 table and oracle",
        "value": res["bf16"]["contributions_per_s"], "unit": "contributions/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": res["bf16"]["p50_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"precision: {n} particles (64 clusters + 10% uniform, h=r32/2, SPH density), "
                               f"Wendland C2, K=4, D=3, tol 1e-3, {size}x{size} perspective, table stored and read in "
                               "fp64 / fp32 / bf16 / fp16",
                   "by_table_precision": res, "oracle_rays_per_format": int(len(rays))},
        "cpu_baseline": None,
    }
    print(json.dumps(result), flush=True)


def run_sprinkle(a, torch, L, synth):
    """Float accumulation variant (Sec. 4.1): the plain set (1M clustered particles, Wendland C2,
    K = 4, D = 3) seen by 128 x 128 rays from the plain camera's eye through a grid over the middle
    plane of the cube (x, y in [0.15, 0.85], z = 0.5); every ray swept in
    float32 without and with 10 reinitialization knots (sph_hoa_float_rays), against the exact
    integer path on the same rays (sph_hoa_approx_rays, whose fields return exactly to zero).
    Residue = the largest |float field| behind the ray's last knot (piece ends from there to t_max)
    over the ray's peak |value|.
    value = contributions/s of the float sweep without reinitialization knots."""
    xyz, h, val = synth.clustered_particles(n=a.particles)
    idx = L.sph_hoa_build_index(xyz, h, val, kernel=L.KERNEL_WENDLAND_C2, degree=3, pieces=4, lut_entries=4096,
                                merge_tol=1e-3)
    cam = synth.plain_camera(128, 128)
    g = np.linspace(0.15, 0.85, 128)
    gx, gy = np.meshgrid(g, g, indexing="xy")
    tgt = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, 0.5)], axis=1)
    eye = np.array(cam["eye"], np.float64)
    dirs = tgt - eye
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    o = torch.as_tensor(np.tile(eye, (len(dirs), 1)).astype(np.float32), device="cuda")
    v = torch.as_tensor(dirs.astype(np.float32), device="cuda")
    t_min, t_max = float(cam["t_min"]), float(cam["t_max"])
    n = o.shape[0]
    # the exact path on the same rays: its fields end exactly at each ray's last knot
    L.sph_hoa_approx_rays(idx, o, v, t_min, t_max)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    ex = L.sph_hoa_approx_rays(idx, o, v, t_min, t_max)
    torch.cuda.synchronize()
    exact_s = time.perf_counter() - ts
    eo = ex["ray_offsets"]
    ecnt = eo[1:] - eo[:-1]
    ecnt_h = ecnt.cpu().numpy()
    te = ex["t_end"].cpu().numpy()
    last_knot_h = np.where(ecnt_h > 0, te[np.maximum(eo[1:].cpu().numpy() - 1, 0)], -1e30)
    res = {}
    for n_re in (0, 10):
        L.sph_hoa_float_rays(idx, o, v, t_min, t_max, n_reinit=n_re)  # warm-up
        torch.cuda.synchronize()
        ts = time.perf_counter()
        out = L.sph_hoa_float_rays(idx, o, v, t_min, t_max, n_reinit=n_re)
        torch.cuda.synchronize()
        dt = time.perf_counter() - ts
        # per-ray maxima on the host over each ray's slot range (unused slots are zero); a device
        # gather of ~1e8 rows by index returned wrong rows with this torch build
        offs = out["ray_offsets"].cpu().numpy()
        cf = out["coef"].cpu().numpy().astype(np.float64)
        ts0 = out["t_start"].cpu().numpy()
        Lg = out["t_end"].cpu().numpy().astype(np.float64) - ts0
        v0 = np.abs(cf[:, 0])
        v1 = np.abs(sum(cf[:, d] * Lg ** d for d in range(cf.shape[1])))
        ray_of_slot = np.repeat(np.arange(n), np.diff(offs))
        # behind the particles: pieces from the ray's last knot on (the exact field is zero there)
        behind = ts0 >= last_knot_h[ray_of_slot] - 1e-5
        vb = np.where(behind, np.maximum(v0, v1), 0.0)
        peak = np.maximum.reduceat(v0, offs[:-1])
        resid = np.maximum.reduceat(vb, offs[:-1])
        del cf, v0, v1, vb, Lg, ts0, ray_of_slot, behind
        keep = (peak > 0) & (ecnt_h > 0)
        rel = resid[keep] / peak[keep]
        res[f"reinit_{n_re}"] = {"s": dt, "contributions_per_s": out["n_pairs"] / dt,
                                 "residue_rel_median": float(np.median(rel)),
                                 "residue_rel_p99": float(np.percentile(rel, 99)), "residue_rel_max": float(rel.max()),
                                 "rays_residue_above_1e-3": int((rel > 1e-3).sum()),
                                 "rays_with_particles": int(rel.size)}
        pairs = out["n_pairs"]
        del out
    result = {
        "metric": "float32 sweep contributions/s; residue behind the particles relative to the ray peak",
        "value": res["reinit_0"]["contributions_per_s"], "unit": "contributions/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": res["reinit_0"]["s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"sprinkle: {a.particles} clustered particles, Wendland C2, K=4, D=3, 128x128 rays "
                               "from the plain camera's eye, float32 sweep with 0 and 10 reinitialization knots",
                   "pairs": pairs, "float": res, "exact_path_s": exact_s,
                   "exact_path_contributions_per_s": pairs / exact_s, "exact_path_residue": 0.0},
        "cpu_baseline": None,
    }
    print(json.dumps(result), flush=True)


def camera_rays(cam, torch):
    """Pixel-centre rays of a pinhole camera as device float32 tensors (origins, unit directions)."""
    eye = np.array(cam["eye"], np.float64)
    fwd = np.array(cam["look_at"], np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    rgt = np.cross(fwd, np.array(cam["up"], np.float64))
    rgt /= np.linalg.norm(rgt)
    upv = np.cross(rgt, fwd)
    gy = math.tan(math.radians(cam["fov_y_deg"]) / 2)
    Wd, Hd = cam["width"], cam["height"]
    jj, ii = np.meshgrid(np.arange(Hd), np.arange(Wd), indexing="ij")
    ax = (((2 * ii + 1) / Wd - 1) * gy * Wd / Hd).reshape(-1, 1)
    by = ((1 - (2 * jj + 1) / Hd) * gy).reshape(-1, 1)
    dirs = fwd[None, :] + ax * rgt[None, :] + by * upv[None, :]
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    ro = torch.as_tensor(np.tile(eye, (len(dirs), 1)).astype(np.float32), device="cuda")
    rv = torch.as_tensor(dirs.astype(np.float32), device="cuda")
    return ro, rv


def run_gradient(a, torch, L, synth):
    """Gradient fields (Sec. 6): on the plain frame's pixel-centre rays (1M clustered particles,
    Wendland C2, K = 4, D = 3, tol 1e-3, 512^2 rays), the value field and the three transverse
    fields of the kernel -w'/r (particle values c/h, each pair's amplitude carrying its
    perpendicular offset from the ray along x, y or z), from which every gradient component along a
    ray is assembled ((v.e) F' - sum_a e_a T_a), all four by one sph_hoa_approx_rays_shared call
    (the hits gathered once) with merged output.  A step is all four fields of all rays; the same
    fields by four separate calls are timed after the timed region.  value = contributions/s over
    the four fields."""
    xyz, h, val = synth.clustered_particles(n=a.particles)
    K, D, tol = 4, 3, 1e-3
    cam = synth.plain_camera(a.size, a.size)
    ro, rv = camera_rays(cam, torch)
    tv = (val.astype(np.float64) / h.astype(np.float64)).astype(np.float32)
    t_idx = time.time()
    idxs = [L.sph_hoa_build_index(xyz, h, val, kernel=L.KERNEL_WENDLAND_C2, degree=D, pieces=K, lut_entries=4096,
                                  merge_tol=tol)]
    idxs += [L.sph_hoa_build_index(xyz, h, tv, kernel=L.KERNEL_WENDLAND_C2_GRAD, degree=D, pieces=K,
                                   lut_entries=4096, merge_tol=tol, transverse=ax) for ax in range(3)]
    build_s = time.time() - t_idx
    warm = L.sph_hoa_approx_rays_shared(idxs, ro, rv, cam["t_min"], cam["t_max"])
    cap = max(int(w["n_pieces"]) for w in warm) + 1024  # outputs sized once
    pieces = [int(w["n_pieces"]) for w in warm]
    del warm
    for _ in range(max(0, a.warmup - 1)):
        L.sph_hoa_approx_rays_shared(idxs, ro, rv, cam["t_min"], cam["t_max"], capacity=cap)
    torch.cuda.synchronize()
    lat, pairs = [], 0
    for _ in range(a.steps):
        ts = time.perf_counter()
        outs = L.sph_hoa_approx_rays_shared(idxs, ro, rv, cam["t_min"], cam["t_max"], capacity=cap)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        pairs += sum(x["n_pairs"] for x in outs)
        del outs
    # the same four fields by separate calls (each gathers its own hits), after the timed region
    sep = []
    for _ in range(2):
        ts = time.perf_counter()
        for idx in idxs:
            L.sph_hoa_approx_rays(idx, ro, rv, cam["t_min"], cam["t_max"], capacity=cap)
        torch.cuda.synchronize()
        sep.append(time.perf_counter() - ts)
    names = ["value F", "T_x", "T_y", "T_z"]
    result = {
        "metric": "particle-ray contributions/s over the value field and the three transverse gradient fields",
        "value": pairs / sum(lat), "unit": "contributions/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": float(np.median(lat) * 1e3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"gradient: {a.size}x{a.size} pixel-centre rays of the plain camera, {a.particles} "
                               "clustered particles, Wendland C2 and its transverse kernel -w'/r, K=4, D=3, "
                               "tol 1e-3, four fields per step through sph_hoa_approx_rays_shared (one gathering)",
                   "pieces": {n: pieces[i] for i, n in enumerate(names)},
                   "separate_calls_ms": float(min(sep) * 1e3),
                   "index_build_s": build_s},
        "cpu_baseline": None,
    }
    for idx in idxs:
        idx.free()
    print(json.dumps(result), flush=True)


def kernel_source_digest():
    import hashlib

    h = hashlib.sha256()
    for f in ("raycast.hip", "device.h", "impl.h"):
        with open(os.path.join(ROOT, "paper_2401_02896_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_traffic():
    """HBM bytes per k_field launch from the committed counter summary, or None when that summary
    was taken on a different kernel source (or is absent)."""
    path = os.path.join(ROOT, "profiles", "k_field_plain_1M_512_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_digest():
        return None
    return float(vals["traffic_bytes_per_launch"])


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}): every ray is independent, so N GPUs would "
              "split the image; this benchmark measures the one-GPU share.", file=sys.stderr)
        sys.exit(2)
    import torch

    if a.calibrate_copy:
        assert torch.cuda.is_available(), "bench.py needs the GPU"
        n = a.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 4, "copies": 5}), flush=True)
        return

    import paper_2401_02896_amd as L
    import synth

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    L.lib()
    if a.workload == "batch":
        return run_batch(a, torch, L, synth)
    if a.workload == "serve":
        return run_serve(a, torch, L, synth)
    if a.workload == "bitlength":
        return run_bitlength(a, torch, L, synth)
    if a.workload == "precision":
        return run_precision(a, torch, L, synth)
    if a.workload == "sprinkle":
        return run_sprinkle(a, torch, L, synth)
    if a.workload == "gradient":
        return run_gradient(a, torch, L, synth)
    t_gen = time.time()
    xyz, h, val = synth.clustered_particles(n=a.particles)
    gen_s = time.time() - t_gen
    kind, K, D, tol = "wendland", 4, 3, 1e-3
    cam = synth.plain_camera(a.size, a.size)
    tf = synth.transfer_function()
    vmin, vmax, step = 0.0, 300.0, 2.0 / 512
    # the optimal-knot table written by the oracle (the shared data artifact both sides load), so that
    # the parity leg below can compare knots and piece boundaries bit for bit
    from tests.golden.make_knot_tables import load as load_knots

    t_idx = time.time()
    idx = L.sph_hoa_build_index(xyz, h, val, kernel=L.KERNEL_WENDLAND_C2, degree=D, pieces=K, lut_entries=4096,
                                merge_tol=tol, knot_table=load_knots(kind, K, D, 4096))
    torch.cuda.synchronize()
    index_s = time.time() - t_idx
    info = idx.info()
    out = torch.empty((cam["height"], cam["width"], 4), dtype=torch.float32, device="cuda")
    for _ in range(a.warmup):
        L.sph_hoa_render(idx, cam, tf, vmin, vmax, step, out=out)
    torch.cuda.synchronize()
    idx.set_timing(True)
    lat = []
    pairs = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        ts = time.perf_counter()
        L.sph_hoa_render(idx, cam, tf, vmin, vmax, step, out=out)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        pairs += idx.stats()["n_pairs"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = idx.stats()
    idx.set_timing(False)
    pairs_per_frame = st["n_pairs"]
    value = pairs / elapsed
    lat_ms = np.array(lat) * 1e3
    field_ms = st["ms_field"] / max(1, st["timed_calls"])
    gather_ms = st["ms_gather"] / max(1, st["timed_calls"])
    # Roofline of the field kernel (ALU bound).  Algorithmic work per contribution: the integer
    # multiplies of the accumulation rule applied once to each of the particle's K + 1 knots,
    # D(D+1)/2 products of a 64-bit coefficient by a 32-bit distance, 2 32-bit multiplies each
    # (v_mad_u64_u32 for the low word, v_mul_lo_u32 for the high word).
    # (The kernel applies the rule three times per knot - aggregate, peak, pieces - and adds the
    # float64 merge, so the fraction also measures that overhead.)
    mul32_per_pair = (K + 1) * (D * (D + 1) // 2) * 2
    achieved = mul32_per_pair * pairs_per_frame / (field_ms * 1e-3) / 1e12
    peak = INT32_MUL_PER_S / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tmul32/s",
                "frac": achieved / peak, "traffic": committed_traffic(), "kernel": "k_field",
                "kernel_ms": field_ms, "gather_ms": gather_ms,
                "algorithmic_mul32_per_pair": mul32_per_pair}
    result = {
        "metric": "particle-ray contributions/s at rel err <=1e-5; p50/p99 frame latency",
        "value": value, "unit": "contributions/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": elapsed / a.steps * 1e3, "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"plain GPU path: {a.particles} clustered particles (16 Gaussians + 10% uniform, "
                               f"h=r32/2, SPH density), Wendland C2, K=4, D=3, tol 1e-3, {a.size}x{a.size} "
                               "perspective rays, render", "pairs_per_frame": pairs_per_frame,
                   "max_hits_per_ray": st["max_hits"],
                   "rays_by_layout": {"lds": st["n_rays"] - st["rays_jumps_device"] - st["rays_scratch_device"]
                                      - st["rays_global"], "jump_rows_in_hbm": st["rays_jumps_device"],
                                      "jump_rows_and_sort_scratch_in_hbm": st["rays_scratch_device"],
                                      "all_in_hbm": st["rays_global"]},
                   "tau": info["tau"], "sigma": info["sigma"], "index_build_s": index_s, "generate_s": gen_s},
        "roofline": roofline,
    }
    # the same frame's rays through sph_hoa_approx_rays (merged fields, no classification), after
    # the timed region: pixel-centre rays of the camera, arbitrary-ray gathering
    ro, rv = camera_rays(cam, torch)
    warm = L.sph_hoa_approx_rays(idx, ro, rv, cam["t_min"], cam["t_max"])
    cap = int(warm["n_pieces"]) + 1024  # output sized once, as a caller reusing buffers would
    del warm
    # warm-up calls while the library's tuner times its field kernel configurations (one call each)
    for _ in range(6):
        L.sph_hoa_approx_rays(idx, ro, rv, cam["t_min"], cam["t_max"], capacity=cap)
    torch.cuda.synchronize()
    alat = []
    for _ in range(3):
        ts = time.perf_counter()
        ap = L.sph_hoa_approx_rays(idx, ro, rv, cam["t_min"], cam["t_max"], capacity=cap)
        torch.cuda.synchronize()
        alat.append(time.perf_counter() - ts)
    result["config"]["approx_rays_p50_ms"] = float(np.median(alat) * 1e3)
    result["config"]["approx_rays_contributions_per_s"] = ap["n_pairs"] / float(np.median(alat))
    result["config"]["approx_rays_pieces"] = int(ap["n_pieces"])
    del ap, ro, rv
    img = out.cpu().numpy().reshape(-1, 4)
    if not a.no_cpu:
        result["cpu_baseline"], result["parity"] = parity_leg(a, L, idx, xyz, h, val, info, cam, tf, vmin, vmax, step,
                                                              kind, K, D, tol, img)
    print(json.dumps(result), flush=True)


def parity_leg(a, L, idx, xyz, h, val, info, cam, tf, vmin, vmax, step, kind, K, D, tol, img):
    """Parity of the timed frame on the seeded 1 % ray subsample (2,621 pixel rays), and the oracle's
    throughput on those rays as the CPU baseline.  Per ray: the render's hit set (sph_hoa_camera_hits)
    equals the oracle's brute-force set; the render's merged partition (sph_hoa_approx_camera) is
    valid by the oracle's checker with its float32 coefficients, evaluated on the library's own
    float32 ends, within 1e-5 of the ray peak of the projections; the pixel is within 1e-4 of the
    oracle's compositing of those projections.  The oracle runs with the library's quanta, whose
    agreement with the oracle's own is reported."""
    from oracle import geometry, grid, quanta
    from tests import gpu_helpers as H

    am = grid.a_max(kind, xyz, h, val)
    hr, pr = grid.representatives(h, val)
    tau_o, sigma_o = quanta.choose_quanta(kind, D, am, hr, pr)
    sc = H.Scene(kind, K, D, 4096, xyz, h, val, tol,
                 quanta=(info["a_max"], info["h_repr"], info["phi_repr"], info["tau"], info["sigma"]))
    oo, vv = geometry.camera_rays(cam)
    sample = np.sort(np.random.default_rng(2621).choice(len(oo), size=min(a.parity_rays, len(oo)), replace=False))
    fo = L.sph_hoa_approx_camera(idx, cam)
    hout = H.host_out(fo)
    del fo
    offs, ids = L.sph_hoa_camera_hits(idx, cam)
    hits = H.hit_lists(offs, ids, sample)
    del offs, ids
    tf64 = tf.astype(np.float64)
    tasks = []
    for r in sample:
        r = int(r)
        g = H.ray_data(hout, r)
        g["hits"] = hits[r]
        tasks.append((r, oo[r], vv[r], float(cam["t_min"]), float(cam["t_max"]), g,
                      {"pixel": (img[r], float(cam["t_min"]), float(cam["t_max"]), tf64, vmin, vmax, step)}))
    del hout
    workers = H.pool_workers()
    t0 = time.perf_counter()
    last = [t0]

    def progress(done):
        now = time.perf_counter()
        if now - last[0] > 20.0 or done == len(tasks):
            last[0] = now
            print(f"parity: {done}/{len(tasks)} rays checked ({now - t0:.0f} s)", file=sys.stderr, flush=True)

    res = H.compare_rays_parallel(sc, tasks, workers=workers, progress=progress)
    elapsed = time.perf_counter() - t0
    s = H.summarize(res)
    n_hits = sum(st.get("hits", 0) for _, st in res.values())
    cpu = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = os.cpu_count() or 1
    base = {"value": n_hits / elapsed, "unit": "contributions/s", "cores": workers, "kind": "oracle",
            "nproc": nproc,
            "sample": f"the seeded 1% subsample of the same 512x512 frame ({len(res)} pixel rays, {n_hits} "
                      f"contributions): FP64 oracle with Python-integer accumulation plus the parity checks, "
                      f"{workers} worker processes (the host share of one GPU; nproc {nproc}) on {cpu}, "
                      f"{elapsed:.1f} s wall"}
    parity = {"rays": len(res), "rays_failed": len(s["bad"]),
              "failures": {str(r): e[:2] for r, e in list(s["bad"].items())[:5]},
              "hit_sets": "bit-exact" if not any("hit set" in x for e in s["bad"].values() for x in e) else "differ",
              "field_max_coef_err_rel_peak": s["max_coef_err"], "field_tol": 1e-5,
              "max_abs_rgba": s["max_pixel_diff"], "rgba_tol": 1e-4,
              "merged_pieces_library": s["pieces_library"], "merged_pieces_plain_greedy": s["pieces_plain_greedy"],
              "quanta_rel_diff": {"tau": abs(info["tau"] / tau_o - 1), "sigma": abs(info["sigma"] / sigma_o - 1)}}
    return base, parity


if __name__ == "__main__":
    main()
