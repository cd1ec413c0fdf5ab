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
    ap.add_argument("--rate", type=float, default=20.0, help="serve workload: Poisson arrival rate (requests/s)")
    ap.add_argument("--duration", type=float, default=8.0, help="serve workload: seconds of arrivals")
    ap.add_argument("--sides", default="64,128,256", help="serve workload: image sides (uniform choice)")
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
    ap.add_argument("--batch-cams", type=int, default=64, help="cameras per batch (batch workload)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="instead of the benchmark, run 5 plain device copies of MIB MiB each (the "
                         "reference kernel for scaling the HBM byte counters) and exit")
    return ap.parse_args()


def run_batch(a, torch, L, synth):
    """Batch workload: a.batch_cams camera bundles (square, side 32..512 log-uniform, eyes on the
    radius-2 sphere about the cube centre, half of them narrow views through cluster cores) over
    a clustered set of a.particles particles (default 2M), Wendland C2, K = 4, D = 3; one step =
    one sph_hoa_render_batch call for all cameras.  Also times the same cameras rendered one
    sph_hoa_render call each."""
    n = a.particles if a.particles != 1_000_000 else 2_000_000
    xyz, h, val = synth.clustered_particles(seed=2, n=n)
    cams = synth.batch_cameras(seed=4, n=a.batch_cams, centres=synth.cluster_centres(seed=2))
    tf = synth.transfer_function()
    vmin, vmax, step = 0.0, 300.0, 2.0 / 512
    idx = L.sph_hoa_build_index(xyz, h, val, kernel=L.KERNEL_WENDLAND_C2, degree=3, pieces=4, lut_entries=4096,
                                merge_tol=1e-3)
    n_rays = sum(c["width"] * c["height"] for c in cams)
    out = torch.empty((n_rays, 4), dtype=torch.float32, device="cuda")
    for _ in range(a.warmup):
        L.sph_hoa_render_batch(idx, cams, tf, vmin, vmax, step, out=out)
    torch.cuda.synchronize()
    idx.set_timing(True)
    lat, pairs = [], 0
    t0 = time.perf_counter()
    for _ in range(a.steps):
        ts = time.perf_counter()
        L.sph_hoa_render_batch(idx, cams, tf, vmin, vmax, step, out=out)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        pairs += idx.stats()["n_pairs"]
    elapsed = time.perf_counter() - t0
    st = idx.stats()
    idx.set_timing(False)
    # the same cameras one call each (one pass, after a warm-up pass)
    for c in cams:
        L.sph_hoa_render(idx, c, tf, vmin, vmax, step)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    sep_pairs = 0
    for c in cams:
        L.sph_hoa_render(idx, c, tf, vmin, vmax, step)
        sep_pairs += idx.stats()["n_pairs"]
    torch.cuda.synchronize()
    sep = time.perf_counter() - ts
    lat_ms = np.array(lat) * 1e3
    result = {
        "metric": "particle-ray contributions/s at rel err <=1e-5; p50/p99 frame latency",
        "value": pairs / elapsed, "unit": "contributions/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": elapsed / a.steps * 1e3, "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"batch: {len(cams)} camera bundles (32^2..512^2, half through cluster cores) over "
                               f"{n} clustered particles, Wendland C2, K=4, D=3, tol 1e-3, one render_batch call",
                   "rays_per_batch": n_rays, "pairs_per_batch": st["n_pairs"], "max_hits_per_ray": st["max_hits"],
                   "field_ms": st["ms_field"] / max(1, st["timed_calls"]),
                   "gather_ms": st["ms_gather"] / max(1, st["timed_calls"]),
                   "rays_by_layout": {"jump_rows_in_hbm": st["rays_jumps_device"],
                                      "jump_rows_and_sort_scratch_in_hbm": st["rays_scratch_device"],
                                      "all_in_hbm": st["rays_global"]},
                   "separate_calls_s": sep, "separate_calls_contributions_per_s": sep_pairs / sep,
                   "batch_speedup_vs_separate_calls": sep / (elapsed / a.steps)},
    }
    print(json.dumps(result), flush=True)


def run_serve(a, torch, L, synth):
    """Serving workload: render requests arrive as a Poisson stream (a.rate per second for
    a.duration seconds) at the native render server holding a resident clustered set (default 2M
    particles, Wendland C2, K = 4, D = 3); each request is one camera on the radius-2 sphere (half
    of them narrow views through cluster cores) with a square image of a side drawn from a.sides.
    Reports latency (submit to completion) and the sustained contribution rate."""
    import threading

    n = a.particles if a.particles != 1_000_000 else 2_000_000
    xyz, h, val = synth.clustered_particles(seed=2, n=n)
    idx = L.sph_hoa_build_index(xyz, h, val, kernel=L.KERNEL_WENDLAND_C2, degree=3, pieces=4, lut_entries=4096,
                                merge_tol=1e-3)
    tf = torch.as_tensor(synth.transfer_function(), device="cuda")
    rng = np.random.default_rng(5)
    sides = [int(x) for x in a.sides.split(",")]
    n_req = int(rng.poisson(a.rate * a.duration))
    arrivals = np.sort(rng.uniform(0.0, a.duration, n_req))
    cams = synth.batch_cameras(seed=5, n=n_req, centres=synth.cluster_centres(seed=2))
    for c in cams:
        side = int(sides[int(rng.integers(len(sides)))])
        c["width"] = c["height"] = side
    srv = L.Server(hbm_budget_bytes=32 << 30)
    slot = srv.add_index(idx)
    # warm-up: one request of each size, not counted
    for sd in sides:
        rid, _ = srv.submit(slot, dict(cams[0], width=sd, height=sd), tf, 0.0, 300.0, 2.0 / 512)
        srv.wait(rid)
    st0 = srv.stats()
    ids = []
    t0 = time.perf_counter()
    for i, c in enumerate(cams):
        dt = arrivals[i] - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        ids.append(srv.submit(slot, c, tf, 0.0, 300.0, 2.0 / 512)[0])
    lat = [srv.wait(rid)[1] for rid in ids]
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    lat = np.array(lat)
    pairs = st["n_pairs"] - st0["n_pairs"]
    batches = st["batches"] - st0["batches"]
    result = {
        "metric": "particle-ray contributions/s at rel err <=1e-5; p50/p99 frame latency",
        "value": pairs / wall, "unit": "contributions/s", "n_gpus": 1, "steps": n_req, "warmup": len(sides),
        "ms_per_step": wall / max(1, n_req) * 1e3, "p50_ms": float(np.percentile(lat, 50)) if n_req else None,
        "p99_ms": float(np.percentile(lat, 99)) if n_req else None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"serve: Poisson requests at {a.rate}/s for {a.duration} s, sides {sides}, resident "
                               f"{n} clustered particles, Wendland C2, K=4, D=3, tol 1e-3, native render server",
                   "requests": n_req, "batches": batches, "mean_requests_per_batch": n_req / max(1, batches),
                   "offered_rays_per_s": sum(c["width"] * c["height"] for c in cams) / a.duration,
                   "served_rays": st["n_rays"] - st0["n_rays"], "pairs": pairs, "wall_s": wall,
                   "worker_busy_s": st["busy_s"] - st0["busy_s"], "max_latency_ms": float(lat.max()) if n_req else None},
    }
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
    """Table storage precision: the plain frame (1M clustered particles, Wendland C2, K = 4, D = 3,
    tol 1e-3, 512^2) rendered with the float table of Sec. 3.1 stored in fp64, fp32, bf16 and fp16.
    Reports the frame time of each and its pixel differences, against the fp64-table frame and
    against the float64 oracle on a bounded sample of rays.  value = contributions/s with the
    bf16 table."""
    xyz, h, val = synth.clustered_particles(n=a.particles)
    kind, K, D, tol = "wendland", 4, 3, 1e-3
    cam = synth.plain_camera(a.size, a.size)
    tf = synth.transfer_function()
    vmin, vmax, step = 0.0, 300.0, 2.0 / 512
    res, imgs = {}, {}
    for fmt in ("fp64", "fp32", "bf16", "fp16"):
        idx = L.sph_hoa_build_index(xyz, h, val, kernel=L.KERNEL_WENDLAND_C2, degree=D, pieces=K, lut_entries=4096,
                                    merge_tol=tol, lut_precision=fmt)
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
        imgs[fmt] = out.reshape(-1, 4).cpu().numpy().astype(np.float64)
        res[fmt] = {"p50_ms": float(np.percentile(np.array(lat) * 1e3, 50)),
                    "contributions_per_s": pairs / sum(lat)}
        if fmt == "fp64":
            info = idx.info()
        idx.free()
    for fmt in ("fp32", "bf16", "fp16"):
        d = np.abs(imgs[fmt] - imgs["fp64"])
        res[fmt]["max_abs_rgba_vs_fp64_table"] = float(d.max())
        res[fmt]["mean_abs_rgba_vs_fp64_table"] = float(d.mean())
    oracle = None
    result = {
        "metric": "particle-ray contributions/s with the bf16 table; pixel error vs fp64 table and oracle",
        "value": res["bf16"]["contributions_per_s"], "unit": "contributions/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": res["bf16"]["p50_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"precision: plain frame ({a.particles} clustered particles, Wendland C2, K=4, D=3, "
                               f"tol 1e-3, {a.size}x{a.size}) with the table stored in fp64 / fp32 / bf16 / fp16",
                   "by_table_precision": res, "oracle_sample": oracle},
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
    Wendland C2, K = 4, D = 3, tol 1e-3, 512^2 rays), the value field and the four fields of the
    transverse kernel -w'/r with particle values c/h^2 and c chi_a/h^2, from which every gradient
    component along a ray is assembled ((v.e) F' - alpha G_0 - beta.(G_x, G_y, G_z)), all five by one
    sph_hoa_approx_rays_shared call (the hits gathered once) with merged output.  A step is all five
    fields of all rays; the same fields by five separate calls are timed after the timed region.
    value = contributions/s over the five fields."""
    xyz, h, val = synth.clustered_particles(n=a.particles)
    K, D, tol = 4, 3, 1e-3
    cam = synth.plain_camera(a.size, a.size)
    ro, rv = camera_rays(cam, torch)
    c = val.astype(np.float64) / (h.astype(np.float64) ** 2)
    gvals = [c.astype(np.float32)] + [(c * xyz[:, k].astype(np.float64)).astype(np.float32) for k in range(3)]
    t_idx = time.time()
    idxs = [L.sph_hoa_build_index(xyz, h, val, kernel=L.KERNEL_WENDLAND_C2, degree=D, pieces=K, lut_entries=4096,
                                  merge_tol=tol)]
    idxs += [L.sph_hoa_build_index(xyz, h, g, kernel=L.KERNEL_WENDLAND_C2_GRAD, degree=D, pieces=K,
                                   lut_entries=4096, merge_tol=tol) for g in gvals]
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
    # the same five fields by separate calls (each gathers its own hits), after the timed region
    sep = []
    for _ in range(2):
        ts = time.perf_counter()
        for idx in idxs:
            L.sph_hoa_approx_rays(idx, ro, rv, cam["t_min"], cam["t_max"], capacity=cap)
        torch.cuda.synchronize()
        sep.append(time.perf_counter() - ts)
    names = ["value F", "G_0 (c/h^2)", "G_x (c chi_x/h^2)", "G_y (c chi_y/h^2)", "G_z (c chi_z/h^2)"]
    result = {
        "metric": "particle-ray contributions/s over the value field and the four transverse gradient fields",
        "value": pairs / sum(lat), "unit": "contributions/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": float(np.median(lat) * 1e3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"gradient: {a.size}x{a.size} pixel-centre rays of the plain camera, {a.particles} "
                               "clustered particles, Wendland C2 and its transverse kernel -w'/r, K=4, D=3, "
                               "tol 1e-3, five fields per step through sph_hoa_approx_rays_shared (one gathering)",
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
