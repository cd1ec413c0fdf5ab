"""Python binding of libsph_hoa (include/sph_hoa.h): argument marshalling only.

Every step of the path runs in the HIP library; this module converts torch
tensors on the ROCm device into the pointers and structs of the C ABI and
raises ``SphHoaError`` on any non-OK status.  If the library has not been
built (``python -m paper_2401_02896_amd.build``), importing the binding
functions raises immediately: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph_hoa.so")

KERNEL_CUBIC = 0
KERNEL_WENDLAND_C2 = 1
KERNEL_WENDLAND_C4 = 2
KERNEL_WENDLAND_C6 = 3
# transverse gradient kernels g = -w'/r of the Wendland kernels (gradient fields, Sec. 6)
KERNEL_WENDLAND_C2_GRAD = 4
KERNEL_WENDLAND_C4_GRAD = 5
KERNEL_WENDLAND_C6_GRAD = 6
FLAG_EXACT = 1
FLAG_LUT_FP32 = 2
FLAG_LUT_BF16 = 4
FLAG_LUT_FP16 = 8
FLAG_TRANSVERSE_X = 16
FLAG_TRANSVERSE_Y = 32
FLAG_TRANSVERSE_Z = 64

STATUS = {0: "OK", 1: "E_INVALID_ARG", 2: "E_OUT_OF_MEMORY", 3: "E_OVERFLOW", 4: "E_DEVICE", 5: "E_UNSUPPORTED",
          6: "E_INTERNAL", 7: "E_BUSY", 8: "E_CANCELLED"}


class SphHoaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int32), ("pieces", ctypes.c_int32), ("lut_entries", ctypes.c_int32),
                ("int_bits", ctypes.c_int32), ("merge_tol", ctypes.c_double), ("a_max", ctypes.c_double),
                ("h_repr", ctypes.c_double), ("phi_repr", ctypes.c_double), ("tau", ctypes.c_double),
                ("knot_table", ctypes.POINTER(ctypes.c_double)), ("flags", ctypes.c_uint32),
                ("jump_table", ctypes.POINTER(ctypes.c_double)), ("jump_table_mid", ctypes.POINTER(ctypes.c_double))]


class IndexInfo(ctypes.Structure):
    _fields_ = [("n_particles", ctypes.c_int64), ("kernel", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("pieces", ctypes.c_int32), ("lut_entries", ctypes.c_int32), ("tau", ctypes.c_double),
                ("sigma", ctypes.c_double), ("a_max", ctypes.c_double), ("h_repr", ctypes.c_double),
                ("phi_repr", ctypes.c_double), ("grid_lo", ctypes.c_double * 3), ("cell0", ctypes.c_double),
                ("n_levels", ctypes.c_int32), ("level_dims", (ctypes.c_int32 * 3) * 32),
                ("lut_flags", ctypes.c_uint32)]


class FloatField(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int64), ("ray_offsets", ctypes.c_void_p), ("ray_counts", ctypes.c_void_p),
                ("t_start", ctypes.c_void_p), ("t_end", ctypes.c_void_p), ("coef", ctypes.c_void_p),
                ("n_slots", ctypes.c_int64), ("n_pairs", ctypes.c_int64)]


class Rays(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("origin", ctypes.c_void_p), ("dir", ctypes.c_void_p),
                ("t_min", ctypes.c_float), ("t_max", ctypes.c_float)]


class Field(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int64), ("ray_offsets", ctypes.c_void_p), ("t_start", ctypes.c_void_p),
                ("t_end", ctypes.c_void_p), ("coef", ctypes.c_void_p), ("ray_peak", ctypes.c_void_p),
                ("n_pieces", ctypes.c_int64), ("n_pairs", ctypes.c_int64), ("n_knots", ctypes.c_int64),
                ("n_exact_pieces", ctypes.c_int64), ("exact_capacity", ctypes.c_int64),
                ("exact_offsets", ctypes.c_void_p), ("exact_t", ctypes.c_void_p), ("exact_end", ctypes.c_void_p),
                ("exact_coef", ctypes.c_void_p), ("knot_capacity", ctypes.c_int64), ("knot_offsets", ctypes.c_void_p),
                ("knot_t", ctypes.c_void_p), ("knot_pid", ctypes.c_void_p), ("knot_kidx", ctypes.c_void_p)]


class Camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_float * 3), ("look_at", ctypes.c_float * 3), ("up", ctypes.c_float * 3),
                ("fov_y_deg", ctypes.c_float), ("ortho", ctypes.c_int32), ("ortho_half_extent", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("t_min", ctypes.c_float),
                ("t_max", ctypes.c_float)]


class TF(ctypes.Structure):
    _fields_ = [("rgba", ctypes.c_void_p), ("n", ctypes.c_int32), ("v_min", ctypes.c_float), ("v_max", ctypes.c_float),
                ("step", ctypes.c_float)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("failed", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("n_rays", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
                ("busy_s", ctypes.c_double), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("rejected", ctypes.c_int64), ("cancelled", ctypes.c_int64),
                ("lanes", ctypes.c_int64), ("overlapped_batches", ctypes.c_int64), ("max_in_flight", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("n_rays", ctypes.c_int64), ("n_pairs", ctypes.c_int64), ("n_knots", ctypes.c_int64),
                ("n_pieces", ctypes.c_int64), ("max_hits", ctypes.c_int64), ("rays_global", ctypes.c_int64),
                ("rays_jumps_device", ctypes.c_int64), ("rays_scratch_device", ctypes.c_int64),
                ("timed_calls", ctypes.c_int64), ("ms_gather", ctypes.c_double), ("ms_field", ctypes.c_double)]


EXPORTS = ["sph_hoa_build_index", "sph_hoa_approx_rays", "sph_hoa_approx_rays_shared", "sph_hoa_approx_camera",
           "sph_hoa_camera_hits", "sph_hoa_ray_hits", "sph_hoa_render", "sph_hoa_render_static", "sph_hoa_render_batch",
           "sph_hoa_server_create", "sph_hoa_server_create_lanes", "sph_hoa_server_add_index", "sph_hoa_server_submit", "sph_hoa_server_wait",
           "sph_hoa_server_get_stats", "sph_hoa_server_destroy", "sph_hoa_server_set_admission",
           "sph_hoa_server_cancel", "sph_hoa_server_pause", "sph_hoa_accumulate_bits", "sph_hoa_float_rays",
           "sph_hoa_index_free",
           "sph_hoa_index_get_info", "sph_hoa_index_get_lut", "sph_hoa_index_get_grid", "sph_hoa_index_get_stats",
           "sph_hoa_index_set_timing",
           "sph_hoa_optimal_knots", "sph_hoa_knot_table", "sph_hoa_lut_coefficients", "sph_hoa_lut_project",
           "sph_hoa_optimal_tau", "sph_hoa_status_string", "sph_hoa_last_error"]

_lib = None


def lib():
    """The loaded library (loads it on first use; raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2401_02896_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
    L.sph_hoa_build_index.argtypes = [vp, vp, vp, i64, ctypes.c_int, ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]
    L.sph_hoa_approx_rays.argtypes = [vp, ctypes.POINTER(Rays), ctypes.POINTER(Field), u32, vp]
    L.sph_hoa_approx_rays_shared.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(Rays), ctypes.POINTER(Field),
                                             u32, vp]
    L.sph_hoa_approx_camera.argtypes = [vp, ctypes.POINTER(Camera), ctypes.POINTER(Field), u32, vp]
    L.sph_hoa_camera_hits.argtypes = [vp, ctypes.POINTER(Camera), vp, vp, i64, ctypes.POINTER(i64), vp]
    L.sph_hoa_ray_hits.argtypes = [vp, ctypes.POINTER(Rays), vp, vp, i64, ctypes.POINTER(i64), vp]
    L.sph_hoa_render.argtypes = [vp, ctypes.POINTER(Camera), ctypes.POINTER(TF), vp, vp]
    L.sph_hoa_render_static.argtypes = [vp, ctypes.POINTER(Camera), ctypes.POINTER(TF), vp, vp]
    L.sph_hoa_static_scratch_bytes.argtypes = []
    L.sph_hoa_static_scratch_bytes.restype = i64
    L.sph_hoa_device_alloc_count.argtypes = []
    L.sph_hoa_device_alloc_count.restype = i64
    L.sph_hoa_render_batch.argtypes = [vp, ctypes.POINTER(Camera), i32, ctypes.POINTER(TF), vp, vp]
    L.sph_hoa_server_create.argtypes = [i64, i64, ctypes.POINTER(vp)]
    L.sph_hoa_server_create_lanes.argtypes = [i64, i64, i32, ctypes.POINTER(vp)]
    L.sph_hoa_server_add_index.argtypes = [vp, vp, ctypes.POINTER(i32)]
    L.sph_hoa_server_submit.argtypes = [vp, i32, ctypes.POINTER(Camera), ctypes.POINTER(TF), vp,
                                        ctypes.POINTER(i64)]
    L.sph_hoa_server_wait.argtypes = [vp, i64, dbl, ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    L.sph_hoa_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.sph_hoa_server_destroy.argtypes = [vp]
    L.sph_hoa_server_set_admission.argtypes = [vp, i64, i64]
    L.sph_hoa_server_cancel.argtypes = [vp, i64, ctypes.POINTER(i32)]
    L.sph_hoa_server_pause.argtypes = [vp, i32]
    L.sph_hoa_float_rays.argtypes = [vp, ctypes.POINTER(Rays), i32, ctypes.POINTER(FloatField), vp]
    L.sph_hoa_accumulate_bits.argtypes = [i32, i32, vp, vp, i32, i64, i32, vp, ctypes.POINTER(ctypes.c_float), vp]
    L.sph_hoa_index_free.argtypes = [vp]
    L.sph_hoa_index_get_info.argtypes = [vp, ctypes.POINTER(IndexInfo)]
    L.sph_hoa_index_get_lut.argtypes = [vp, vp, vp, vp]
    L.sph_hoa_index_get_grid.argtypes = [vp, vp, vp, vp, vp]
    L.sph_hoa_index_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.sph_hoa_index_set_timing.argtypes = [vp, i32]
    L.sph_hoa_optimal_knots.argtypes = [ctypes.c_int, i32, i32, dbl, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    L.sph_hoa_knot_table.argtypes = [ctypes.c_int, i32, i32, i32, vp, vp]
    L.sph_hoa_lut_coefficients.argtypes = [ctypes.c_int, i32, i32, i32, vp, vp, vp, vp]
    L.sph_hoa_lut_project.argtypes = [ctypes.c_int, i32, i32, i32, vp, vp, vp, vp, vp]
    L.sph_hoa_optimal_tau.argtypes = [ctypes.c_int, i32, dbl, dbl, dbl, ctypes.POINTER(dbl)]
    L.sph_hoa_status_string.argtypes = [ctypes.c_int]
    L.sph_hoa_status_string.restype = ctypes.c_char_p
    L.sph_hoa_last_error.restype = ctypes.c_char_p
    for name in EXPORTS[:-2]:
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status):
    if status != 0:
        raise SphHoaError(status, lib().sph_hoa_last_error().decode())


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev_f32(a, shape_last=None):
    import torch

    t = a if isinstance(a, torch.Tensor) else torch.as_tensor(a)
    t = t.to(device="cuda", dtype=torch.float32).contiguous()
    return t


class Index:
    """Owns an sph_hoa_index handle (sph_hoa_build_index / sph_hoa_index_free)."""

    def __init__(self, handle, K, D, n):
        self.handle = handle
        self.K, self.D, self.n = K, D, n

    def free(self):
        if self.handle:
            _check(lib().sph_hoa_index_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self):
        inf = IndexInfo()
        _check(lib().sph_hoa_index_get_info(self.handle, ctypes.byref(inf)))
        return {"n_particles": inf.n_particles, "kernel": inf.kernel, "degree": inf.degree, "pieces": inf.pieces,
                "lut_entries": inf.lut_entries, "tau": inf.tau, "sigma": inf.sigma, "a_max": inf.a_max,
                "h_repr": inf.h_repr, "phi_repr": inf.phi_repr, "grid_lo": list(inf.grid_lo), "cell0": inf.cell0,
                "n_levels": inf.n_levels,
                "level_dims": [list(inf.level_dims[l]) for l in range(inf.n_levels)], "lut_flags": inf.lut_flags}

    def lut(self):
        import numpy as np

        inf = self.info()
        n, P, D = inf["lut_entries"], (self.K + 1) // 2, self.D
        theta = np.zeros((n, P))
        shat = np.zeros((n, P, D + 1))
        smid = np.zeros((n, D + 1))
        _check(lib().sph_hoa_index_get_lut(self.handle, theta.ctypes.data_as(ctypes.c_void_p),
                                           shat.ctypes.data_as(ctypes.c_void_p), smid.ctypes.data_as(ctypes.c_void_p)))
        return theta, shat, smid

    def grid(self):
        import torch

        morton = torch.empty(self.n, dtype=torch.int64, device="cuda")
        level = torch.empty(self.n, dtype=torch.int32, device="cuda")
        order = torch.empty(self.n, dtype=torch.int32, device="cuda")
        _check(lib().sph_hoa_index_get_grid(self.handle, _ptr(morton), _ptr(level), _ptr(order), _stream()))
        return morton, level, order

    def set_timing(self, on=True):
        _check(lib().sph_hoa_index_set_timing(self.handle, 1 if on else 0))

    def stats(self):
        s = Stats()
        _check(lib().sph_hoa_index_get_stats(self.handle, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in Stats._fields_}


def sph_hoa_build_index(xyz, h, value, kernel=KERNEL_CUBIC, degree=2, pieces=4, lut_entries=4096, merge_tol=1e-3,
                        a_max=0.0, h_repr=0.0, phi_repr=0.0, tau=0.0, knot_table=None, lut_precision="fp64",
                        jump_table=None, jump_table_mid=None, transverse=None):
    """Build an index (sph_hoa_build_index).  xyz [n,3], h [n], value [n]: tensors or arrays.
    lut_precision: storage precision of the float table, "fp64", "fp32", "bf16" or "fp16".
    jump_table [lut_entries, ceil(K/2), D+1] / jump_table_mid [lut_entries, D+1] (even K): projection
    jumps replacing the library's own (with knot_table).  transverse = 0, 1 or 2: a transverse
    gradient field along that axis (SPH_HOA_FLAG_TRANSVERSE_X/Y/Z)."""
    import numpy as np

    x = _dev_f32(xyz)
    hh = _dev_f32(h)
    v = _dev_f32(value)
    n = int(hh.numel())
    if x.numel() != 3 * n or v.numel() != n:
        raise ValueError("xyz must be [n, 3], h and value [n]")
    flags = {"fp64": 0, "fp32": FLAG_LUT_FP32, "bf16": FLAG_LUT_BF16, "fp16": FLAG_LUT_FP16}.get(lut_precision)
    if flags is None:
        raise ValueError(f"lut_precision must be fp64, fp32, bf16 or fp16, got {lut_precision!r}")
    if transverse is not None:
        flags |= {0: FLAG_TRANSVERSE_X, 1: FLAG_TRANSVERSE_Y, 2: FLAG_TRANSVERSE_Z}[int(transverse)]
    p = Params(degree, pieces, lut_entries, 64, merge_tol, a_max, h_repr, phi_repr, tau, None, flags)
    kt = None
    if knot_table is not None:
        kt = np.ascontiguousarray(knot_table, dtype=np.float64)
        p.knot_table = kt.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    jt = jm = None
    if jump_table is not None:
        jt = np.ascontiguousarray(jump_table, dtype=np.float64)
        p.jump_table = jt.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if jump_table_mid is not None:
        jm = np.ascontiguousarray(jump_table_mid, dtype=np.float64)
        p.jump_table_mid = jm.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    handle = ctypes.c_void_p()
    _check(lib().sph_hoa_build_index(_ptr(x), _ptr(hh), _ptr(v), n, kernel, ctypes.byref(p), _stream(),
                                     ctypes.byref(handle)))
    return Index(handle, pieces, degree, n)


def sph_hoa_float_rays(index, origin, direction, t_min, t_max, n_reinit=0):
    """Float accumulation variant (sph_hoa_float_rays): per-ray pieces of the float32 sweep.

    Returns a dict: ray_offsets [n+1], ray_counts [n], t_start, t_end, coef [slots, D+1] (powers of
    t - t_start), all device tensors over the slot layout, and n_pairs."""
    import torch

    o = _dev_f32(origin).reshape(-1, 3)
    d = _dev_f32(direction).reshape(-1, 3)
    n = o.shape[0]
    D = index.D
    r = Rays(n, _ptr(o).value, _ptr(d).value, t_min, t_max)
    offs = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(max(n, 1), dtype=torch.int64, device="cuda")
    f = FloatField()
    f.capacity = 0
    f.ray_offsets, f.ray_counts = _ptr(offs).value, _ptr(cnt).value
    st = lib().sph_hoa_float_rays(index.handle, ctypes.byref(r), int(n_reinit), ctypes.byref(f), _stream())
    if st == 0 and n == 0:
        return {"ray_offsets": offs, "ray_counts": cnt[:0], "t_start": None, "t_end": None, "coef": None,
                "n_pairs": 0}
    if st != 2:
        _check(st)
    slots = int(f.n_slots)
    t0 = torch.zeros(max(slots, 1), dtype=torch.float32, device="cuda")
    t1 = torch.zeros(max(slots, 1), dtype=torch.float32, device="cuda")
    coef = torch.zeros(max(slots, 1) * (D + 1), dtype=torch.float32, device="cuda")
    f.capacity = slots
    f.t_start, f.t_end, f.coef = _ptr(t0).value, _ptr(t1).value, _ptr(coef).value
    _check(lib().sph_hoa_float_rays(index.handle, ctypes.byref(r), int(n_reinit), ctypes.byref(f), _stream()))
    return {"ray_offsets": offs, "ray_counts": cnt[:n], "t_start": t0[:slots], "t_end": t1[:slots],
            "coef": coef[: slots * (D + 1)].reshape(-1, D + 1), "n_pairs": int(f.n_pairs)}


def _alloc_field(n, D, cap, ecap, exact):
    """Device output tensors of one sph_hoa_field and the struct pointing at them."""
    import torch

    t = {"offs": torch.empty(n + 1, dtype=torch.int64, device="cuda"),
         "t0": torch.empty(max(cap, 1), dtype=torch.float32, device="cuda"),
         "t1": torch.empty(max(cap, 1), dtype=torch.float32, device="cuda"),
         "coef": torch.empty(max(cap, 1) * (D + 1), dtype=torch.float32, device="cuda"),
         "peak": torch.empty(max(n, 1), dtype=torch.float32, device="cuda")}
    f = Field()
    f.capacity = cap
    f.ray_offsets, f.t_start, f.t_end, f.coef, f.ray_peak = (_ptr(t["offs"]).value, _ptr(t["t0"]).value,
                                                             _ptr(t["t1"]).value, _ptr(t["coef"]).value,
                                                             _ptr(t["peak"]).value)
    if exact:
        t["offsets"] = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        t["t"] = torch.empty(max(ecap, 1), dtype=torch.int64, device="cuda")
        t["end"] = torch.empty(max(ecap, 1), dtype=torch.int64, device="cuda")
        t["ecoef"] = torch.empty(max(ecap, 1) * (D + 1), dtype=torch.int64, device="cuda")
        t["knot_offsets"] = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        t["knot_t"] = torch.empty(max(ecap, 1), dtype=torch.int64, device="cuda")
        t["knot_pid"] = torch.empty(max(ecap, 1), dtype=torch.int32, device="cuda")
        t["knot_kidx"] = torch.empty(max(ecap, 1), dtype=torch.int32, device="cuda")
        f.exact_capacity = ecap
        f.exact_offsets, f.exact_t, f.exact_end, f.exact_coef = (_ptr(t["offsets"]).value, _ptr(t["t"]).value,
                                                                 _ptr(t["end"]).value, _ptr(t["ecoef"]).value)
        f.knot_capacity = ecap
        f.knot_offsets, f.knot_t, f.knot_pid, f.knot_kidx = (_ptr(t["knot_offsets"]).value, _ptr(t["knot_t"]).value,
                                                             _ptr(t["knot_pid"]).value, _ptr(t["knot_kidx"]).value)
    return f, t


def _field_result(f, t, n, D, exact):
    out = {"ray_offsets": t["offs"], "t_start": t["t0"][: f.n_pieces], "t_end": t["t1"][: f.n_pieces],
           "coef": t["coef"][: f.n_pieces * (D + 1)].reshape(-1, D + 1), "ray_peak": t["peak"][:n],
           "n_pieces": f.n_pieces, "n_pairs": f.n_pairs, "n_knots": f.n_knots, "n_exact_pieces": f.n_exact_pieces}
    if exact:
        out["exact_offsets"] = t["offsets"]
        out["exact_t"] = t["t"][: f.n_exact_pieces]
        out["exact_end"] = t["end"][: f.n_exact_pieces]
        out["exact_coef"] = t["ecoef"][: f.n_exact_pieces * (D + 1)].reshape(-1, D + 1)
        out["knot_offsets"] = t["knot_offsets"]
        out["knot_t"] = t["knot_t"][: f.n_knots]
        out["knot_pid"] = t["knot_pid"][: f.n_knots]
        out["knot_kidx"] = t["knot_kidx"][: f.n_knots]
    return out


def sph_hoa_approx_rays(index, origin, direction, t_min, t_max, capacity=None, exact=False, exact_capacity=None):
    """Per-ray merged fields (sph_hoa_approx_rays).  Returns a dict of device tensors and counts.

    capacity: pieces to allocate (default: grows and retries once on E_OUT_OF_MEMORY).
    """
    o = _dev_f32(origin).reshape(-1, 3)
    d = _dev_f32(direction).reshape(-1, 3)
    n = o.shape[0]
    D = index.D
    cap = capacity if capacity is not None else max(1024, 64 * n)
    ecap = exact_capacity if exact_capacity is not None else max(1024, 64 * n)
    for attempt in range(2):
        f, t = _alloc_field(n, D, cap, ecap, exact)
        r = Rays(n, _ptr(o).value, _ptr(d).value, t_min, t_max)
        st = lib().sph_hoa_approx_rays(index.handle, ctypes.byref(r), ctypes.byref(f), FLAG_EXACT if exact else 0,
                                       _stream())
        if st == 2 and attempt == 0 and capacity is None:
            cap = max(cap, int(f.n_pieces) + 1)
            ecap = max(ecap, int(f.n_exact_pieces) + 1, int(f.n_knots) + 1)
            continue
        _check(st)
        break
    return _field_result(f, t, n, D, exact)


def sph_hoa_approx_rays_shared(indices, origin, direction, t_min, t_max, capacity=None, exact=False,
                               exact_capacity=None):
    """Fields of several indices of the same particles along the same rays, the hits gathered once
    (sph_hoa_approx_rays_shared).  Returns one dict per index, as sph_hoa_approx_rays.

    capacity: pieces to allocate per field (default: grows on E_OUT_OF_MEMORY and retries)."""
    o = _dev_f32(origin).reshape(-1, 3)
    d = _dev_f32(direction).reshape(-1, 3)
    n = o.shape[0]
    k = len(indices)
    caps = [capacity if capacity is not None else max(1024, 64 * n)] * k
    ecaps = [exact_capacity if exact_capacity is not None else max(1024, 64 * n)] * k
    for attempt in range(k + 1):
        allocs = [_alloc_field(n, ix.D, caps[i], ecaps[i], exact) for i, ix in enumerate(indices)]
        fields = (Field * k)(*[f for f, _ in allocs])
        handles = (ctypes.c_void_p * k)(*[ix.handle.value if isinstance(ix.handle, ctypes.c_void_p) else ix.handle
                                          for ix in indices])
        r = Rays(n, _ptr(o).value, _ptr(d).value, t_min, t_max)
        st = lib().sph_hoa_approx_rays_shared(handles, k, ctypes.byref(r), fields, FLAG_EXACT if exact else 0,
                                              _stream())
        if st == 2 and capacity is None and attempt < k:
            # the call stops at the first field that does not fit; the fields after it have not run,
            # so they get at least the same capacity (fields of the same rays are of similar size)
            grown = False
            for i in range(k):
                if fields[i].n_pieces > caps[i] or (exact and (fields[i].n_exact_pieces > ecaps[i]
                                                               or fields[i].n_knots > ecaps[i])):
                    caps[i] = max(caps[i], int(fields[i].n_pieces) + 1)
                    ecaps[i] = max(ecaps[i], int(fields[i].n_exact_pieces) + 1, int(fields[i].n_knots) + 1)
                    for j in range(i + 1, k):
                        caps[j] = max(caps[j], caps[i] + caps[i] // 8)
                        ecaps[j] = max(ecaps[j], ecaps[i] + ecaps[i] // 8)
                    grown = True
                    break
            if grown:
                continue
        _check(st)
        break
    return [_field_result(fields[i], allocs[i][1], n, ix.D, exact) for i, ix in enumerate(indices)]


def make_camera(cam: dict) -> Camera:
    c = Camera()
    c.eye[:] = [float(x) for x in cam["eye"]]
    c.look_at[:] = [float(x) for x in cam["look_at"]]
    c.up[:] = [float(x) for x in cam["up"]]
    c.fov_y_deg = float(cam.get("fov_y_deg", 0.0))
    c.ortho = int(cam.get("ortho", 0))
    c.ortho_half_extent = float(cam.get("ortho_half_extent", 0.0))
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.t_min, c.t_max = float(cam["t_min"]), float(cam["t_max"])
    return c


def sph_hoa_approx_camera(index, camera: dict, capacity=None, exact=False, exact_capacity=None):
    """Fields along a camera's pixel rays with the render's gathering (sph_hoa_approx_camera);
    returns the dict of sph_hoa_approx_rays (capacity: as there)."""
    c = make_camera(camera)
    n = c.width * c.height
    D = index.D
    cap = capacity if capacity is not None else max(1024, 64 * n)
    ecap = exact_capacity if exact_capacity is not None else max(1024, 64 * n)
    for attempt in range(2):
        f, t = _alloc_field(n, D, cap, ecap, exact)
        st = lib().sph_hoa_approx_camera(index.handle, ctypes.byref(c), ctypes.byref(f), FLAG_EXACT if exact else 0,
                                         _stream())
        if st == 2 and attempt == 0 and capacity is None:
            cap = max(cap, int(f.n_pieces) + 1)
            ecap = max(ecap, int(f.n_exact_pieces) + 1, int(f.n_knots) + 1)
            continue
        _check(st)
        break
    return _field_result(f, t, n, D, exact)


def _hits(call, n, capacity):
    import torch

    offs = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    cap = capacity if capacity is not None else max(1024, 256 * n)
    for attempt in range(2):
        ids = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
        npairs = ctypes.c_int64(0)
        st = call(_ptr(offs), _ptr(ids), cap, ctypes.byref(npairs))
        if st == 2 and attempt == 0 and capacity is None and npairs.value > cap:
            cap = int(npairs.value)
            continue
        _check(st)
        break
    return offs, ids[: npairs.value]


def sph_hoa_camera_hits(index, camera: dict, capacity=None):
    """Hit lists of a camera's pixel rays as the render gathers them (sph_hoa_camera_hits): returns
    (offsets [n + 1] int64, ids [pairs] int32 input indices), device tensors; each ray's ids are in
    an unspecified order."""
    c = make_camera(camera)
    return _hits(lambda o, i, cap, npr: lib().sph_hoa_camera_hits(index.handle, ctypes.byref(c), o, i, cap, npr,
                                                                  _stream()), c.width * c.height, capacity)


def sph_hoa_ray_hits(index, origin, direction, t_min, t_max, capacity=None):
    """Hit lists of arbitrary rays as sph_hoa_approx_rays gathers them (sph_hoa_ray_hits)."""
    o = _dev_f32(origin).reshape(-1, 3)
    d = _dev_f32(direction).reshape(-1, 3)
    n = o.shape[0]
    r = Rays(n, _ptr(o).value, _ptr(d).value, t_min, t_max)
    return _hits(lambda op, i, cap, npr: lib().sph_hoa_ray_hits(index.handle, ctypes.byref(r), op, i, cap, npr,
                                                                _stream()), n, capacity)


def sph_hoa_render(index, camera: dict, tf_rgba, v_min, v_max, step, out=None):
    """Render an image (sph_hoa_render); returns a [height, width, 4] float32 device tensor."""
    import torch

    c = make_camera(camera)
    tf = _dev_f32(tf_rgba).reshape(-1, 4)
    if out is None:
        out = torch.empty((c.height, c.width, 4), dtype=torch.float32, device="cuda")
    t = TF(_ptr(tf).value, tf.shape[0], v_min, v_max, step)
    _check(lib().sph_hoa_render(index.handle, ctypes.byref(c), ctypes.byref(t), _ptr(out), _stream()))
    return out


def sph_hoa_render_static(index, camera: dict, tf_rgba, v_min, v_max, step, out=None):
    """sph_hoa_render with every per-call buffer in the library's fixed static device scratch (no
    allocation inside the call; `out` may be preallocated)."""
    import torch

    c = make_camera(camera)
    tf = _dev_f32(tf_rgba).reshape(-1, 4)
    if out is None:
        out = torch.empty((c.height, c.width, 4), dtype=torch.float32, device="cuda")
    t = TF(_ptr(tf).value, tf.shape[0], v_min, v_max, step)
    _check(lib().sph_hoa_render_static(index.handle, ctypes.byref(c), ctypes.byref(t), _ptr(out), _stream()))
    return out


def sph_hoa_static_scratch_bytes():
    """Size of the fixed static scratch array of sph_hoa_render_static (bytes)."""
    return int(lib().sph_hoa_static_scratch_bytes())


def sph_hoa_device_alloc_count():
    """Device allocations the library has made in this process so far."""
    return int(lib().sph_hoa_device_alloc_count())


def sph_hoa_render_batch(index, cameras, tf_rgba, v_min, v_max, step, out=None):
    """Render a batch of cameras in one launch chain (sph_hoa_render_batch).  Returns the flat
    float32 device tensor of all images (camera order) and the list of [height, width, 4] views."""
    import torch

    cs = (Camera * max(1, len(cameras)))()
    sizes = []
    for i, cam in enumerate(cameras):
        cs[i] = make_camera(cam)
        sizes.append((cs[i].height, cs[i].width))
    n = sum(h * w for h, w in sizes)
    tf = _dev_f32(tf_rgba).reshape(-1, 4)
    if out is None:
        out = torch.empty((max(1, n), 4), dtype=torch.float32, device="cuda")
    t = TF(_ptr(tf).value, tf.shape[0], v_min, v_max, step)
    _check(lib().sph_hoa_render_batch(index.handle, cs, len(cameras), ctypes.byref(t), _ptr(out), _stream()))
    views, o = [], 0
    for h, w in sizes:
        views.append(out[o:o + h * w].view(h, w, 4))
        o += h * w
    return out, views


class Server:
    """Render server (sph_hoa_server_*): resident indices, a request queue and continuous batching
    by native worker lanes (each with its own stream).  submit() returns a request id; wait() blocks
    until the image is in the output tensor."""

    def __init__(self, hbm_budget_bytes=8 << 30, max_batch_rays=1 << 24, lanes=2):
        h = ctypes.c_void_p()
        _check(lib().sph_hoa_server_create_lanes(int(hbm_budget_bytes), int(max_batch_rays), int(lanes),
                                                 ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def add_index(self, index):
        slot = ctypes.c_int32()
        _check(lib().sph_hoa_server_add_index(self.handle, index.handle, ctypes.byref(slot)))
        self._keep[("index", slot.value)] = index
        return slot.value

    def submit(self, slot, camera: dict, tf_rgba, v_min, v_max, step, out=None):
        import torch

        c = make_camera(camera)
        tf = _dev_f32(tf_rgba).reshape(-1, 4)
        if out is None:
            out = torch.empty((c.height, c.width, 4), dtype=torch.float32, device="cuda")
        # inputs written on torch's stream must be complete before the server's stream reads them
        torch.cuda.current_stream().synchronize()
        t = TF(_ptr(tf).value, tf.shape[0], v_min, v_max, step)
        rid = ctypes.c_int64()
        _check(lib().sph_hoa_server_submit(self.handle, slot, ctypes.byref(c), ctypes.byref(t), _ptr(out),
                                           ctypes.byref(rid)))
        self._keep[rid.value] = (tf, out)
        return rid.value, out

    def wait(self, request_id, timeout_s=-1.0):
        """(done, latency_ms); raises SphHoaError if the request failed."""
        done = ctypes.c_int32()
        lat = ctypes.c_double()
        try:
            _check(lib().sph_hoa_server_wait(self.handle, int(request_id), float(timeout_s), ctypes.byref(done),
                                             ctypes.byref(lat)))
        finally:
            if done.value:
                self._keep.pop(request_id, None)
        return bool(done.value), lat.value

    def set_admission(self, max_queued=0, max_request_bytes=0):
        """Refuse submissions when max_queued requests wait (E_BUSY) or when one request alone
        would need more than max_request_bytes of device memory (E_OUT_OF_MEMORY); 0: no limit."""
        _check(lib().sph_hoa_server_set_admission(self.handle, int(max_queued), int(max_request_bytes)))

    def pause(self, paused=True):
        """Stop (True) or resume (False) the worker taking new batches; submissions still queue."""
        _check(lib().sph_hoa_server_pause(self.handle, 1 if paused else 0))

    def cancel(self, request_id):
        """True if the request was still queued and is now cancelled (its wait raises
        E_CANCELLED); False if it already ran or is running."""
        c = ctypes.c_int32()
        _check(lib().sph_hoa_server_cancel(self.handle, int(request_id), ctypes.byref(c)))
        return bool(c.value)

    def stats(self):
        s = ServerStats()
        _check(lib().sph_hoa_server_get_stats(self.handle, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self.handle:
            _check(lib().sph_hoa_server_destroy(self.handle))
            self.handle = None
            self._keep.clear()


def sph_hoa_optimal_knots(kernel, pieces, degree, lam):
    """Library's optimal knots for one distance parameter (host only)."""
    import numpy as np

    P = (pieces + 1) // 2
    th = (ctypes.c_double * P)()
    e2 = ctypes.c_double()
    _check(lib().sph_hoa_optimal_knots(kernel, pieces, degree, lam, th, ctypes.byref(e2)))
    return np.array(list(th)), e2.value


def sph_hoa_knot_table(kernel, pieces, degree, n):
    """Library's optimal-knot table and per-entry squared errors (host only)."""
    import numpy as np

    th = np.zeros((n, (pieces + 1) // 2))
    e2 = np.zeros(n)
    _check(lib().sph_hoa_knot_table(kernel, pieces, degree, n, th.ctypes.data_as(ctypes.c_void_p),
                                    e2.ctypes.data_as(ctypes.c_void_p)))
    return th, e2


def sph_hoa_lut_coefficients(kernel, pieces, degree, theta):
    """Library's projection jumps for the given knot table (host only): (shat, smid, err2)."""
    import numpy as np

    th = np.ascontiguousarray(theta, dtype=np.float64)
    n, P = th.shape
    shat = np.zeros((n, P, degree + 1))
    smid = np.zeros((n, degree + 1))
    e2 = np.zeros(n)
    _check(lib().sph_hoa_lut_coefficients(kernel, pieces, degree, n, th.ctypes.data_as(ctypes.c_void_p),
                                          shat.ctypes.data_as(ctypes.c_void_p), smid.ctypes.data_as(ctypes.c_void_p),
                                          e2.ctypes.data_as(ctypes.c_void_p)))
    return shat, smid, e2


def sph_hoa_lut_project(kernel, pieces, degree, theta):
    """Projection jumps for the given knot table on the device (sph_hoa_lut_project): theta
    [n, ceil(K/2)] (tensor or array) -> device float64 tensors (shat [n, P, D+1], smid [n, D+1],
    err2 [n])."""
    import torch

    th = torch.as_tensor(theta, dtype=torch.float64).to("cuda").contiguous()
    n, P = th.shape
    shat = torch.empty((n, P, degree + 1), dtype=torch.float64, device=th.device)
    smid = torch.empty((n, degree + 1), dtype=torch.float64, device=th.device)
    e2 = torch.empty(n, dtype=torch.float64, device=th.device)
    _check(lib().sph_hoa_lut_project(kernel, pieces, degree, n, _ptr(th), _ptr(shat), _ptr(smid), _ptr(e2),
                                     _stream()))
    return shat, smid, e2


def sph_hoa_optimal_tau(kernel, degree, sigma, h_repr, phi_repr):
    """Library's length quantum (host only)."""
    t = ctypes.c_double()
    _check(lib().sph_hoa_optimal_tau(kernel, degree, sigma, h_repr, phi_repr, ctypes.byref(t)))
    return t.value


def sph_hoa_accumulate_bits(bits, degree, dist, jumps, n_threads, steps, want_out=True):
    """Accumulation rule in wrap-around `bits`-bit integers (Sec. 5.1 cost study).

    dist: uint32 [n_table]; jumps: uint32 [n_table, degree + 1, bits // 32] (low limb first).
    Returns (states uint32 [n_threads, degree + 1, bits // 32] or None, kernel milliseconds)."""
    import numpy as np

    L = bits // 32
    d = np.ascontiguousarray(dist, dtype=np.uint32)
    j = np.ascontiguousarray(jumps, dtype=np.uint32)
    if j.shape != (d.shape[0], degree + 1, L):
        raise ValueError(f"jumps must have shape {(d.shape[0], degree + 1, L)}, got {j.shape}")
    out = np.zeros((n_threads, degree + 1, L), dtype=np.uint32) if want_out else None
    ms = ctypes.c_float()
    _check(lib().sph_hoa_accumulate_bits(bits, degree, d.ctypes.data_as(ctypes.c_void_p),
                                         j.ctypes.data_as(ctypes.c_void_p), d.shape[0], n_threads, steps,
                                         out.ctypes.data_as(ctypes.c_void_p) if want_out else None,
                                         ctypes.byref(ms), _stream()))
    return out, ms.value
