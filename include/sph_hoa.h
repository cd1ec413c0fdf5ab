/*
 * sph_hoa.h - C ABI of the MI355X library for particle-wise higher-order SPH
 * field approximation on viewing rays (arXiv 2401.02896, "Particle-Wise
 * Higher-Order SPH Field Approximation for DVR").
 *
 * Pipeline (Sec. 2, three passes): for every ray, each SPH particle whose
 * kernel support the ray crosses contributes an L2-optimal even piecewise
 * polynomial of degree D with K pieces (Sec. 3), quantized to integer knots
 * (Sec. 4.2-4.3); per ray the knots are sorted and accumulated exactly with
 * the integer update rule (Eq. accumulation-rule); the resulting exact field
 * is merged under an error bound and classified / composited front to back.
 *
 * Conventions for every call:
 *  - All array arguments are DEVICE pointers (hipMalloc'd or torch tensors on
 *    the current ROCm device) unless stated otherwise; the caller owns them.
 *  - `stream` is a hipStream_t (NULL = default stream).  Work is enqueued on
 *    it; calls that must report counts synchronise it (stated per call).
 *  - No call throws across the ABI.  Every call returns a status; on failure
 *    sph_hoa_last_error() (thread-local) holds a detail message and outputs
 *    are unspecified except where stated.
 *  - Host-detectable argument errors are reported before anything is launched.
 */
#ifndef SPH_HOA_H
#define SPH_HOA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPH_HOA_OK = 0,
  SPH_HOA_E_INVALID_ARG = 1,   /* bad argument: NULL, NaN, h <= 0, non-unit direction, bad K/D ... */
  SPH_HOA_E_OUT_OF_MEMORY = 2, /* device allocation failed, or a caller capacity is too small */
  SPH_HOA_E_OVERFLOW = 3,      /* a quantized position or coefficient leaves its integer range: knot
                                  positions are int64 quanta (|t| + q h_max < 4e18 tau), and the
                                  knots of one ray must span fewer than 2^32 quanta (positions are
                                  handled relative to the ray's first knot in 32 bits) */
  SPH_HOA_E_DEVICE = 4,        /* HIP runtime error */
  SPH_HOA_E_UNSUPPORTED = 5,   /* configuration outside the implemented range */
  SPH_HOA_E_INTERNAL = 6,      /* an internal invariant failed (e.g. a ray's knots did not cancel) */
  SPH_HOA_E_BUSY = 7,          /* render server: request rejected, the queue is at its limit */
  SPH_HOA_E_CANCELLED = 8      /* render server: the request was cancelled before it ran */
} sph_hoa_status;

typedef enum {
  SPH_HOA_KERNEL_CUBIC = 0,       /* cubic B-spline, Eq. cubic-kernel, support q = 2 */
  SPH_HOA_KERNEL_WENDLAND_C2 = 1, /* (21/16pi)(1-r/2)^4(1+2r), support q = 2 */
  SPH_HOA_KERNEL_WENDLAND_C4 = 2, /* (495/256pi)(1-r/2)^6(1+3r+35/12 r^2), support q = 2 */
  SPH_HOA_KERNEL_WENDLAND_C6 = 3, /* (1365/512pi)(1-r/2)^8(1+4r+25/4 r^2+4r^3), support q = 2 */
  /* Transverse gradient kernels g(r) = -w'(r)/r of the Wendland kernels (Sec. 6: the procedure
   * carries over to other features that particles generate additively, such as gradients).  With
   * y = (x - chi)/h a particle's gradient is h^-4 w'(r) y / r; on a ray x = o + t v its component
   * along a unit axis e is (v.e) d/dt[h^-3 w] - h^-5 g(r) (alpha + beta.chi), where
   * alpha = o.e - (o.v)(v.e) and beta = (v.e) v - e are constants of the ray.  The gradient along e
   * is therefore (v.e) F'(t) - alpha G0(t) - beta.(Gx, Gy, Gz)(t): F the field of w with values c,
   * G0 and Gx, Gy, Gz the fields of g with values c/h^2 and c chi_x/h^2, c chi_y/h^2, c chi_z/h^2
   * (indices built from those values; values may be negative). */
  SPH_HOA_KERNEL_WENDLAND_C2_GRAD = 4, /* (21/16pi) 5 (1-r/2)^3 */
  SPH_HOA_KERNEL_WENDLAND_C4_GRAD = 5, /* (495/256pi)(14/3)(1-r/2)^5(1+5r/2) */
  SPH_HOA_KERNEL_WENDLAND_C6_GRAD = 6  /* (1365/512pi)(11/2)(1-r/2)^7(1+7r/2+4r^2) */
} sph_hoa_kernel;

/* approx_rays: also return the sorted knots and the pre-merge exact integer pieces */
#define SPH_HOA_FLAG_EXACT 1u
/* sph_hoa_params.flags: storage precision of the float table (the knots theta_k and projection
 * jumps s-hat of Sec. 3.1), for the precision study.  Every table value is rounded once, when the
 * index is built, to the nearest float32 (LUT_FP32), to the nearest bfloat16 of that float32
 * (LUT_BF16: 8 significant bits, ties to even) or to the nearest IEEE binary16 of that float32
 * (LUT_FP16: 11 significant bits, subnormals below 2^-14, ties to even; a value beyond 65504
 * becomes infinite and is reported by the render as E_OVERFLOW); the per-hit quantization
 * (Sec. 4.3) then uses the rounded values, and the integer accumulation stays exact (the closure is
 * computed from the rounded jumps).  At most one of them; none: float64. */
#define SPH_HOA_FLAG_LUT_FP32 2u
#define SPH_HOA_FLAG_LUT_BF16 4u
#define SPH_HOA_FLAG_LUT_FP16 8u
/* sph_hoa_params.flags: a transverse gradient field (Sec. 6; at most one of the three): every
 * (particle, ray) pair contributes with amplitude value * m, m = ((o + t_chi v - chi) . e_a) / h the
 * particle's perpendicular offset from the ray along axis a in units of its smoothing length
 * (|m| <= Lambda < q), so that with kernel <kernel>_GRAD (g = -w'/r) and values c / h the field T_a
 * gives the gradient of the value field across the ray: e.grad f = (v.e) F'(t) - sum_a e_a T_a(t).
 * Quanta derived from the data (a_max <= 0) then bound |value * m| (twice the value bound). */
#define SPH_HOA_FLAG_TRANSVERSE_X 16u
#define SPH_HOA_FLAG_TRANSVERSE_Y 32u
#define SPH_HOA_FLAG_TRANSVERSE_Z 64u

/* Method parameters (Sec. 3.2 K and D, Sec. 4.4 quanta, Sec. 5 bit length). */
typedef struct {
  int32_t degree;       /* D: polynomial degree, 1..6 */
  int32_t pieces;       /* K: non-trivial pieces per particle, 1..6, with K*D >= 2 */
  int32_t lut_entries;  /* number of equidistant Lambda table entries (Sec. 3.1); 0 -> 4096; 2..65536 */
  int32_t int_bits;     /* integer bit length (Sec. 5.1); only 64 is implemented; 0 -> 64 */
  double merge_tol;     /* merge tolerance relative to the ray's peak; 0 disables merging */
  double a_max;         /* > 0: bound on |field| used for sigma = a_max / INT_MAX (Sec. 4.4); else derived */
  double h_repr;        /* > 0: representative smoothing length (Sec. 4.4); else lower median of h */
  double phi_repr;      /* > 0: representative amplitude / h^3; else lower median of |value| / h^3 */
  double tau;           /* > 0: length quantum to use instead of the minimiser of Q_D */
  const double* knot_table; /* optional HOST array [lut_entries][ceil(K/2)] of optimal knots theta_k
                               (units of h) replacing the library's own optimisation (Sec. 3.4); copied */
  uint32_t flags;       /* 0 or one of SPH_HOA_FLAG_LUT_FP32 / _BF16 / _FP16 */
  const double* jump_table;     /* optional HOST [lut_entries][ceil(K/2)][D+1]: projection jumps s-hat at
                                   +theta_k (Sec. 3.1) replacing the library's projection; requires
                                   knot_table (the knots they belong to); copied */
  const double* jump_table_mid; /* with jump_table and even K: HOST [lut_entries][D+1] jumps at 0 */
} sph_hoa_params;

typedef struct sph_hoa_index_s* sph_hoa_index; /* opaque; owns its device memory */

/* Read-back of the quantities an index was built with (host struct). */
typedef struct {
  int64_t n_particles;
  int32_t kernel, degree, pieces, lut_entries;
  double tau, sigma, a_max, h_repr, phi_repr;
  double grid_lo[3];
  double cell0;         /* finest cell size c_0 (a power of two) */
  int32_t n_levels;
  int32_t level_dims[32][3];
  uint32_t lut_flags;   /* table storage precision the index was built with (params.flags) */
} sph_hoa_index_info;

/* Rays x(t) = origin + t * dir, t in [t_min, t_max] (Fig. 1). */
typedef struct {
  int64_t n;
  const float* origin;  /* device [n][3] */
  const float* dir;     /* device [n][3], unit length (|dir|^2 within 1e-5 of 1) */
  float t_min, t_max;   /* t_min < t_max, |t| < 2^30 * tau */
} sph_hoa_rays;

/* Output of approx_rays.  Merged piece i of ray r is index ray_offsets[r] + j:
 * F(t) = sum_d coef[i][d] * u^d with u = (t - t_start[i]) / (t_end[i] - t_start[i]),
 * valid on [t_start[i], t_end[i]]; the field is zero outside a ray's pieces.  The pieces' exact
 * ends are integer knot positions times tau; t_start / t_end hold their float32 roundings, and the
 * coefficients are re-expressed about those stored ends (in float64, then rounded to float32), so
 * u computed from t_start / t_end evaluates the merged piece itself.  A piece whose two float32
 * ends coincide (shorter than their resolution) holds its start value in coef[i][0] and zeros. */
typedef struct {
  int64_t capacity;      /* pieces allocated by the caller */
  int64_t* ray_offsets;  /* device [n + 1] */
  float* t_start;        /* device [capacity] */
  float* t_end;          /* device [capacity] */
  float* coef;           /* device [capacity][D + 1] */
  float* ray_peak;       /* device [n]: sigma * max |a_0| over the ray's exact pieces */
  /* outputs written by the call (host fields): */
  int64_t n_pieces;      /* merged pieces written (or needed, on E_OUT_OF_MEMORY) */
  int64_t n_pairs;       /* (particle, ray) contributions */
  int64_t n_knots;
  int64_t n_exact_pieces;
  /* exact mode (params flags of the call = SPH_HOA_FLAG_EXACT); all device, may be NULL otherwise */
  int64_t exact_capacity;  /* capacity of exact_t / exact_coef (pieces) */
  int64_t* exact_offsets;  /* [n + 1] */
  int64_t* exact_t;        /* [exact_capacity] start of the piece in quanta (end = next start) */
  int64_t* exact_end;      /* [exact_capacity] end of the piece in quanta */
  int64_t* exact_coef;     /* [exact_capacity][D + 1] integer localized coefficients a_d */
  int64_t knot_capacity;   /* capacity of the knot arrays */
  int64_t* knot_offsets;   /* [n + 1] */
  int64_t* knot_t;         /* [knot_capacity] knot position in quanta, sorted per ray */
  int32_t* knot_pid;       /* [knot_capacity] particle input index (ties broken by pid, then kidx) */
  int32_t* knot_kidx;      /* [knot_capacity] k + ceil(K/2) for the knot at t0 + sign(k) o_|k| */
} sph_hoa_field;

typedef struct {
  float eye[3], look_at[3], up[3];
  float fov_y_deg;          /* perspective vertical field of view */
  int32_t ortho;            /* 1: orthographic, rays parallel to look_at - eye */
  float ortho_half_extent;  /* orthographic half height of the view */
  int32_t width, height;    /* pixels; ray index = row * width + col, row 0 at the top */
  float t_min, t_max;       /* ray segment */
} sph_hoa_camera;

/* 1-D transfer function: n RGBA control points equally spaced on [v_min, v_max],
 * linearly interpolated and clamped; rgb = emission density, a = extinction. */
typedef struct {
  const float* rgba;  /* device [n][4] */
  int32_t n;          /* >= 2 */
  float v_min, v_max; /* v_max > v_min */
  float step;         /* sampling step along the ray (world units), > 0, (t_max - t_min) / step < 2^30 */
} sph_hoa_tf;

/* Counters of the last approx_rays / render on an index (host struct). */
typedef struct {
  int64_t n_rays;
  int64_t n_pairs;
  int64_t n_knots;
  int64_t n_pieces;       /* merged pieces (render: pieces composited) */
  int64_t max_hits;       /* largest number of contributions on one ray */
  int64_t rays_global;    /* rays whose whole per-ray layout was in device memory instead of LDS */
  int64_t rays_jumps_device; /* rays with keys in LDS, per-hit jump rows in device memory */
  int64_t rays_scratch_device; /* rays with keys in LDS, jump rows and sort scratch in device memory */
  /* with timing enabled (sph_hoa_index_set_timing): device time summed over the timed calls
   * since timing was (re-)enabled, from hipEvents recorded on the call's stream */
  int64_t timed_calls;
  double ms_gather;       /* hit gathering (both passes) */
  double ms_field;        /* per-ray field kernel (knots, sort, accumulation, merge, composite) */
} sph_hoa_stats;

/*
 * Build the particle index and the per-configuration tables.
 *  xyz [n][3], h [n] (> 0), value [n] (amplitude m*alpha/rho, Sec. 1): device float32, copied.
 *  Computes the optimal-knot table and projection coefficients (Sec. 3.1-3.4) for
 *  (kernel, K, D, lut_entries), the quanta tau and sigma (Sec. 4.4), and a
 *  multi-level Morton grid of the particles.  Synchronises `stream`.
 *  On success *out receives a handle to free with sph_hoa_index_free.
 */
sph_hoa_status sph_hoa_build_index(const float* xyz, const float* h, const float* value, int64_t n,
                                   sph_hoa_kernel kernel, const sph_hoa_params* params, void* stream,
                                   sph_hoa_index* out);

/*
 * Per-ray higher-order field for arbitrary rays (Sec. 2 passes 1-3 without
 * classification).  Writes out->ray_offsets, pieces and ray_peak; fills the
 * host counters of *out.  flags: 0 or SPH_HOA_FLAG_EXACT.  Synchronises `stream`.
 * If out->capacity (or an exact-mode capacity) is too small, returns
 * SPH_HOA_E_OUT_OF_MEMORY with the required count in n_pieces (and
 * n_exact_pieces / n_knots); nothing else is guaranteed then.
 */
sph_hoa_status sph_hoa_approx_rays(sph_hoa_index idx, const sph_hoa_rays* rays, sph_hoa_field* out,
                                   uint32_t flags, void* stream);

/*
 * Fields of several indices along the same rays with one hit gathering (Sec. 2 pass 1 done once):
 * out[i] receives exactly what sph_hoa_approx_rays(idx[i], rays, &out[i], flags, stream) gives.
 * For fields that the same particles generate with other values or kernels, e.g. the value field
 * and the four transverse gradient fields (Sec. 6; SPH_HOA_KERNEL_WENDLAND_C2_GRAD).
 * idx: HOST array of n_idx >= 1 indices built from the same positions and smoothing lengths (same
 * order; values, kernel, K, D and quanta may differ) — compared on the device first,
 * SPH_HOA_E_INVALID_ARG if they differ.  out: HOST array of n_idx fields, each as for
 * sph_hoa_approx_rays.  Processes idx[0] first (it gathers), then the others in order; on an
 * error the outputs from the failing index on are undefined.  Synchronises `stream`.
 */
sph_hoa_status sph_hoa_approx_rays_shared(const sph_hoa_index* idx, int32_t n_idx, const sph_hoa_rays* rays,
                                          sph_hoa_field* out, uint32_t flags, void* stream);

/*
 * Render: camera rays, per-ray field, merge with the index's merge_tol,
 * classification with `tf` and front-to-back emission-absorption compositing.
 * rgba_out: device float32 [height][width][4] (premultiplied colour, alpha = 1 - T).
 * Asynchronous on `stream` except for one read of the per-frame hit counts.
 */
sph_hoa_status sph_hoa_render(sph_hoa_index idx, const sph_hoa_camera* cam, const sph_hoa_tf* tf,
                              float* rgba_out, void* stream);

/*
 * sph_hoa_render without allocation, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, hosts that forbid hipMalloc): same arguments, checks
 * and result as sph_hoa_render (bit for bit), but every per-call device buffer (rays, hit counts
 * and lists, screen-tile lists, sort and scan temporaries, the field kernel's slabs and counters)
 * is placed in one fixed array of sph_hoa_static_scratch_bytes() bytes (128 MiB) that the library
 * holds on each device it runs on until the process ends; the call makes no hipMalloc, hipFree
 * or other allocating call.  A frame whose buffers do not fit (about 4 bytes per contribution
 * for the hit lists plus 48 per ray, and at least one field work-group's slab; fewer persistent
 * field work-groups run when not all slabs fit) returns SPH_HOA_E_OUT_OF_MEMORY; the device
 * work is then drained and nothing is written to rgba_out.  All calls on one device share the
 * array: calls that overlap on one device (from several host threads or streams) race and must
 * be serialised by the caller.  Synchronises `stream` before returning.  The index's own
 * per-call buffers are left as they were.
 */
sph_hoa_status sph_hoa_render_static(sph_hoa_index idx, const sph_hoa_camera* cam, const sph_hoa_tf* tf,
                                     float* rgba_out, void* stream);
/* Size in bytes of the fixed per-device scratch array of sph_hoa_render_static. */
int64_t sph_hoa_static_scratch_bytes(void);
/* Number of device allocations (hipMalloc) the library has made in this process so far, for
 * callers that check that a region of their code allocates nothing.  Thread-safe. */
int64_t sph_hoa_device_alloc_count(void);

/*
 * Fields along a camera's pixel rays, with the rays and the hit gathering of sph_hoa_render (the
 * screen-tile binning of Sec. 2's first pass): out receives what sph_hoa_approx_rays gives for
 * arbitrary rays (ray index = row * width + col; same flags, capacities and errors), and the merged
 * pieces are those sph_hoa_render classifies and composites for that camera.  Synchronises `stream`.
 */
sph_hoa_status sph_hoa_approx_camera(sph_hoa_index idx, const sph_hoa_camera* cam, sph_hoa_field* out,
                                     uint32_t flags, void* stream);

/*
 * First pass only (Sec. 2: every particle is assigned to all relevant viewing rays; Fig. 1: a
 * particle is relevant to a ray when Lambda < q and its support interval overlaps [t_min, t_max]).
 * sph_hoa_camera_hits gathers as sph_hoa_render does (screen tiles), sph_hoa_ray_hits as
 * sph_hoa_approx_rays does (grid walk).  hit_offsets: device int64 [n + 1]; hit_ids: device int32
 * [capacity], the particles' input indices; ray r's hits are hit_ids[hit_offsets[r] ..
 * hit_offsets[r + 1]) in an unspecified order.  *n_pairs (host) receives the number of hits; when
 * it exceeds capacity the call returns E_OUT_OF_MEMORY with *n_pairs set and hit_ids untouched.
 * Synchronises `stream`.
 */
sph_hoa_status sph_hoa_camera_hits(sph_hoa_index idx, const sph_hoa_camera* cam, int64_t* hit_offsets,
                                   int32_t* hit_ids, int64_t capacity, int64_t* n_pairs, void* stream);
sph_hoa_status sph_hoa_ray_hits(sph_hoa_index idx, const sph_hoa_rays* rays, int64_t* hit_offsets,
                                int32_t* hit_ids, int64_t capacity, int64_t* n_pairs, void* stream);

/*
 * Render a batch of cameras (each with its own size, frame and t range) with one launch chain:
 * all their rays are generated, gathered (grid walk), scheduled longest first and processed
 * together, so many small images share the GPU.  Each image equals the one sph_hoa_render gives
 * for that camera (same hit sets, fields and compositing arithmetic).
 * cams: HOST array [n_cams] (0 <= n_cams <= 2^20), copied.  rgba_out: device float32, the images
 * concatenated in camera order, each [height][width][4]; at most 2^32 rays in total.
 * Synchronises `stream` once (per-frame hit counts); NULL cams / rgba_out allowed when n_cams = 0.
 */
sph_hoa_status sph_hoa_render_batch(sph_hoa_index idx, const sph_hoa_camera* cams, int32_t n_cams,
                                    const sph_hoa_tf* tf, float* rgba_out, void* stream);

/* ---------------------------------------------------------------- float accumulation variant
 *
 * The update rule swept along each ray in float32 (Sec. 4.1), with optional reinitialization
 * knots, for measuring what the quantization of Sec. 4.2 avoids.  Same hits, closest points and
 * table entries as the exact path; per hit the knots sit at tc -+ zf theta_k (and tc for even K)
 * with tc, zf, vf the float32 roundings of t_chi, zeta, amplitude, and carry the jumps
 * s-hat_kd vf / zf^(3+d) (at -theta_k times (-1)^(d+1); at 0 the table's middle jump).  Knots are
 * ordered by (position, particle input index, kidx) and swept by one thread per ray: shift the
 * state to the knot (in-place Taylor shift), add the jump.  n_reinit >= 1 places reinitialization
 * knots at T_s = t_min + s (t_max - t_min) / (n_reinit + 1), s = 1..n_reinit (float32): each holds
 * the sum, in increasing particle input index, of the localized coefficients at T_s of every
 * particle whose first knot is <= T_s < its last knot (each from that particle's own float sweep
 * of its knots <= T_s); the sweep takes them after all knots at positions <= T_s.  Output: one
 * piece per gap between consecutive event positions, coefficients of (t - t_start)^d at its start,
 * and a last piece from the final event to t_max (exactly zero in exact arithmetic).  Ray r's
 * pieces occupy slots [ray_offsets[r], ray_offsets[r] + ray_counts[r]) with
 * ray_offsets[r] = (K + 1) * (hits before r) + r * (n_reinit + 2); the call needs
 * capacity >= ray_offsets[n], reported in n_slots (E_OUT_OF_MEMORY, with nothing written, when
 * capacity is smaller: call again with enough).  0 <= n_reinit <= 1024.  Synchronises `stream`. */
typedef struct {
  int64_t capacity;      /* piece slots allocated by the caller */
  int64_t* ray_offsets;  /* device [n + 1] */
  int64_t* ray_counts;   /* device [n] */
  float* t_start;        /* device [capacity] */
  float* t_end;          /* device [capacity] */
  float* coef;           /* device [capacity][D + 1], powers of (t - t_start) */
  int64_t n_slots;       /* out (host): slots the call needs */
  int64_t n_pairs;       /* out (host) */
} sph_hoa_float_field;

sph_hoa_status sph_hoa_float_rays(sph_hoa_index idx, const sph_hoa_rays* rays, int32_t n_reinit,
                                  sph_hoa_float_field* out, void* stream);

/* ---------------------------------------------------------------- render server
 *
 * A resident request loop with continuous batching: indices stay in device memory, render requests
 * (one camera each) are queued from any host thread, and the server's lanes (worker threads, each
 * with its own stream and per-call device state) render them.  A free lane starts the oldest
 * queued request as soon as its estimated transient device memory fits in what the batches already
 * in flight leave of the budget (or when nothing is in flight), together with the queued requests
 * of the same index and transfer function, in arrival order, that still fit (memory and
 * max_batch_rays), as one sph_hoa_render_batch launch chain.  Requests arriving while batches run
 * are thus admitted as memory is returned and their work overlaps the running batches on the
 * device; batches of different indices run side by side on different lanes.  Each image is
 * bit-identical to sph_hoa_render of its camera alone.  An index added to a server belongs to it
 * until the server is destroyed (no other call may use it meanwhile); the transfer function's
 * device array and the output buffers must stay valid until the request has completed.
 */
typedef struct sph_hoa_server_s* sph_hoa_server;

typedef struct {
  int64_t completed, failed, queued, batches;
  int64_t n_rays, n_pairs;    /* over the completed batches */
  double busy_s;              /* lane time spent rendering, summed over the lanes */
  double p50_ms, p99_ms, max_ms; /* request latency, submit to completion, over completed requests */
  int64_t rejected;           /* submissions refused by the admission limits */
  int64_t cancelled;          /* requests cancelled while queued */
  int64_t lanes;              /* worker lanes */
  int64_t overlapped_batches; /* batches that started while another batch was being rendered */
  int64_t max_in_flight;      /* most batches rendered at once */
} sph_hoa_server_stats;

/* hbm_budget_bytes: admission bound on the estimated transient device memory of all batches in
 * flight (a single request larger than it still runs, alone); max_batch_rays: bound on a batch's
 * rays.  sph_hoa_server_create uses 2 lanes; sph_hoa_server_create_lanes takes 1..16. */
sph_hoa_status sph_hoa_server_create(int64_t hbm_budget_bytes, int64_t max_batch_rays, sph_hoa_server* out);
sph_hoa_status sph_hoa_server_create_lanes(int64_t hbm_budget_bytes, int64_t max_batch_rays, int32_t n_lanes,
                                           sph_hoa_server* out);
/* Admission limits checked at submission (0: no limit): max_queued - a submission that finds
 * this many requests waiting is refused with E_BUSY; max_request_bytes - a request whose own
 * estimated transient device memory exceeds it is refused with E_OUT_OF_MEMORY (it could never
 * run within that bound).  Refused submissions get no id and count in stats.rejected. */
sph_hoa_status sph_hoa_server_set_admission(sph_hoa_server server, int64_t max_queued, int64_t max_request_bytes);
/* paused != 0: the lanes start no new batch (batches already running complete; submissions still
 * queue); 0: resume.  Destroying a paused server still renders what is queued. */
sph_hoa_status sph_hoa_server_pause(sph_hoa_server server, int32_t paused);
/* Registers an index; *slot names it in submissions. */
sph_hoa_status sph_hoa_server_add_index(sph_hoa_server server, sph_hoa_index idx, int32_t* slot);
/* Queues one render (arguments as sph_hoa_render, checked now); *request_id names it. */
sph_hoa_status sph_hoa_server_submit(sph_hoa_server server, int32_t slot, const sph_hoa_camera* cam,
                                     const sph_hoa_tf* tf, float* rgba_out, int64_t* request_id);
/* Waits up to timeout_s seconds (< 0: without limit).  *done = 1 once the request has completed
 * (then its image is in rgba_out, *latency_ms holds its latency if non-NULL, the id is released,
 * and the status is the request's own); *done = 0 on time-out (status OK, id still valid). */
sph_hoa_status sph_hoa_server_wait(sph_hoa_server server, int64_t request_id, double timeout_s, int32_t* done,
                                   double* latency_ms);
/* Cancels a request that is still queued: *cancelled = 1, and its wait then reports done with
 * status E_CANCELLED (its output buffer is left untouched).  A request already taken by a lane or
 * completed is not affected (*cancelled = 0).  Unknown id: E_INVALID_ARG. */
sph_hoa_status sph_hoa_server_cancel(sph_hoa_server server, int64_t request_id, int32_t* cancelled);
sph_hoa_status sph_hoa_server_get_stats(sph_hoa_server server, sph_hoa_server_stats* stats);
/* Renders what is still queued, stops the lanes and frees the server (not its indices).  No other
 * call on this server may be running or follow (waits included). */
sph_hoa_status sph_hoa_server_destroy(sph_hoa_server server);

/* ---------------------------------------------------------------- integer bit length
 *
 * Microbenchmark of the accumulation rule (Eq. accumulation-rule) in wrap-around W-bit integers,
 * the cost the paper weighs in Sec. 5.1 (32-bit against emulated 64, 96 and 128 bits).  W = bits
 * in {32, 64, 96, 128}; a W-bit value is W/32 uint32 limbs, low limb first.  n_threads independent
 * accumulators each take `steps` knots: knot s of accumulator g is table entry
 * k = (g + s mod 4) mod n_table.  At knot 0 the state is jumps[k]; at every later knot the state is
 * first shifted forward by dist[k] (the distance from the previous knot: D (D + 1) / 2
 * multiply-adds of a W-bit coefficient by the 32-bit distance) and then jumps[k] is added, all
 * modulo 2^W.  Host buffers (read or written before the call returns): dist [n_table],
 * jumps [n_table][D + 1][W/32], out_host [n_threads][D + 1][W/32] (the final states; NULL: timing
 * only).  *ms_out (may be NULL): the kernel's duration from hipEvents on `stream`.  Limits:
 * 1 <= degree <= 6, n_table >= 1, 1 <= n_threads <= 2^26, steps a positive multiple of 4;
 * otherwise E_INVALID_ARG.  Synchronous; device buffers are allocated and freed per call. */
sph_hoa_status sph_hoa_accumulate_bits(int32_t bits, int32_t degree, const uint32_t* dist, const uint32_t* jumps,
                                       int32_t n_table, int64_t n_threads, int32_t steps, uint32_t* out_host,
                                       float* ms_out, void* stream);

sph_hoa_status sph_hoa_index_free(sph_hoa_index idx);

/* Host copy of the index parameters. */
sph_hoa_status sph_hoa_index_get_info(sph_hoa_index idx, sph_hoa_index_info* info);

/* Host copies of the table: theta [lut_entries][P], shat [lut_entries][P][D+1] (jump
 * coefficients at +theta_k), smid [lut_entries][D+1] (jump at 0, even K); any may be NULL. */
sph_hoa_status sph_hoa_index_get_lut(sph_hoa_index idx, double* theta, double* shat, double* smid);

/* Device copies of the grid keys: morton [n] (Morton code of the particle's cell), level [n],
 * order [n] (input index of the i-th particle in (level, Morton, index) order); any may be NULL. */
sph_hoa_status sph_hoa_index_get_grid(sph_hoa_index idx, uint64_t* morton, int32_t* level, int32_t* order,
                                      void* stream);

/* Counters of the last call on this index; synchronises the stream of that call. */
sph_hoa_status sph_hoa_index_get_stats(sph_hoa_index idx, sph_hoa_stats* stats);

/* on != 0: record hipEvents around the gather and field kernels of every later call and
 * accumulate their durations into the stats (resets the sums); 0: stop. */
sph_hoa_status sph_hoa_index_set_timing(sph_hoa_index idx, int32_t on);

/* Host-only: the library's optimal knots for one Lambda (Sec. 3.4), theta_out[ceil(K/2)],
 * and the squared L2 error of the optimum.  No GPU work. */
sph_hoa_status sph_hoa_optimal_knots(sph_hoa_kernel kernel, int32_t pieces, int32_t degree, double lambda,
                                     double* theta_out, double* err2_out);

/* Host-only: the library's optimal-knot table (Sec. 3.1, 3.4) for n equidistant Lambda_i = (i + 1/2) q / n,
 * theta_out[n][ceil(K/2)], and the squared L2 error of each entry err2_out[n] (may be NULL). */
sph_hoa_status sph_hoa_knot_table(sph_hoa_kernel kernel, int32_t pieces, int32_t degree, int32_t n, double* theta_out,
                                  double* err2_out);

/* Host-only: the projection of B_Lambda onto the candidate space for given knots (Sec. 3.3,
 * Eq. optimal-approx-for-given-knots) as localized jump coefficients, for every entry of a table:
 * theta [n][ceil(K/2)] (input), shat_out [n][ceil(K/2)][D+1] (jump at +theta_k), smid_out [n][D+1]
 * (jump at 0 for even K; may be NULL), err2_out [n] (may be NULL). */
sph_hoa_status sph_hoa_lut_coefficients(sph_hoa_kernel kernel, int32_t pieces, int32_t degree, int32_t n,
                                        const double* theta, double* shat_out, double* smid_out, double* err2_out);

/* The same projection on the device (Sec. 3.3, App. A.1/A.2; the table of Sec. 3.1), as used by
 * sph_hoa_build_index: one wave per entry Lambda_i = (i + 1/2) q / n forms the normal equations of
 * the candidate basis by Gauss-Legendre quadrature and solves them in float64.  All four arrays are
 * device memory owned by the caller: theta [n][ceil(K/2)] (input, positive and increasing per row),
 * shat_out [n][ceil(K/2)][D+1], smid_out [n][D+1] (zero for odd K), err2_out [n].  Runs on `stream`
 * and synchronises it.  E_INVALID_ARG for a row that is not positive and increasing or whose
 * projection is singular. */
sph_hoa_status sph_hoa_lut_project(sph_hoa_kernel kernel, int32_t pieces, int32_t degree, int32_t n,
                                   const double* theta, double* shat_out, double* smid_out, double* err2_out,
                                   void* stream);

/* Host-only: the length quantum minimising Q_D(tau / h_repr, sigma / phi_repr) (Sec. 4.4, App. A.5). */
sph_hoa_status sph_hoa_optimal_tau(sph_hoa_kernel kernel, int32_t degree, double sigma, double h_repr,
                                   double phi_repr, double* tau_out);

const char* sph_hoa_status_string(sph_hoa_status s);
const char* sph_hoa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPH_HOA_H */
