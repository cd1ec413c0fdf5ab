// Internal declarations shared by the library's translation units.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <map>
#include <vector>

#include "../../include/sph_hoa.h"
#include "tables.h"

namespace sph {

constexpr int kMaxLevels = 32;
constexpr int kMaxD = 6;
constexpr int kMaxP = 3;
constexpr int kChunk = 16;          // knots per merge chunk
// Field kernel configurations: threads per ray work-group (256 or 512) and work-groups per CU
// (which also splits the CU's LDS between the rays), numbered 1..4 (256 threads, 1..4 per CU) and
// 5..6 (512 threads, 1..2 per CU).  field_cfg_valid: the ones a degree can run without spilling
// registers; rendering keeps one thread count per degree (512 for D <= 3, 256 above), because the
// compositing partials are combined over the work-group's threads and a pixel must not depend on
// the configuration, while the fields (integer sums, chunked merge) are the same bits under every
// configuration.  The tuner picks among the valid ones per workload signature.
constexpr int kFieldCfgs = 6;
constexpr int field_cfg_threads(int cfg) { return cfg > 4 ? 512 : 256; }
constexpr int field_cfg_wgs(int cfg) { return cfg > 4 ? cfg - 4 : cfg; }
constexpr bool field_cfg_valid(int D, bool render, int cfg) {
  return cfg < 1 || cfg > kFieldCfgs ? false
         : field_cfg_threads(cfg) == 512
             ? (D <= 3 && field_cfg_wgs(cfg) <= 2)
             : (!(render && D <= 3) &&
                field_cfg_wgs(cfg) <= (render ? (D <= 5 ? 3 : 2) : (D <= 1 ? 4 : (D <= 4 ? 3 : 2))));
}
constexpr int kFieldThreadsMin = 256;
constexpr int64_t kLdsPerCu = 160 * 1024;
constexpr int64_t kMaxAxisCells = int64_t(1) << 19;
constexpr int64_t kMaxLevel0Cells = int64_t(1) << 24;
constexpr double kAmaxMargin = 1.25;

// error-flag bits raised by kernels
enum : uint32_t {
  kFlagBadInput = 1u,       // NaN / h <= 0 / non-unit direction
  kFlagPosRange = 2u,       // a ray's knots span 2^32 quanta or more, or a knot offset reached 2^31
  kFlagCoefRange = 4u,      // a quantized coefficient left |x| < 2^62
  kFlagTail = 8u,           // a ray's accumulated coefficients did not return to zero
  kFlagWindow = 16u,        // grid enumeration window too small (internal)
  kFlagCapacity = 32u,      // an output capacity was exceeded
};

struct Error : std::runtime_error {
  sph_hoa_status status;
  Error(sph_hoa_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

// A named range on the host timeline (roctx): rocprofv3 --marker-trace shows each ABI call and
// each phase of a frame as a range; without a profiler attached a push/pop pair costs a few
// nanoseconds.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

inline void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(SPH_HOA_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

struct LevelInfo {
  double c, inv_c;
  int n[3];
  int64_t cell_off;  // offset of this level's cells in the cell arrays
  int64_t n_particles;
};

struct GridDev {
  double lo[3];
  int n_levels;
  LevelInfo lv[kMaxLevels];
};

// Device allocations the library has made in this process (every one goes through DevBuf).
inline std::atomic<int64_t> g_device_allocs{0};

// Bump region in caller-provided device memory: per-call buffers bound to it take their space
// from it instead of allocating (see bind_static_scratch).
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
};

// Device buffer that grows on demand and frees itself.  When bound to an arena it never
// allocates: growing takes the next aligned range of the arena, or fails with E_OUT_OF_MEMORY.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  Arena* arena = nullptr;
  // defer = true: growing keeps the old allocation instead of freeing it (hipFree waits for all
  // work on the device, which would stall the work of other streams) and grows by at least half, so
  // that few generations are kept; they are freed together once they outgrow the new allocation
  // (one wait for every few growths) and when the buffer is destroyed
  bool defer = false;
  std::vector<void*> kept;
  size_t kept_bytes = 0;
  void ensure(size_t b) {
    if (b <= bytes) return;
    if (arena) {
      const size_t off = (arena->used + 255) & ~size_t(255);
      if (off > arena->cap || b > arena->cap - off)
        throw Error(SPH_HOA_E_OUT_OF_MEMORY, "the call needs more than the " + std::to_string(arena->cap) +
                                                 " bytes of static scratch memory");
      p = arena->base + off;
      bytes = b;
      arena->used = off + b;
      return;
    }
    if (p) {
      if (defer) {
        kept.push_back(p);
        kept_bytes += bytes;
      } else {
        (void)hipFree(p);
      }
    }
    if (defer) {
      b = std::max(b, bytes + bytes / 2);
      if (kept_bytes > b) {
        for (void* q : kept) (void)hipFree(q);
        kept.clear();
        kept_bytes = 0;
      }
    }
    p = nullptr;
    bytes = 0;
    if (b == 0) return;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(SPH_HOA_E_OUT_OF_MEMORY, "device allocation of " + std::to_string(b) + " bytes failed");
    }
    g_device_allocs.fetch_add(1, std::memory_order_relaxed);
    bytes = b;
  }
  // bytes that ensure() could still hand out (unbounded when not bound to an arena)
  size_t room() const {
    if (!arena) return SIZE_MAX;
    const size_t off = (arena->used + 255) & ~size_t(255);
    return off >= arena->cap ? 0 : arena->cap - off;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
  ~DevBuf() {
    if (p && !arena) (void)hipFree(p);
    for (void* q : kept) (void)hipFree(q);
  }
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

// Per-call constants of the method.
struct MethodConsts {
  int K, D, P, even_k, n_lut, kernel;
  double tau, sigma, q, merge_tol;
};

// Most field work-groups per CU for degree D (render or field output) that the kernel's registers
// allow without spilling.

// Online choice of the field kernel's work-groups per CU (1 to 4; a ray's layout gets 1 / wgs of
// the CU's LDS) per workload signature (degree, mode, log2 of the mean and of the largest hits per
// ray): each candidate is timed once on a real call (its output is identical), then the fastest is
// kept.
struct FieldTuner {
  struct Key {
    int D, render, mean_bucket, max_bucket;
    bool operator<(const Key& o) const {
      if (D != o.D) return D < o.D;
      if (render != o.render) return render < o.render;
      if (mean_bucket != o.mean_bucket) return mean_bucket < o.mean_bucket;
      return max_bucket < o.max_bucket;
    }
  };
  struct Entry {
    double ms_per_pair[kFieldCfgs + 1] = {-1.0, -1.0, -1.0, -1.0, -1.0, -1.0, -1.0};  // by configuration
  };
  // candidates (field kernel configurations), in the order they are measured
  static constexpr int kOrder[kFieldCfgs] = {6, 2, 3, 4, 5, 1};
  std::map<Key, Entry> table;
  bool pending = false;
  Key pend_key{};
  int pend_slot = 0;
  int64_t pend_pairs = 0;
  hipEvent_t ev[2] = {};
  static Key key_of(int D, bool render, int64_t pairs, int64_t rays, int64_t max_hits);
  int choose(const Key& k);
  int chosen(const Key& k) const;  // the best measured configuration (the first valid candidate while none is); times nothing
  void begin(const Key& k, int cfg, int64_t pairs, hipStream_t st);
  void end(hipStream_t st);
  void collect();
  FieldTuner() = default;
  FieldTuner(const FieldTuner&) = delete;
  FieldTuner& operator=(const FieldTuner&) = delete;
  ~FieldTuner();
};

// Per-call device state of the frame path (rays, hit lists, tiles, field-kernel slabs, counters),
// its statistics, the work-group tuner and optional kernel timing.  Every index owns one; the
// render server gives each of its lanes its own, so that batches of one index can be in flight on
// several streams at once.
struct Workspace {
  DevBuf rays_o, rays_v;        // double [n][3]
  DevBuf hit_count, hit_off;    // int64 [n + 1]
  DevBuf hit_slots;             // uint32 [n][slots]: single-pass gathering of arbitrary rays
  int64_t last_max_hits = 0;    // largest hit count of the previous arbitrary-ray call
  DevBuf hits;                  // uint32 [pairs]
  // where the previous arbitrary-ray call left its hit lists (for fields sharing that gathering):
  // per-ray slots of last_hit_slots entries, or compact lists in `hits` (last_hit_slots = 0)
  int64_t last_hit_slots = 0;
  int64_t last_hit_rays = -1;   // ray count of that call (-1: none)
  int64_t last_hit_max = 0;     // its largest hit count
  DevBuf tile_count, tile_off, tile_items;  // screen-tile binning of the particles (camera rays)
  DevBuf tile_masks;                         // per tile item: the tile pixels it hits
  DevBuf tile_order;                         // tiles by decreasing candidate count
  DevBuf scan_tmp;
  DevBuf counters;              // uint64 small counters / flags
  DevBuf slab;                  // per-work-group node / heavy-ray storage
  DevBuf ray_meta;              // per-ray outputs of the field kernel
  DevBuf out_stage, exact_stage;
  DevBuf cams_dev, ray_tr;          // camera batches: frames, ray offsets, per-ray segments
  DevBuf order_keys, order;         // processing order of arbitrary rays and batches
  DevBuf sort_hist, sort_offs;
  sph_hoa_stats stats{};
  FieldTuner tuner;
  bool render_stats_pending = false;  // placement counters of the last render not read back yet
  bool no_alloc = false;              // inside sph_hoa_render_static: no allocation, no tuner timing
  int time_slices = 1;                // > 1: field kernel launched in about this many slices
  // optional event timing of the kernels (sph_hoa_index_set_timing)
  bool timing = false;
  bool timing_pending = false;
  hipEvent_t ev[6] = {};
  int64_t timed_calls = 0;
  double ms_gather = 0.0, ms_field = 0.0;
  void collect_timing();
  // every per-call device buffer, once
  template <class F>
  void for_each_buf(F f) {
    DevBuf* list[] = {&rays_o,   &rays_v,      &hit_count,   &hit_off,  &hit_slots,  &hits,       &tile_count,
                      &tile_off, &tile_items,  &tile_masks,  &tile_order, &scan_tmp, &counters,   &slab,
                      &ray_meta, &out_stage,   &exact_stage, &cams_dev, &ray_tr,     &order_keys, &order,
                      &sort_hist, &sort_offs};
    for (DevBuf* b : list) f(*b);
  }
  Workspace() = default;
  Workspace(const Workspace&) = delete;
  Workspace& operator=(const Workspace&) = delete;
  ~Workspace() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

struct Index {
  int64_t n = 0;
  Kernel kernel = Kernel::Cubic;
  int K = 4, D = 2, P = 2, n_lut = 4096;
  double tau = 0, sigma = 0, a_max = 0, h_repr = 0, phi_repr = 0, merge_tol = 0;
  GridDev grid{};
  double cell0 = 0;
  int grid_bits = 1;  // Morton bits per axis in the sort keys
  Table table;
  uint32_t lut_flags = 0;  // table storage precision (SPH_HOA_FLAG_LUT_*), 0: float64
  int trans_axis = -1;     // transverse gradient field along this axis (SPH_HOA_FLAG_TRANSVERSE_*), -1: none
  // device data (Morton order)
  DevBuf pos4;    // float4 x, y, z, h
  DevBuf val;     // float amplitude
  DevBuf orig;    // int32 input index
  DevBuf morton;  // uint64 key (level << 57 | morton)
  DevBuf cell_begin, cell_end;  // uint32 per cell, all levels
  DevBuf lut_theta, lut_shat;   // double
  int lut_fmt = 0;              // field-kernel table format: 0 float64, 1 float32, 2 bfloat16, 3 binary16
  DevBuf lut_theta_n, lut_shat_n;  // the table in that narrower format (lut_fmt > 0)
  DevBuf lut_smid;              // double [n][D+1] jumps at 0 (even K; float variant only)
  DevBuf float_scratch;         // float variant, per work-group
  Workspace ws;  // the index's own per-call state
  hipStream_t last_stream = nullptr;
};

}  // namespace sph

struct sph_hoa_index_s {
  sph::Index ix;
};

namespace sph {

// render server (serve.cpp)
struct Server;
Server* server_create(int64_t hbm_budget, int64_t max_rays, int n_lanes);
void server_destroy(Server* s);
int server_add_index(Server* s, sph_hoa_index idx);
sph_hoa_index server_index(Server* s, int slot);
int64_t server_submit(Server* s, int slot, const sph_hoa_camera* cam, const sph_hoa_tf* tf, float* out);
bool server_wait(Server* s, int64_t id, double timeout_s, double* latency_ms, sph_hoa_status* req_status,
                 std::string* req_error);
void server_stats(Server* s, sph_hoa_server_stats* st);
void server_set_admission(Server* s, int64_t max_queued, int64_t max_request_bytes);
bool server_cancel(Server* s, int64_t id);
void server_pause(Server* s, bool paused);

// render with every per-call buffer in the library's static device scratch (static_scratch.hip)
void render_static(Index& ix, const sph_hoa_camera* cam, const sph_hoa_tf* tf, float* rgba, hipStream_t st);
int64_t static_scratch_bytes();

// table projection on the device (lutproj.hip): theta, shat, smid, err2 device arrays of a table of
// n entries; project_table_device fills T.shat / smid / err2 from T.theta
void lut_project_device(Kernel k, int K, int D, int n, const double* theta, double* shat, double* smid, double* err2,
                        hipStream_t st);
void project_table_device(Table& T, hipStream_t st);

// build (index.hip)
void build_index_device(Index& ix, const float* xyz, const float* h, const float* value, hipStream_t st);
void get_grid_device(Index& ix, uint64_t* morton, int32_t* level, int32_t* order, hipStream_t st);

// per-frame (raycast.hip)
// Hit lists of the first pass, exported as input indices (sph_hoa_camera_hits / sph_hoa_ray_hits).
struct HitsOut {
  int64_t* offsets;  // device [n + 1]
  int32_t* ids;      // device [capacity]
  int64_t capacity;
  int64_t n_pairs;   // out
};

struct FieldOut {
  sph_hoa_field* field;  // approx mode (null for render)
  float* rgba;           // render mode
  const sph_hoa_tf* tf;
  bool exact;
  sph_hoa_float_field* flt = nullptr;  // float accumulation variant (floatpath.hip)
  int n_reinit = 0;
  HitsOut* hits = nullptr;  // stop after the gathering and export the hit lists
};

// float accumulation variant (floatpath.hip)
struct FloatArgs {
  const double *o, *v;
  int64_t n_rays;
  double t_min, t_max;
  const int64_t* hit_off;
  const uint32_t* hits;
  int64_t hit_slots;  // > 0: ray r's hits at hits[r * hit_slots ...]
  const float4* pos4;
  const float* val;
  const int32_t* orig;
  const double *theta, *shat, *smid;
  int n_lut, K, P, even_k, D, n_reinit;
  char* scratch;
  int64_t scratch_stride, cap_h;
  const int64_t* out_off;
  int64_t* out_cnt;
  float *t0, *t1, *coef;
  uint32_t* flags;
};
int64_t float_field_capacity(int64_t total_pairs, int64_t n_rays, int K, int n_reinit);
void launch_float_field(FloatArgs& F, int64_t max_hits, DevBuf& scratch, int64_t* out_off, hipStream_t st);
// n_batch > 0: render the cameras batch[0..n_batch) together (rays concatenated in camera order)
// gathered != nullptr (arbitrary rays only): take the hit lists of gathered's previous call on the
// same rays instead of gathering (the two indices hold the same particles: same_particles)
// workspace: the per-call state to use (null: the index's own); gathered uses its own index's
void run_rays(Index& ix, int64_t n_rays, bool camera, const sph_hoa_camera* cam, const sph_hoa_rays* rays,
              FieldOut& out, hipStream_t st, const sph_hoa_camera* batch = nullptr, int n_batch = 0,
              const Index* gathered = nullptr, Workspace* workspace = nullptr);
// true if a and b hold the same particles in the same order (positions, smoothing lengths and
// input indices bit for bit), so that every ray has the same hit list in both (index.hip)
bool same_particles(const Index& a, const Index& b, hipStream_t st);

// integer bit-length microbenchmark of the accumulation rule (bitlength.hip); host buffers
void accumulate_bits(int bits, int D, const uint32_t* dist, const uint32_t* jumps, int n_table, int64_t n_threads,
                     int steps, uint32_t* out_host, float* ms, hipStream_t st);

// small device utilities (util.hip)
void device_exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, DevBuf& tmp, hipStream_t st);
// device radix sort of n uint64 keys by their low `bits` bits (index.hip); true if the result is in alt
bool device_sort_u64(uint64_t* keys, uint64_t* alt, int64_t n, int bits, DevBuf& hist, DevBuf& offs, DevBuf& tmp,
                     hipStream_t st);

}  // namespace sph
