// Rendering without allocation: every per-call device buffer of sph_hoa_render (rays, hit
// counts and lists, screen-tile lists, sort and scan temporaries, the field kernel's per-work-group
// slabs and counters) is placed in one fixed array of device memory that the library's code object
// holds for the life of the process, so the call makes no hipMalloc / hipFree.
//
// The array's name is a host-side stand-in: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is handed to kernels,
// memsets and copies.  Calls on one device share the array, so calls that overlap on one device
// race; each call clears what it needs (its counters) itself.
#include <hip/hip_runtime.h>

#include <mutex>

#include "impl.h"

namespace sph {
namespace {

constexpr int64_t kStaticScratchBytes = int64_t(128) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kStaticScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on the first call per device)
char* scratch_ptr() {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "device");
  if (dev < 0 || dev >= kMaxDevices) throw Error(SPH_HOA_E_UNSUPPORTED, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "static scratch address");
    if (!p) throw Error(SPH_HOA_E_DEVICE, "static scratch address is null");
    g_ptr[dev] = p;
  }
  return static_cast<char*>(g_ptr[dev]);
}

// Binds the index's per-call buffers to the arena for the lifetime of the guard, then puts the
// index's own allocations back.
struct Bind {
  Index& ix;
  DevBuf* bufs[32];
  void* saved_p[32];
  size_t saved_b[32];
  int n = 0;
  Bind(Index& x, Arena* a) : ix(x) {
    ix.ws.for_each_buf([&](DevBuf& b) {
      bufs[n] = &b;
      saved_p[n] = b.p;
      saved_b[n] = b.bytes;
      b.p = nullptr;
      b.bytes = 0;
      b.arena = a;
      ++n;
    });
    ix.ws.no_alloc = true;
  }
  ~Bind() {
    for (int i = 0; i < n; ++i) {
      bufs[i]->p = saved_p[i];
      bufs[i]->bytes = saved_b[i];
      bufs[i]->arena = nullptr;
    }
    ix.ws.no_alloc = false;
    ix.ws.last_hit_rays = -1;  // no hit lists of this call survive in the index's own buffers
  }
  Bind(const Bind&) = delete;
  Bind& operator=(const Bind&) = delete;
};

}  // namespace

int64_t static_scratch_bytes() { return kStaticScratchBytes; }

void render_static(Index& ix, const sph_hoa_camera* cam, const sph_hoa_tf* tf, float* rgba, hipStream_t st) {
  Arena arena;
  arena.base = scratch_ptr();
  arena.cap = (size_t)kStaticScratchBytes;
  Bind bind(ix, &arena);
  FieldOut fo{nullptr, rgba, tf, false};
  try {
    run_rays(ix, (int64_t)cam->width * cam->height, true, cam, nullptr, fo, st);
  } catch (...) {
    // the arena is reused by the next call on this device: nothing of this call may still run
    (void)hipStreamSynchronize(st);
    throw;
  }
  hip_check(hipStreamSynchronize(st), "sync");
  if (ix.ws.render_stats_pending) {
    // the placement counters live in the arena: read them before it is released
    unsigned long long c[6];
    hip_check(hipMemcpy(c, ix.ws.counters.p, sizeof(c), hipMemcpyDeviceToHost), "copy");
    ix.ws.stats.rays_global = (int64_t)c[3];
    ix.ws.stats.rays_jumps_device = (int64_t)c[4];
    ix.ws.stats.rays_scratch_device = (int64_t)c[5];
    ix.ws.render_stats_pending = false;
  }
}

}  // namespace sph
