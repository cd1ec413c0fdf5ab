// C ABI of the library (include/sph_hoa.h): argument checking, index lifetime,
// table caching and the choice of quanta; device work lives in index.hip and
// raycast.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>

#include "impl.h"

struct sph_hoa_server_s {
  sph::Server* s;
};

namespace {

thread_local std::string g_last_error;

sph_hoa_status fail(sph_hoa_status s, const std::string& m) {
  g_last_error = m;
  return s;
}

template <class F>
sph_hoa_status guarded(F&& f) {
  try {
    g_last_error.clear();
    f();
    return SPH_HOA_OK;
  } catch (const sph::Error& e) {
    return fail(e.status, e.what());
  } catch (const std::bad_alloc&) {
    return fail(SPH_HOA_E_OUT_OF_MEMORY, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(SPH_HOA_E_INTERNAL, e.what());
  }
}

void require(bool ok, const std::string& m) {
  if (!ok) throw sph::Error(SPH_HOA_E_INVALID_ARG, m);
}

int host_threads() {
  const unsigned h = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(h, 32u));
}

// Tables from the library's own optimisation, shared between indices of one process.
std::mutex g_table_mu;
std::map<std::tuple<int, int, int, int>, std::shared_ptr<const sph::Table>> g_tables;

std::shared_ptr<const sph::Table> cached_table(sph::Kernel k, int K, int D, int n) {
  const auto key = std::make_tuple((int)k, K, D, n);
  {
    std::lock_guard<std::mutex> lk(g_table_mu);
    auto it = g_tables.find(key);
    if (it != g_tables.end()) return it->second;
  }
  auto t = std::make_shared<const sph::Table>(sph::build_table(k, K, D, n, nullptr, host_threads()));
  std::lock_guard<std::mutex> lk(g_table_mu);
  g_tables[key] = t;
  return t;
}

sph::Kernel kernel_of(sph_hoa_kernel k) {
  if (k == SPH_HOA_KERNEL_CUBIC) return sph::Kernel::Cubic;
  if (k == SPH_HOA_KERNEL_WENDLAND_C2) return sph::Kernel::Wendland;
  if (k == SPH_HOA_KERNEL_WENDLAND_C4) return sph::Kernel::WendlandC4;
  if (k == SPH_HOA_KERNEL_WENDLAND_C6) return sph::Kernel::WendlandC6;
  if (k == SPH_HOA_KERNEL_WENDLAND_C2_GRAD) return sph::Kernel::WendlandGrad;
  if (k == SPH_HOA_KERNEL_WENDLAND_C4_GRAD) return sph::Kernel::WendlandC4Grad;
  if (k == SPH_HOA_KERNEL_WENDLAND_C6_GRAD) return sph::Kernel::WendlandC6Grad;
  throw sph::Error(SPH_HOA_E_INVALID_ARG, "unknown kernel");
}

void check_method(int K, int D) {
  require(D >= 1 && D <= sph::kMaxD, "degree must be in 1..6");
  require(K >= 1 && K <= 6, "pieces must be in 1..6");
  require((K * D) / 2 >= 1, "K = D = 1 leaves only the zero function");
}

}  // namespace

namespace {
// Float64 -> nearest float32, then for bf16 the nearest value with 8 significant bits (ties to
// even) and for fp16 the nearest IEEE binary16 (the storage formats of the table precision study).
enum class Storage { F32, BF16, F16 };
double round_storage(double x, Storage fmt) {
  const float f = (float)x;
  if (fmt == Storage::F32 || !std::isfinite(f)) return (double)f;
  if (fmt == Storage::F16) return (double)(_Float16)f;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u = (u + 0x7fffu + lsb) & 0xffff0000u;
  float r;
  std::memcpy(&r, &u, 4);
  return (double)r;
}
}  // namespace

extern "C" {

const char* sph_hoa_status_string(sph_hoa_status s) {
  switch (s) {
    case SPH_HOA_OK: return "ok";
    case SPH_HOA_E_INVALID_ARG: return "invalid argument";
    case SPH_HOA_E_OUT_OF_MEMORY: return "out of memory or capacity too small";
    case SPH_HOA_E_OVERFLOW: return "integer range exceeded";
    case SPH_HOA_E_DEVICE: return "device error";
    case SPH_HOA_E_UNSUPPORTED: return "unsupported configuration";
    case SPH_HOA_E_INTERNAL: return "internal invariant failed";
    case SPH_HOA_E_BUSY: return "request queue full";
    case SPH_HOA_E_CANCELLED: return "request cancelled";
  }
  return "unknown status";
}

const char* sph_hoa_last_error(void) { return g_last_error.c_str(); }

sph_hoa_status sph_hoa_build_index(const float* xyz, const float* h, const float* value, int64_t n,
                                   sph_hoa_kernel kernel, const sph_hoa_params* p, void* stream,
                                   sph_hoa_index* out) {
  sph::TraceRange trace_range("sph_hoa_build_index");
  if (!out) return fail(SPH_HOA_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  std::unique_ptr<sph_hoa_index_s> H(new sph_hoa_index_s());
  const sph_hoa_status s = guarded([&]() {
    require(xyz && h && value && p, "NULL argument");
    require(n > 0 && n < (int64_t(1) << 31), "particle count must be in 1..2^31-1");
    const sph::Kernel k = kernel_of(kernel);
    check_method(p->pieces, p->degree);
    const int n_lut = p->lut_entries == 0 ? 4096 : p->lut_entries;
    require(n_lut >= 2 && n_lut <= 65536, "lut_entries must be in 2..65536");
    require(p->int_bits == 0 || p->int_bits == 64, "only 64-bit integers are implemented");
    require(std::isfinite(p->merge_tol) && p->merge_tol >= 0.0, "merge_tol must be finite and >= 0");
    require(std::isfinite(p->a_max) && std::isfinite(p->h_repr) && std::isfinite(p->phi_repr) &&
                std::isfinite(p->tau), "quanta parameters must be finite");
    const uint32_t lut_bits = SPH_HOA_FLAG_LUT_FP32 | SPH_HOA_FLAG_LUT_BF16 | SPH_HOA_FLAG_LUT_FP16;
    const uint32_t trans_bits = SPH_HOA_FLAG_TRANSVERSE_X | SPH_HOA_FLAG_TRANSVERSE_Y | SPH_HOA_FLAG_TRANSVERSE_Z;
    require((p->flags & ~(lut_bits | trans_bits)) == 0,
            "params.flags: only the SPH_HOA_FLAG_LUT_* table precisions and SPH_HOA_FLAG_TRANSVERSE_*");
    const uint32_t lut_flag = p->flags & lut_bits, trans_flag = p->flags & trans_bits;
    require(lut_flag == 0 || lut_flag == SPH_HOA_FLAG_LUT_FP32 || lut_flag == SPH_HOA_FLAG_LUT_BF16 ||
                lut_flag == SPH_HOA_FLAG_LUT_FP16,
            "params.flags: one table precision");
    require(trans_flag == 0 || trans_flag == SPH_HOA_FLAG_TRANSVERSE_X || trans_flag == SPH_HOA_FLAG_TRANSVERSE_Y ||
                trans_flag == SPH_HOA_FLAG_TRANSVERSE_Z,
            "params.flags: one transverse axis");
    sph::Index& ix = H->ix;
    ix.n = n;
    ix.kernel = k;
    ix.K = p->pieces;
    ix.D = p->degree;
    ix.P = (p->pieces + 1) / 2;
    ix.n_lut = n_lut;
    ix.merge_tol = p->merge_tol;
    ix.a_max = p->a_max > 0 ? p->a_max : 0.0;
    ix.trans_axis = trans_flag == SPH_HOA_FLAG_TRANSVERSE_X ? 0
                    : trans_flag == SPH_HOA_FLAG_TRANSVERSE_Y ? 1
                    : trans_flag == SPH_HOA_FLAG_TRANSVERSE_Z ? 2
                                                              : -1;
    ix.h_repr = p->h_repr > 0 ? p->h_repr : 0.0;
    ix.phi_repr = p->phi_repr > 0 ? p->phi_repr : 0.0;
    if (p->knot_table) {
      for (int64_t i = 0; i < (int64_t)n_lut * ix.P; ++i)
        require(std::isfinite(p->knot_table[i]) && p->knot_table[i] > 0.0, "knot_table entries must be > 0");
      for (int i = 0; i < n_lut; ++i)
        for (int m = 1; m < ix.P; ++m)
          require(p->knot_table[i * ix.P + m] > p->knot_table[i * ix.P + m - 1], "knot_table rows must increase");
      ix.table = sph::build_table(k, ix.K, ix.D, n_lut, p->knot_table, host_threads(), false);
    } else {
      ix.table = *cached_table(k, ix.K, ix.D, n_lut);
    }
    // the projection of every entry onto its knots' candidate space, on the device (Sec. 3.3)
    sph::project_table_device(ix.table, (hipStream_t)stream);
    if (p->jump_table) {
      require(p->knot_table != nullptr, "jump_table needs the knot_table it belongs to");
      const int64_t ns = (int64_t)n_lut * ix.P * (ix.D + 1);
      for (int64_t i = 0; i < ns; ++i) require(std::isfinite(p->jump_table[i]), "jump_table entries must be finite");
      ix.table.shat.assign(p->jump_table, p->jump_table + ns);
      const int64_t nm = (int64_t)n_lut * (ix.D + 1);
      if (ix.K % 2 == 0) {
        require(p->jump_table_mid != nullptr, "even K needs jump_table_mid");
        for (int64_t i = 0; i < nm; ++i)
          require(std::isfinite(p->jump_table_mid[i]), "jump_table_mid entries must be finite");
        ix.table.smid.assign(p->jump_table_mid, p->jump_table_mid + nm);
      } else {
        ix.table.smid.assign(nm, 0.0);
      }
    }
    if (lut_flag != 0) {
      const Storage fmt = (lut_flag == SPH_HOA_FLAG_LUT_BF16)   ? Storage::BF16
                          : (lut_flag == SPH_HOA_FLAG_LUT_FP16) ? Storage::F16
                                                                : Storage::F32;
      for (double& x : ix.table.theta) x = round_storage(x, fmt);
      for (double& x : ix.table.shat) x = round_storage(x, fmt);
      for (double& x : ix.table.smid) x = round_storage(x, fmt);
      ix.lut_flags = lut_flag;
    }
    hipStream_t st = (hipStream_t)stream;
    ix.lut_theta.ensure(sizeof(double) * ix.table.theta.size());
    ix.lut_shat.ensure(sizeof(double) * ix.table.shat.size());
    sph::hip_check(hipMemcpyAsync(ix.lut_theta.p, ix.table.theta.data(), sizeof(double) * ix.table.theta.size(),
                                  hipMemcpyHostToDevice, st), "copy");
    sph::hip_check(hipMemcpyAsync(ix.lut_shat.p, ix.table.shat.data(), sizeof(double) * ix.table.shat.size(),
                                  hipMemcpyHostToDevice, st), "copy");
    if (ix.lut_flags != 0) {
      // the field kernel reads the rounded table in its own storage format (every value widens
      // exactly to the rounded float64 kept beside it)
      ix.lut_fmt = (ix.lut_flags == SPH_HOA_FLAG_LUT_FP32) ? 1 : (ix.lut_flags == SPH_HOA_FLAG_LUT_BF16) ? 2 : 3;
      auto narrow = [&](const std::vector<double>& src, sph::DevBuf& dst) {
        const size_t n = src.size();
        if (ix.lut_fmt == 1) {
          std::vector<float> v(n);
          for (size_t i = 0; i < n; ++i) v[i] = (float)src[i];
          dst.ensure(sizeof(float) * std::max<size_t>(1, n));
          sph::hip_check(hipMemcpy(dst.p, v.data(), sizeof(float) * n, hipMemcpyHostToDevice), "copy");
        } else {
          std::vector<uint16_t> v(n);
          for (size_t i = 0; i < n; ++i) {
            const float f = (float)src[i];
            if (ix.lut_fmt == 2) {
              uint32_t u;
              std::memcpy(&u, &f, 4);
              v[i] = (uint16_t)(u >> 16);  // exact: the value already has 8 significant bits
            } else {
              const _Float16 hf = (_Float16)f;  // exact: already a binary16 value
              std::memcpy(&v[i], &hf, 2);
            }
          }
          dst.ensure(sizeof(uint16_t) * std::max<size_t>(1, n));
          sph::hip_check(hipMemcpy(dst.p, v.data(), sizeof(uint16_t) * n, hipMemcpyHostToDevice), "copy");
        }
      };
      narrow(ix.table.theta, ix.lut_theta_n);
      narrow(ix.table.shat, ix.lut_shat_n);
    }
    ix.lut_smid.ensure(sizeof(double) * std::max<size_t>(1, ix.table.smid.size()));
    if (!ix.table.smid.empty())
      sph::hip_check(hipMemcpyAsync(ix.lut_smid.p, ix.table.smid.data(), sizeof(double) * ix.table.smid.size(),
                                    hipMemcpyHostToDevice, st), "copy");
    const bool derived_amax = !(p->a_max > 0);
    sph::build_index_device(ix, xyz, h, value, st);
    // a transverse field's amplitudes are value * m with |m| < q = 2: twice the value bound
    if (ix.trans_axis >= 0 && derived_amax) ix.a_max *= 2.0;
    const double int_max = 9223372036854775807.0;  // 2^63 - 1 (rounds to 2^63 in double)
    if (ix.a_max > 0.0) {
      ix.sigma = ix.a_max / int_max;
    } else {
      ix.sigma = 1.0;  // every amplitude is zero: any quantum represents the zero field
    }
    if (p->tau > 0) {
      ix.tau = p->tau;
    } else if (ix.phi_repr > 0.0) {
      ix.tau = sph::optimal_tau(k, ix.D, ix.sigma, ix.h_repr, ix.phi_repr);
    } else {
      ix.tau = ix.h_repr * 1e-3;
    }
    require(ix.tau > 0.0 && std::isfinite(ix.tau), "could not determine a length quantum");
  });
  if (s != SPH_HOA_OK) return s;
  *out = H.release();
  return SPH_HOA_OK;
}

sph_hoa_status sph_hoa_index_free(sph_hoa_index idx) {
  if (!idx) return fail(SPH_HOA_E_INVALID_ARG, "NULL index");
  return guarded([&]() {
    if (idx->ix.last_stream) (void)hipStreamSynchronize(idx->ix.last_stream);
    delete idx;
  });
}

namespace {

// Output arrays of a field call for n rays; returns whether exact mode is on.
// Knot positions are 64-bit integers (length quanta): the segment, widened by the coarsest cell
// (at least q h_max), must stay within that range.  Inside a ray the kernel handles positions
// relative to the ray's first knot in unsigned 32 bits and reports E_OVERFLOW for a ray whose knots
// span 2^32 quanta or more.
void check_positions(const sph::Index& ix, double t_min, double t_max) {
  const double c = ix.grid.lv[ix.grid.n_levels - 1].c;
  if (!((std::max(std::fabs(t_min), std::fabs(t_max)) + c) / ix.tau < 4.0e18))
    throw sph::Error(SPH_HOA_E_OVERFLOW, "ray positions beyond the 64-bit range of length quanta");
}

bool check_field_out(const sph::Index& ix, const sph_hoa_field* out, int64_t n, uint32_t flags) {
  require(out->capacity >= 0, "capacity must be >= 0");
  if (n > 0) {
    require(out->ray_offsets && out->ray_peak, "NULL output arrays");
    require(out->capacity == 0 || (out->t_start && out->t_end && out->coef), "NULL piece arrays");
  }
  const bool exact = (flags & SPH_HOA_FLAG_EXACT) != 0;
  if (exact && ix.n >= (int64_t(1) << 29))
    throw sph::Error(SPH_HOA_E_UNSUPPORTED, "exact mode needs fewer than 2^29 particles");
  if (exact && n > 0) {
    require(out->exact_offsets && out->knot_offsets, "exact mode needs offset arrays");
    require(out->exact_capacity == 0 || (out->exact_t && out->exact_end && out->exact_coef), "exact arrays");
    require(out->knot_capacity == 0 || (out->knot_t && out->knot_pid && out->knot_kidx), "knot arrays");
  }
  return exact;
}

// One field of sph_hoa_approx_rays; gathered: the index whose call on the same rays just gathered
// the hits (shared gathering) or nullptr.
void approx_rays_one(sph_hoa_index idx, const sph_hoa_rays* rays, sph_hoa_field* out, uint32_t flags, void* stream,
                     const sph::Index* gathered) {
  require(idx && rays && out, "NULL argument");
  require(flags == 0 || flags == SPH_HOA_FLAG_EXACT, "unknown flags");
  require(rays->n >= 0 && rays->n < (int64_t(1) << 31), "ray count must be in 0..2^31-1");
  require(std::isfinite(rays->t_min) && std::isfinite(rays->t_max) && rays->t_min < rays->t_max,
          "need finite t_min < t_max");
  if (rays->n > 0) require(rays->origin && rays->dir, "NULL ray arrays");
  const bool exact = check_field_out(idx->ix, out, rays->n, flags);
  sph::Index& ix = idx->ix;
  check_positions(ix, (double)rays->t_min, (double)rays->t_max);
  sph::FieldOut fo{out, nullptr, nullptr, exact};
  hipStream_t st = (hipStream_t)stream;
  ix.last_stream = st;
  if (rays->n == 0) {
    out->n_pieces = out->n_pairs = out->n_knots = out->n_exact_pieces = 0;
    if (out->ray_offsets) {
      const int64_t z = 0;
      sph::hip_check(hipMemcpyAsync(out->ray_offsets, &z, 8, hipMemcpyHostToDevice, st), "copy");
      sph::hip_check(hipStreamSynchronize(st), "sync");
    }
    return;
  }
  sph::run_rays(ix, rays->n, false, nullptr, rays, fo, st, nullptr, 0, gathered);
}

}  // namespace

sph_hoa_status sph_hoa_approx_rays(sph_hoa_index idx, const sph_hoa_rays* rays, sph_hoa_field* out, uint32_t flags,
                                   void* stream) {
  sph::TraceRange trace_range("sph_hoa_approx_rays");
  return guarded([&]() { approx_rays_one(idx, rays, out, flags, stream, nullptr); });
}

sph_hoa_status sph_hoa_approx_rays_shared(const sph_hoa_index* idx, int32_t n_idx, const sph_hoa_rays* rays,
                                          sph_hoa_field* out, uint32_t flags, void* stream) {
  sph::TraceRange trace_range("sph_hoa_approx_rays_shared");
  return guarded([&]() {
    require(idx && out && rays, "NULL argument");
    require(n_idx >= 1, "need at least one index");
    for (int32_t i = 0; i < n_idx; ++i) require(idx[i] != nullptr, "NULL index");
    hipStream_t st = (hipStream_t)stream;
    for (int32_t i = 1; i < n_idx; ++i)
      require(sph::same_particles(idx[0]->ix, idx[i]->ix, st),
              "shared gathering needs indices of the same particles (positions, smoothing lengths, order)");
    approx_rays_one(idx[0], rays, &out[0], flags, stream, nullptr);
    for (int32_t i = 1; i < n_idx; ++i)
      approx_rays_one(idx[i], rays, &out[i], flags, stream, rays->n > 0 ? &idx[0]->ix : nullptr);
  });
}

sph_hoa_status sph_hoa_float_rays(sph_hoa_index idx, const sph_hoa_rays* rays, int32_t n_reinit,
                                  sph_hoa_float_field* out, void* stream) {
  sph::TraceRange trace_range("sph_hoa_float_rays");
  return guarded([&]() {
    require(idx && rays && out, "NULL argument");
    require(rays->n >= 0 && rays->n < (int64_t(1) << 31), "ray count must be in 0..2^31-1");
    require(std::isfinite(rays->t_min) && std::isfinite(rays->t_max) && rays->t_min < rays->t_max,
            "need finite t_min < t_max");
    require(n_reinit >= 0 && n_reinit <= 1024, "n_reinit must be in 0..1024");
    require(out->capacity >= 0, "capacity must be >= 0");
    if (rays->n > 0) {
      require(rays->origin && rays->dir, "NULL ray arrays");
      require(out->ray_offsets && out->ray_counts, "NULL output arrays");
      require(out->capacity == 0 || (out->t_start && out->t_end && out->coef), "NULL piece arrays");
    }
    sph::Index& ix = idx->ix;
    require(ix.n < (int64_t(1) << 29), "the float variant needs fewer than 2^29 particles");
    hipStream_t st = (hipStream_t)stream;
    ix.last_stream = st;
    out->n_slots = out->n_pairs = 0;
    if (rays->n == 0) {
      if (out->ray_offsets) {
        const int64_t z = 0;
        sph::hip_check(hipMemcpyAsync(out->ray_offsets, &z, 8, hipMemcpyHostToDevice, st), "copy");
        sph::hip_check(hipStreamSynchronize(st), "sync");
      }
      return;
    }
    sph::FieldOut fo{nullptr, nullptr, nullptr, false};
    fo.flt = out;
    fo.n_reinit = n_reinit;
    sph::run_rays(ix, rays->n, false, nullptr, rays, fo, st);
  });
}

namespace {

void check_camera(const sph::Index& ix, const sph_hoa_camera* cam, const sph_hoa_tf* tf) {
  require(cam->width > 0 && cam->height > 0 && (int64_t)cam->width * cam->height < (int64_t(1) << 31),
          "bad image size");
  require(std::isfinite(cam->t_min) && std::isfinite(cam->t_max) && cam->t_min < cam->t_max,
          "need finite t_min < t_max");
  for (int k = 0; k < 3; ++k)
    require(std::isfinite(cam->eye[k]) && std::isfinite(cam->look_at[k]) && std::isfinite(cam->up[k]),
            "camera vectors must be finite");
  if (cam->ortho)
    require(std::isfinite(cam->ortho_half_extent) && cam->ortho_half_extent > 0, "ortho_half_extent must be > 0");
  else
    require(cam->fov_y_deg > 0 && cam->fov_y_deg < 180, "fov_y_deg must be in (0, 180)");
  const double fx = (double)cam->look_at[0] - cam->eye[0], fy = (double)cam->look_at[1] - cam->eye[1],
               fz = (double)cam->look_at[2] - cam->eye[2];
  const double cx = fy * cam->up[2] - fz * cam->up[1], cy = fz * cam->up[0] - fx * cam->up[2],
               cz = fx * cam->up[1] - fy * cam->up[0];
  require(fx * fx + fy * fy + fz * fz > 0 && cx * cx + cy * cy + cz * cz > 0, "degenerate camera frame");
  if (tf)
    require(((double)cam->t_max - (double)cam->t_min) / (double)tf->step < 1073741824.0,
            "step too small: more than 2^30 samples per ray");
  check_positions(ix, (double)cam->t_min, (double)cam->t_max);
}

void check_tf(const sph_hoa_tf* tf) {
  require(tf->rgba && tf->n >= 2, "transfer function needs >= 2 control points");
  require(std::isfinite(tf->v_min) && std::isfinite(tf->v_max) && tf->v_max > tf->v_min, "need v_min < v_max");
  require(std::isfinite(tf->step) && tf->step > 0, "step must be > 0");
}

}  // namespace

sph_hoa_status sph_hoa_render(sph_hoa_index idx, const sph_hoa_camera* cam, const sph_hoa_tf* tf, float* rgba_out,
                              void* stream) {
  sph::TraceRange trace_range("sph_hoa_render");
  return guarded([&]() {
    require(idx && cam && tf && rgba_out, "NULL argument");
    sph::Index& ix = idx->ix;
    check_tf(tf);
    check_camera(ix, cam, tf);
    hipStream_t st = (hipStream_t)stream;
    ix.last_stream = st;
    sph::FieldOut fo{nullptr, rgba_out, tf, false};
    sph::run_rays(ix, (int64_t)cam->width * cam->height, true, cam, nullptr, fo, st);
  });
}

sph_hoa_status sph_hoa_render_static(sph_hoa_index idx, const sph_hoa_camera* cam, const sph_hoa_tf* tf,
                                     float* rgba_out, void* stream) {
  sph::TraceRange trace_range("sph_hoa_render_static");
  return guarded([&]() {
    require(idx && cam && tf && rgba_out, "NULL argument");
    sph::Index& ix = idx->ix;
    check_tf(tf);
    check_camera(ix, cam, tf);
    hipStream_t st = (hipStream_t)stream;
    ix.last_stream = st;
    sph::render_static(ix, cam, tf, rgba_out, st);
  });
}

int64_t sph_hoa_static_scratch_bytes(void) { return sph::static_scratch_bytes(); }

int64_t sph_hoa_device_alloc_count(void) { return sph::g_device_allocs.load(); }

sph_hoa_status sph_hoa_approx_camera(sph_hoa_index idx, const sph_hoa_camera* cam, sph_hoa_field* out, uint32_t flags,
                                     void* stream) {
  sph::TraceRange trace_range("sph_hoa_approx_camera");
  return guarded([&]() {
    require(idx && cam && out, "NULL argument");
    require(flags == 0 || flags == SPH_HOA_FLAG_EXACT, "unknown flags");
    sph::Index& ix = idx->ix;
    check_camera(ix, cam, nullptr);
    const int64_t n = (int64_t)cam->width * cam->height;
    const bool exact = check_field_out(ix, out, n, flags);
    hipStream_t st = (hipStream_t)stream;
    ix.last_stream = st;
    sph::FieldOut fo{out, nullptr, nullptr, exact};
    sph::run_rays(ix, n, true, cam, nullptr, fo, st);
  });
}

namespace {
void check_hits_out(int64_t n, const int64_t* offsets, const int32_t* ids, int64_t capacity, const int64_t* n_pairs) {
  require(n_pairs != nullptr, "NULL n_pairs");
  require(capacity >= 0, "capacity must be >= 0");
  require(n == 0 || offsets != nullptr, "NULL hit_offsets");
  require(capacity == 0 || ids != nullptr, "NULL hit_ids");
}
}  // namespace

sph_hoa_status sph_hoa_camera_hits(sph_hoa_index idx, const sph_hoa_camera* cam, int64_t* hit_offsets,
                                   int32_t* hit_ids, int64_t capacity, int64_t* n_pairs, void* stream) {
  sph::TraceRange trace_range("sph_hoa_camera_hits");
  if (n_pairs) *n_pairs = 0;
  sph::HitsOut ho{hit_offsets, hit_ids, capacity, 0};
  const sph_hoa_status s = guarded([&]() {
    require(idx && cam, "NULL argument");
    sph::Index& ix = idx->ix;
    check_camera(ix, cam, nullptr);
    const int64_t n = (int64_t)cam->width * cam->height;
    check_hits_out(n, hit_offsets, hit_ids, capacity, n_pairs);
    hipStream_t st = (hipStream_t)stream;
    ix.last_stream = st;
    sph::FieldOut fo{nullptr, nullptr, nullptr, false};
    fo.hits = &ho;
    sph::run_rays(ix, n, true, cam, nullptr, fo, st);
  });
  if (n_pairs) *n_pairs = ho.n_pairs;
  return s;
}

sph_hoa_status sph_hoa_ray_hits(sph_hoa_index idx, const sph_hoa_rays* rays, int64_t* hit_offsets, int32_t* hit_ids,
                                int64_t capacity, int64_t* n_pairs, void* stream) {
  sph::TraceRange trace_range("sph_hoa_ray_hits");
  if (n_pairs) *n_pairs = 0;
  sph::HitsOut ho{hit_offsets, hit_ids, capacity, 0};
  const sph_hoa_status s = guarded([&]() {
    require(idx && rays, "NULL argument");
    require(rays->n >= 0 && rays->n < (int64_t(1) << 31), "ray count must be in 0..2^31-1");
    require(std::isfinite(rays->t_min) && std::isfinite(rays->t_max) && rays->t_min < rays->t_max,
            "need finite t_min < t_max");
    if (rays->n > 0) require(rays->origin && rays->dir, "NULL ray arrays");
    check_hits_out(rays->n, hit_offsets, hit_ids, capacity, n_pairs);
    sph::Index& ix = idx->ix;
    hipStream_t st = (hipStream_t)stream;
    ix.last_stream = st;
    if (rays->n == 0) {
      if (hit_offsets) {
        const int64_t z = 0;
        sph::hip_check(hipMemcpyAsync(hit_offsets, &z, 8, hipMemcpyHostToDevice, st), "copy");
        sph::hip_check(hipStreamSynchronize(st), "sync");
      }
      return;
    }
    sph::FieldOut fo{nullptr, nullptr, nullptr, false};
    fo.hits = &ho;
    sph::run_rays(ix, rays->n, false, nullptr, rays, fo, st);
  });
  if (n_pairs) *n_pairs = ho.n_pairs;
  return s;
}

sph_hoa_status sph_hoa_render_batch(sph_hoa_index idx, const sph_hoa_camera* cams, int32_t n_cams,
                                    const sph_hoa_tf* tf, float* rgba_out, void* stream) {
  sph::TraceRange trace_range("sph_hoa_render_batch");
  return guarded([&]() {
    require(idx && tf && (n_cams == 0 || (cams && rgba_out)), "NULL argument");
    require(n_cams >= 0 && n_cams <= (1 << 20), "n_cams must be in [0, 2^20]");
    sph::Index& ix = idx->ix;
    check_tf(tf);
    int64_t n = 0;
    for (int32_t c = 0; c < n_cams; ++c) {
      check_camera(ix, &cams[c], tf);
      n += (int64_t)cams[c].width * cams[c].height;
    }
    require(n < (int64_t(1) << 32), "more than 2^32 rays in one batch");
    hipStream_t st = (hipStream_t)stream;
    ix.last_stream = st;
    if (n == 0) return;
    sph::FieldOut fo{nullptr, rgba_out, tf, false};
    sph::run_rays(ix, n, false, nullptr, nullptr, fo, st, cams, n_cams);
  });
}

sph_hoa_status sph_hoa_index_get_info(sph_hoa_index idx, sph_hoa_index_info* info) {
  return guarded([&]() {
    require(idx && info, "NULL argument");
    const sph::Index& ix = idx->ix;
    std::memset(info, 0, sizeof(*info));
    info->n_particles = ix.n;
    info->kernel = (int)ix.kernel;
    info->degree = ix.D;
    info->pieces = ix.K;
    info->lut_entries = ix.n_lut;
    info->tau = ix.tau;
    info->sigma = ix.sigma;
    info->a_max = ix.a_max;
    info->h_repr = ix.h_repr;
    info->phi_repr = ix.phi_repr;
    for (int a = 0; a < 3; ++a) info->grid_lo[a] = ix.grid.lo[a];
    info->cell0 = ix.cell0;
    info->n_levels = ix.grid.n_levels;
    for (int l = 0; l < ix.grid.n_levels; ++l)
      for (int a = 0; a < 3; ++a) info->level_dims[l][a] = ix.grid.lv[l].n[a];
    info->lut_flags = ix.lut_flags;
  });
}

sph_hoa_status sph_hoa_index_get_lut(sph_hoa_index idx, double* theta, double* shat, double* smid) {
  return guarded([&]() {
    require(idx, "NULL index");
    const sph::Table& t = idx->ix.table;
    if (theta) std::memcpy(theta, t.theta.data(), sizeof(double) * t.theta.size());
    if (shat) std::memcpy(shat, t.shat.data(), sizeof(double) * t.shat.size());
    if (smid) std::memcpy(smid, t.smid.data(), sizeof(double) * t.smid.size());
  });
}

sph_hoa_status sph_hoa_index_get_grid(sph_hoa_index idx, uint64_t* morton, int32_t* level, int32_t* order,
                                      void* stream) {
  return guarded([&]() {
    require(idx, "NULL index");
    sph::get_grid_device(idx->ix, morton, level, order, (hipStream_t)stream);
  });
}

sph_hoa_status sph_hoa_index_get_stats(sph_hoa_index idx, sph_hoa_stats* stats) {
  return guarded([&]() {
    require(idx && stats, "NULL argument");
    sph::Index& ix = idx->ix;
    if (ix.last_stream) sph::hip_check(hipStreamSynchronize(ix.last_stream), "sync");
    ix.ws.collect_timing();
    ix.ws.tuner.collect();
    if (ix.ws.render_stats_pending) {
      // a render does not wait for its kernels; its placement counters are read back here
      unsigned long long c[6];
      sph::hip_check(hipMemcpy(c, ix.ws.counters.p, sizeof(c), hipMemcpyDeviceToHost), "copy");
      ix.ws.stats.rays_global = (int64_t)c[3];
      ix.ws.stats.rays_jumps_device = (int64_t)c[4];
      ix.ws.stats.rays_scratch_device = (int64_t)c[5];
      ix.ws.render_stats_pending = false;
    }
    *stats = ix.ws.stats;
    stats->timed_calls = idx->ix.ws.timed_calls;
    stats->ms_gather = idx->ix.ws.ms_gather;
    stats->ms_field = idx->ix.ws.ms_field;
  });
}

sph_hoa_status sph_hoa_index_set_timing(sph_hoa_index idx, int32_t on) {
  return guarded([&]() {
    require(idx, "NULL index");
    sph::Index& ix = idx->ix;
    if (ix.last_stream) sph::hip_check(hipStreamSynchronize(ix.last_stream), "sync");
    ix.ws.collect_timing();
    if (on)
      for (auto& e : ix.ws.ev)
        if (!e) sph::hip_check(hipEventCreate(&e), "event create");
    ix.ws.timing = on != 0;
    ix.ws.timed_calls = 0;
    ix.ws.ms_gather = ix.ws.ms_field = 0.0;
  });
}

sph_hoa_status sph_hoa_optimal_knots(sph_hoa_kernel kernel, int32_t pieces, int32_t degree, double lambda,
                                     double* theta_out, double* err2_out) {
  return guarded([&]() {
    require(theta_out && err2_out, "NULL argument");
    check_method(pieces, degree);
    require(lambda >= 0.0 && lambda < sph::kSupport, "lambda must be in [0, q)");
    const sph::Kernel k = kernel_of(kernel);
    sph::optimal_knots(k, pieces, degree, lambda, sph::default_starts((pieces + 1) / 2), theta_out, err2_out);
  });
}

sph_hoa_status sph_hoa_knot_table(sph_hoa_kernel kernel, int32_t pieces, int32_t degree, int32_t n,
                                  double* theta_out, double* err2_out) {
  sph::TraceRange trace_range("sph_hoa_knot_table");
  return guarded([&]() {
    require(theta_out, "NULL argument");
    check_method(pieces, degree);
    require(n >= 2 && n <= 65536, "n must be in 2..65536");
    auto t = cached_table(kernel_of(kernel), pieces, degree, n);
    std::memcpy(theta_out, t->theta.data(), sizeof(double) * t->theta.size());
    if (err2_out) std::memcpy(err2_out, t->err2.data(), sizeof(double) * t->err2.size());
  });
}

sph_hoa_status sph_hoa_lut_coefficients(sph_hoa_kernel kernel, int32_t pieces, int32_t degree, int32_t n,
                                        const double* theta, double* shat_out, double* smid_out, double* err2_out) {
  sph::TraceRange trace_range("sph_hoa_lut_coefficients");
  return guarded([&]() {
    require(theta && shat_out, "NULL argument");
    check_method(pieces, degree);
    require(n >= 2 && n <= 65536, "n must be in 2..65536");
    const int P = (pieces + 1) / 2;
    for (int64_t i = 0; i < (int64_t)n * P; ++i) require(std::isfinite(theta[i]) && theta[i] > 0, "theta must be > 0");
    sph::Table t = sph::build_table(kernel_of(kernel), pieces, degree, n, theta, host_threads());
    std::memcpy(shat_out, t.shat.data(), sizeof(double) * t.shat.size());
    if (smid_out) std::memcpy(smid_out, t.smid.data(), sizeof(double) * t.smid.size());
    if (err2_out) std::memcpy(err2_out, t.err2.data(), sizeof(double) * t.err2.size());
  });
}

sph_hoa_status sph_hoa_lut_project(sph_hoa_kernel kernel, int32_t pieces, int32_t degree, int32_t n,
                                   const double* theta, double* shat_out, double* smid_out, double* err2_out,
                                   void* stream) {
  sph::TraceRange trace_range("sph_hoa_lut_project");
  return guarded([&]() {
    require(theta && shat_out && smid_out && err2_out, "NULL argument");
    check_method(pieces, degree);
    require(n >= 2 && n <= 65536, "n must be in 2..65536");
    sph::lut_project_device(kernel_of(kernel), pieces, degree, n, theta, shat_out, smid_out, err2_out,
                            static_cast<hipStream_t>(stream));
  });
}

sph_hoa_status sph_hoa_optimal_tau(sph_hoa_kernel kernel, int32_t degree, double sigma, double h_repr,
                                   double phi_repr, double* tau_out) {
  return guarded([&]() {
    require(tau_out, "NULL argument");
    require(degree >= 1 && degree <= sph::kMaxD, "degree must be in 1..6");
    require(sigma > 0 && h_repr > 0 && phi_repr > 0, "sigma, h_repr, phi_repr must be > 0");
    *tau_out = sph::optimal_tau(kernel_of(kernel), degree, sigma, h_repr, phi_repr);
  });
}

sph_hoa_status sph_hoa_accumulate_bits(int32_t bits, int32_t degree, const uint32_t* dist, const uint32_t* jumps,
                                       int32_t n_table, int64_t n_threads, int32_t steps, uint32_t* out_host,
                                       float* ms_out, void* stream) {
  sph::TraceRange trace_range("sph_hoa_accumulate_bits");
  return guarded([&]() {
    require(dist && jumps, "NULL argument");
    sph::accumulate_bits(bits, degree, dist, jumps, n_table, n_threads, steps, out_host, ms_out,
                         static_cast<hipStream_t>(stream));
  });
}

}  // extern "C"

sph_hoa_status sph_hoa_server_create_lanes(int64_t hbm_budget_bytes, int64_t max_batch_rays, int32_t n_lanes,
                                           sph_hoa_server* out) {
  return guarded([&]() {
    require(out != nullptr, "NULL argument");
    require(hbm_budget_bytes > 0 && max_batch_rays > 0, "budget and max_batch_rays must be > 0");
    require(n_lanes >= 1 && n_lanes <= 16, "n_lanes must be in 1..16");
    *out = nullptr;
    std::unique_ptr<sph_hoa_server_s> h(new sph_hoa_server_s{nullptr});
    h->s = sph::server_create(hbm_budget_bytes, max_batch_rays, n_lanes);
    *out = h.release();
  });
}

sph_hoa_status sph_hoa_server_create(int64_t hbm_budget_bytes, int64_t max_batch_rays, sph_hoa_server* out) {
  return sph_hoa_server_create_lanes(hbm_budget_bytes, max_batch_rays, 2, out);
}

sph_hoa_status sph_hoa_server_add_index(sph_hoa_server server, sph_hoa_index idx, int32_t* slot) {
  return guarded([&]() {
    require(server && idx && slot, "NULL argument");
    *slot = sph::server_add_index(server->s, idx);
  });
}

sph_hoa_status sph_hoa_server_submit(sph_hoa_server server, int32_t slot, const sph_hoa_camera* cam,
                                     const sph_hoa_tf* tf, float* rgba_out, int64_t* request_id) {
  return guarded([&]() {
    require(server && cam && tf && rgba_out && request_id, "NULL argument");
    check_tf(tf);
    check_camera(sph::server_index(server->s, slot)->ix, cam, tf);
    *request_id = sph::server_submit(server->s, slot, cam, tf, rgba_out);
  });
}

sph_hoa_status sph_hoa_server_wait(sph_hoa_server server, int64_t request_id, double timeout_s, int32_t* done,
                                   double* latency_ms) {
  return guarded([&]() {
    require(server && done, "NULL argument");
    *done = 0;
    sph_hoa_status rs = SPH_HOA_OK;
    std::string re;
    if (!sph::server_wait(server->s, request_id, timeout_s, latency_ms, &rs, &re)) return;
    *done = 1;
    if (rs != SPH_HOA_OK) throw sph::Error(rs, "request failed: " + re);
  });
}

sph_hoa_status sph_hoa_server_set_admission(sph_hoa_server server, int64_t max_queued, int64_t max_request_bytes) {
  return guarded([&]() {
    require(server != nullptr, "NULL argument");
    require(max_queued >= 0 && max_request_bytes >= 0, "limits must be >= 0");
    sph::server_set_admission(server->s, max_queued, max_request_bytes);
  });
}

sph_hoa_status sph_hoa_server_pause(sph_hoa_server server, int32_t paused) {
  return guarded([&]() {
    require(server != nullptr, "NULL argument");
    sph::server_pause(server->s, paused != 0);
  });
}

sph_hoa_status sph_hoa_server_cancel(sph_hoa_server server, int64_t request_id, int32_t* cancelled) {
  return guarded([&]() {
    require(server && cancelled, "NULL argument");
    *cancelled = 0;
    *cancelled = sph::server_cancel(server->s, request_id) ? 1 : 0;
  });
}

sph_hoa_status sph_hoa_server_get_stats(sph_hoa_server server, sph_hoa_server_stats* stats) {
  return guarded([&]() {
    require(server && stats, "NULL argument");
    sph::server_stats(server->s, stats);
  });
}

sph_hoa_status sph_hoa_server_destroy(sph_hoa_server server) {
  return guarded([&]() {
    if (!server) return;
    sph::server_destroy(server->s);
    delete server;
  });
}
