// Render server: resident indices, a request queue and continuous batching.
//
// Requests (one camera each) are queued by any host thread, subject to admission limits (queue
// length, one request's estimated memory); a queued request can be cancelled.  The server runs
// several lanes, each a worker thread with its own stream and per-call device state.  A free lane
// takes the oldest request as soon as its estimated transient device memory fits in what the
// batches already in flight leave of the budget (or nothing is in flight), adds the queued
// requests with the same index and transfer function in arrival order while the batch stays
// within the remaining budget and the ray bound, renders the batch with one batched launch chain
// (run_rays over all its cameras) and copies each image to its request's output.  Requests that
// arrive while batches run are admitted by the next free lane as memory is returned, so their work
// overlaps the running batches on the device.  Every image is bit-identical to sph_hoa_render of
// the same camera alone (each ray is computed exactly as the single path does, whatever batch or
// lane carries it).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "impl.h"

namespace sph {
namespace {

// Field-kernel launches per batch on a lane that shares the device with other lanes: a batch that
// arrives while another lane's field kernel runs gets compute units within about 1/8 of that
// kernel's time.
constexpr int kLaneTimeSlices = 8;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  int64_t id = 0;
  int slot = 0;
  sph_hoa_camera cam{};
  sph_hoa_tf tf{};
  float* out = nullptr;
  double t_submit = 0.0, t_done = 0.0;
  bool done = false;
  sph_hoa_status status = SPH_HOA_OK;
  std::string error;
};

bool same_tf(const sph_hoa_tf& a, const sph_hoa_tf& b) {
  return a.rgba == b.rgba && a.n == b.n && a.v_min == b.v_min && a.v_max == b.v_max && a.step == b.step;
}

}  // namespace

struct Server;

// One worker with its own stream, per-call device state and image staging.
struct Lane {
  Server* srv = nullptr;
  hipStream_t stream = nullptr;
  Workspace ws;
  DevBuf staging;
  std::thread worker;
};

struct Server {
  int64_t budget = 0, max_rays = 0;
  std::vector<sph_hoa_index> indices;
  std::vector<double> hits_per_ray;  // running estimate per index (admission)
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<int64_t, std::shared_ptr<Request>> live;
  int64_t next_id = 1;
  bool stop = false, paused = false;
  std::vector<std::unique_ptr<Lane>> lanes;
  int64_t in_flight_bytes = 0;  // estimated device memory of the batches being rendered
  int in_flight = 0;            // batches being rendered
  // statistics
  std::vector<double> latencies_ms;
  int64_t completed = 0, failed = 0, batches = 0, pairs = 0, rays = 0, rejected = 0, cancelled = 0;
  int64_t overlapped = 0;  // batches that started while another batch was being rendered
  int max_in_flight = 0;
  // admission limits (0: none)
  int64_t max_queued = 0, max_request_bytes = 0;
  double busy_s = 0.0;

  // device bytes of one request's transient buffers, from the index's hits-per-ray estimate
  int64_t estimate_bytes(int slot, const sph_hoa_camera& c) const {
    const int64_t n = (int64_t)c.width * c.height;
    const double hpr = std::max(1.0, hits_per_ray[slot]);
    const int64_t tiles = (int64_t)((c.width + 7) / 8) * ((c.height + 7) / 8);
    // rays (o, v, segment), counts/offsets, image, hit lists, tile lists (about one entry per hit)
    return n * (48 + 8 + 16 + 16) + (int64_t)(n * hpr * 8.0) + tiles * 24;
  }

  // the oldest request may start: it fits in what the running batches leave of the budget, or
  // nothing runs (a request larger than the budget then runs alone)
  bool head_admissible() const {
    if (queue.empty()) return false;
    const Request& h = *queue.front();
    return in_flight == 0 || in_flight_bytes + estimate_bytes(h.slot, h.cam) <= budget;
  }

  void run(Lane& lane) {
    for (;;) {
      std::vector<std::shared_ptr<Request>> batch;
      sph_hoa_index index = nullptr;
      int64_t bytes = 0;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return (stop && queue.empty()) || ((stop || !paused) && head_admissible()); });
        if (queue.empty()) return;  // stop requested and drained (a stop overrides a pause)
        // oldest request first; then compatible requests in arrival order within what is left
        const std::shared_ptr<Request> head = queue.front();
        queue.pop_front();
        batch.push_back(head);
        index = indices[head->slot];
        bytes = estimate_bytes(head->slot, head->cam);
        const int64_t left = std::max<int64_t>(budget - in_flight_bytes, bytes);
        int64_t nr = (int64_t)head->cam.width * head->cam.height;
        for (auto it = queue.begin(); it != queue.end();) {
          const Request& q = **it;
          const int64_t b = estimate_bytes(q.slot, q.cam);
          const int64_t r = (int64_t)q.cam.width * q.cam.height;
          if (q.slot == head->slot && same_tf(q.tf, head->tf) && bytes + b <= left && nr + r <= max_rays) {
            bytes += b;
            nr += r;
            batch.push_back(*it);
            it = queue.erase(it);
          } else {
            ++it;
          }
        }
        if (in_flight > 0) ++overlapped;
        ++in_flight;
        max_in_flight = std::max(max_in_flight, in_flight);
        in_flight_bytes += bytes;
      }
      render(lane, index, batch);
      {
        std::lock_guard<std::mutex> lk(mu);
        --in_flight;
        in_flight_bytes -= bytes;
      }
      cv_work.notify_all();  // memory returned: another lane may admit the next request
    }
  }

  void render(Lane& lane, sph_hoa_index index, std::vector<std::shared_ptr<Request>>& batch) {
    const double t0 = now_s();
    sph_hoa_status st = SPH_HOA_OK;
    std::string err;
    int64_t n_pairs = 0, n_rays = 0;
    try {
      std::vector<sph_hoa_camera> cams;
      for (auto& r : batch) {
        cams.push_back(r->cam);
        n_rays += (int64_t)r->cam.width * r->cam.height;
      }
      Index& ix = index->ix;
      lane.staging.ensure(sizeof(float) * 4 * (size_t)n_rays);
      FieldOut fo{nullptr, lane.staging.as<float>(), &batch[0]->tf, false};
      run_rays(ix, n_rays, false, nullptr, nullptr, fo, lane.stream, cams.data(), (int)cams.size(), nullptr,
               &lane.ws);
      int64_t off = 0;
      for (auto& r : batch) {
        const int64_t n = (int64_t)r->cam.width * r->cam.height;
        hip_check(hipMemcpyAsync(r->out, lane.staging.as<float>() + 4 * off, sizeof(float) * 4 * (size_t)n,
                                 hipMemcpyDeviceToDevice, lane.stream),
                  "copy");
        off += n;
      }
      hip_check(hipStreamSynchronize(lane.stream), "sync");
      n_pairs = lane.ws.stats.n_pairs;
    } catch (const Error& e) {
      st = e.status;
      err = e.what();
    } catch (const std::exception& e) {
      st = SPH_HOA_E_INTERNAL;
      err = e.what();
    }
    const double t1 = now_s();
    std::lock_guard<std::mutex> lk(mu);
    busy_s += t1 - t0;
    ++batches;
    if (st == SPH_HOA_OK && n_rays > 0) {
      const int slot = batch[0]->slot;
      const double hpr = (double)n_pairs / (double)n_rays;
      hits_per_ray[slot] = hits_per_ray[slot] <= 0.0 ? hpr : 0.5 * (hits_per_ray[slot] + hpr);
      pairs += n_pairs;
      rays += n_rays;
    }
    for (auto& r : batch) {
      r->t_done = t1;
      r->done = true;
      r->status = st;
      r->error = err;
      if (st == SPH_HOA_OK) {
        ++completed;
        latencies_ms.push_back((r->t_done - r->t_submit) * 1e3);
      } else {
        ++failed;
      }
    }
    cv_done.notify_all();
  }
};

Server* server_create(int64_t hbm_budget, int64_t max_rays, int n_lanes) {
  std::unique_ptr<Server> s(new Server);
  s->budget = hbm_budget;
  s->max_rays = max_rays;
  for (int i = 0; i < n_lanes; ++i) {
    std::unique_ptr<Lane> l(new Lane);
    l->srv = s.get();
    hip_check(hipStreamCreateWithFlags(&l->stream, hipStreamNonBlocking), "stream");
    if (n_lanes > 1) l->ws.time_slices = kLaneTimeSlices;
    // growing a lane's buffers must not wait for the other lanes' work (hipFree would)
    l->ws.for_each_buf([](DevBuf& b) { b.defer = true; });
    l->staging.defer = true;
    s->lanes.push_back(std::move(l));
  }
  for (auto& l : s->lanes) {
    Lane* lp = l.get();
    Server* raw = s.get();
    l->worker = std::thread([raw, lp] { raw->run(*lp); });
  }
  return s.release();
}

void server_destroy(Server* s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& l : s->lanes) l->worker.join();  // the lanes drain the queue first
  for (auto& l : s->lanes) (void)hipStreamDestroy(l->stream);
  delete s;
}

int server_add_index(Server* s, sph_hoa_index idx) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->indices.push_back(idx);
  s->hits_per_ray.push_back(-1.0);
  return (int)s->indices.size() - 1;
}

sph_hoa_index server_index(Server* s, int slot) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (slot < 0 || slot >= (int)s->indices.size()) throw Error(SPH_HOA_E_INVALID_ARG, "unknown index slot");
  return s->indices[slot];
}

int64_t server_submit(Server* s, int slot, const sph_hoa_camera* cam, const sph_hoa_tf* tf, float* out) {
  auto r = std::make_shared<Request>();
  r->slot = slot;
  r->cam = *cam;
  r->tf = *tf;
  r->out = out;
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (slot < 0 || slot >= (int)s->indices.size()) throw Error(SPH_HOA_E_INVALID_ARG, "unknown index slot");
    if (s->stop) throw Error(SPH_HOA_E_INVALID_ARG, "server is shutting down");
    if (s->max_request_bytes > 0) {
      const int64_t b = s->estimate_bytes(slot, *cam);
      if (b > s->max_request_bytes) {
        ++s->rejected;
        throw Error(SPH_HOA_E_OUT_OF_MEMORY, "request needs about " + std::to_string(b) +
                                                 " bytes of device memory, above the per-request limit");
      }
    }
    if (s->max_queued > 0 && (int64_t)s->queue.size() >= s->max_queued) {
      ++s->rejected;
      throw Error(SPH_HOA_E_BUSY, "request queue is full");
    }
    r->id = s->next_id++;
    s->live[r->id] = r;
    s->queue.push_back(r);
  }
  s->cv_work.notify_one();
  return r->id;
}

bool server_wait(Server* s, int64_t id, double timeout_s, double* latency_ms, sph_hoa_status* req_status,
                 std::string* req_error) {
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->live.find(id);
  if (it == s->live.end()) throw Error(SPH_HOA_E_INVALID_ARG, "unknown or already collected request id");
  std::shared_ptr<Request> r = it->second;
  const auto pred = [&] { return r->done; };
  if (timeout_s < 0) s->cv_done.wait(lk, pred);
  else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) return false;
  s->live.erase(id);
  if (latency_ms) *latency_ms = (r->t_done - r->t_submit) * 1e3;
  *req_status = r->status;
  *req_error = r->error;
  return true;
}

void server_set_admission(Server* s, int64_t max_queued, int64_t max_request_bytes) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->max_queued = max_queued;
  s->max_request_bytes = max_request_bytes;
}

void server_pause(Server* s, bool paused) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->paused = paused;
  }
  s->cv_work.notify_all();
}

bool server_cancel(Server* s, int64_t id) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->live.find(id);
    if (it == s->live.end()) throw Error(SPH_HOA_E_INVALID_ARG, "unknown or already collected request id");
    const std::shared_ptr<Request> r = it->second;
    auto q = std::find(s->queue.begin(), s->queue.end(), r);
    if (q == s->queue.end()) return false;  // taken by the worker or already done
    s->queue.erase(q);
    r->done = true;
    r->status = SPH_HOA_E_CANCELLED;
    r->error = "cancelled";
    r->t_done = now_s();
    ++s->cancelled;
  }
  s->cv_done.notify_all();
  return true;
}

void server_stats(Server* s, sph_hoa_server_stats* st) {
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(st, 0, sizeof(*st));
  st->rejected = s->rejected;
  st->cancelled = s->cancelled;
  st->completed = s->completed;
  st->failed = s->failed;
  st->queued = (int64_t)s->queue.size();
  st->batches = s->batches;
  st->n_rays = s->rays;
  st->n_pairs = s->pairs;
  st->busy_s = s->busy_s;
  st->lanes = (int64_t)s->lanes.size();
  st->overlapped_batches = s->overlapped;
  st->max_in_flight = s->max_in_flight;
  std::vector<double> l = s->latencies_ms;
  if (!l.empty()) {
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) {
      const double x = p * (double)(l.size() - 1);
      const size_t i = (size_t)x;
      const double f = x - (double)i;
      return i + 1 < l.size() ? l[i] * (1.0 - f) + l[i + 1] * f : l[i];
    };
    st->p50_ms = pct(0.50);
    st->p99_ms = pct(0.99);
    st->max_ms = l.back();
  }
}

}  // namespace sph
