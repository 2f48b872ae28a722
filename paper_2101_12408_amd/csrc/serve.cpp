// Serving runtime: continuous batching of simulation-step requests on one GPU.
//
// A request carries a scene (parameters and the host particle state) and a number of
// implicit steps.  Worker threads, each with its own non-blocking stream, take requests
// in arrival order.  A worker sizes the request's memory (the surface buffers for up to
// twice as many samples as particles, at least 4096), then waits for its admission turn:
// requests are admitted strictly in arrival order, each once the device arena
// (caller-allocated HBM) has room for its context workspace and buffers.  Every step draws
// its surface samples on the device from the resident positions (mpm_sample_surface_dev;
// FP32 positions in MIXED).
// A request whose samples outgrow that size releases its memory and goes back to the
// front of the queue once, sized by the count it found.
// It uploads the state, runs the steps through mpm_step, downloads the result and frees
// its memory.  Up to max_concurrent requests are on the device at once, on separate
// streams, so a request that arrives while others run starts as soon as a worker and
// memory are free.  Its work then overlaps theirs on the GPU.  A request's result does
// not depend on what else runs (the step is deterministic per scene).
//
// Host-only code over the public C ABI; the library allocates no device memory here
// either (the arena is the caller's).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mpm.h"

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with coalescing free list (offsets only).
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        size_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  size_t size_, used_ = 0;
  std::map<size_t, size_t> free_;
};

struct Request {
  mpm_request r{};
  const double* src[8] = {};     // input state: the caller's arrays (borrow) or f
  std::vector<double> f[8];      // x v A J V0 m T gradT, [comp][n] double: input copy, then result
  std::vector<int64_t> orig;     // request-order index of each device slot
  mpm_completion c{};
  int64_t cap_hint = 0;          // surface capacity after an overflow (0: the size rule)
  bool requeued = false;
};

// run_request's status for a request whose samples exceeded its surface buffers.
constexpr int kResize = -1;

struct Worker {
  hipStream_t stream = nullptr;
  void* stage = nullptr;         // pinned staging
  size_t stage_bytes = 0;
};

}  // namespace

struct mpm_server {
  char* arena = nullptr;
  Arena alloc{0};
  int device = 0;
  int workers = 1;
  std::vector<std::thread> threads;
  std::mutex mu;
  std::condition_variable cv;      // queue, admission turn, memory, completion
  std::deque<Request*> queue;
  std::map<int64_t, Request*> done;
  std::vector<mpm_completion> fresh;
  uint64_t next_ticket = 0, admit_turn = 0;
  int64_t submitted = 0, completed = 0, rejected = 0, running = 0, picked = 0;
  int64_t peak_bytes = 0;
  int32_t peak_running = 0;
  bool stop = false;
  std::string err;
};

namespace {

int components(int field, int dim) {
  switch (field) {
    case 0: case 1: case 7: return dim;   // x v gradT
    case 2: return dim * dim;             // A
    default: return 1;                    // J V0 m T
  }
}


void ensure_stage(Worker& w, size_t bytes) {
  if (w.stage_bytes >= bytes) return;
  if (w.stage) (void)hipHostFree(w.stage);
  w.stage = nullptr;
  w.stage_bytes = 0;
  if (hipHostMalloc(&w.stage, bytes, hipHostMallocDefault) == hipSuccess) w.stage_bytes = bytes;
}

// Host double [count] -> device real.
bool upload(Worker& w, void* dst, const double* src, size_t count, bool fp64) {
  const size_t bytes = count * (fp64 ? 8 : 4);
  if (!count) return true;
  ensure_stage(w, bytes);
  if (w.stage_bytes < bytes) return false;
  if (fp64) std::memcpy(w.stage, src, bytes);
  else {
    float* f = (float*)w.stage;
    for (size_t i = 0; i < count; ++i) f[i] = (float)src[i];
  }
  return hipMemcpyAsync(dst, w.stage, bytes, hipMemcpyHostToDevice, w.stream) == hipSuccess &&
         hipStreamSynchronize(w.stream) == hipSuccess;
}

// Device real [count] -> host double.
bool download(Worker& w, double* dst, const void* src, size_t count, bool fp64) {
  const size_t bytes = count * (fp64 ? 8 : 4);
  if (!count) return true;
  ensure_stage(w, bytes);
  if (w.stage_bytes < bytes) return false;
  if (hipMemcpyAsync(w.stage, src, bytes, hipMemcpyDeviceToHost, w.stream) != hipSuccess ||
      hipStreamSynchronize(w.stream) != hipSuccess)
    return false;
  if (fp64) std::memcpy(dst, w.stage, bytes);
  else {
    const float* f = (const float*)w.stage;
    for (size_t i = 0; i < count; ++i) dst[i] = f[i];
  }
  return true;
}

bool download_i32(Worker& w, int32_t* dst, const void* src, size_t count) {
  if (!count) return true;
  return hipMemcpyAsync(dst, src, count * 4, hipMemcpyDeviceToHost, w.stream) == hipSuccess &&
         hipStreamSynchronize(w.stream) == hipSuccess;
}

// Runs an admitted request: returns the status.  mem: the request's arena block.
int run_request(mpm_server* srv, Worker& w, Request& q, char* mem, size_t ws_bytes, int64_t cap_surf) {
  const mpm_params& p = q.r.params;
  const int dim = p.dim;
  const int64_t N = q.r.n_part;
  const bool fp64 = p.precision == MPM_FP64;
  const size_t R = fp64 ? 8 : 4;
  // carve: workspace | particle fields | surface s, dA, label
  char* cur = mem;
  void* ws = cur;
  cur += align_up(ws_bytes);
  void* pf[8];
  for (int k = 0; k < 8; ++k) {
    pf[k] = cur;
    cur += align_up((size_t)components(k, dim) * N * R);
  }
  void* ds = cur;
  cur += align_up((size_t)dim * cap_surf * R);
  void* ddA = cur;
  cur += align_up((size_t)dim * cap_surf * R);
  int32_t* dlab = (int32_t*)cur;
  mpm_ctx* ctx = nullptr;
  int rc = mpm_ctx_create(&p, ws, ws_bytes, N, cap_surf, &ctx);
  if (rc != MPM_OK) return rc;
  for (int k = 0; k < 8 && rc == MPM_OK; ++k)
    if (!upload(w, pf[k], q.src[k], (size_t)components(k, dim) * N, fp64)) rc = MPM_EHIP;
  q.orig.resize(N);
  for (int64_t i = 0; i < N; ++i) q.orig[i] = i;
  std::vector<int32_t> perm(N);
  std::vector<int64_t> orig2(N);
  mpm_particles P{N, pf[0], pf[1], pf[2], pf[3], pf[4], pf[5], pf[6], pf[7]};
  for (int st = 0; st < q.r.n_steps && rc == MPM_OK; ++st) {
    int64_t S = 0;
    rc = mpm_sample_surface_dev(ctx, &P, q.r.ls_radius, q.r.sample_density, q.r.seed, q.r.first_step + st,
                                q.r.label_lo, q.r.label_hi, ds, ddA, dlab, cap_surf, &S, w.stream);
    if (rc != MPM_OK) break;
    if (S > cap_surf) {
      if (st == 0 && !q.requeued) {
        q.cap_hint = S + S / 2 + 1024;
        rc = kResize;
      } else {
        rc = MPM_ENOMEM;
      }
      break;
    }
    mpm_surface Sd{S, ds, ddA, dlab};
    mpm_ctx* cs[1] = {ctx};
    mpm_particles* ps[1] = {&P};
    const mpm_surface* ss[1] = {&Sd};
    rc = mpm_step(cs, ps, ss, 1, q.r.implicit, w.stream);
    mpm_stats stt{};
    mpm_get_stats(ctx, &stt);
    q.c.newton_iters += stt.newton_iters;
    q.c.cg_iters += stt.cg_iters;
    q.c.n_surf = S;
    if (rc != MPM_OK) break;
    // the step wrote the particles back in cell order: compose the slot permutation
    void* permd = nullptr;
    if (mpm_grid_view(ctx, MPM_F_PERM, &permd) != MPM_OK || !download_i32(w, perm.data(), permd, N)) {
      rc = MPM_EHIP;
      break;
    }
    for (int64_t k = 0; k < N; ++k) orig2[k] = q.orig[perm[k]];
    q.orig.swap(orig2);
    q.c.steps_done = st + 1;
  }
  // results back in request order
  if (rc == MPM_OK && q.r.keep_result) {
    std::vector<double> tmp;
    for (int k = 0; k < 8 && rc == MPM_OK; ++k) {
      const int nc = components(k, dim);
      tmp.resize((size_t)nc * N);
      q.f[k].resize((size_t)nc * N);
      if (!download(w, tmp.data(), pf[k], (size_t)nc * N, fp64)) { rc = MPM_EHIP; break; }
      for (int a = 0; a < nc; ++a)
        for (int64_t s2 = 0; s2 < N; ++s2) q.f[k][(size_t)a * N + q.orig[s2]] = tmp[(size_t)a * N + s2];
    }
  }
  (void)hipStreamSynchronize(w.stream);
  mpm_ctx_destroy(ctx);
  (void)srv;
  return rc;
}

void finish(mpm_server* srv, Request* q, int status) {
  // caller holds srv->mu
  q->c.status = status;
  q->c.t_done = now_s();
  srv->fresh.push_back(q->c);
  srv->completed++;
  if (status == MPM_EBUDGET) srv->rejected++;
  if (q->r.keep_result) srv->done[q->r.id] = q;
  else delete q;
}

void worker_main(mpm_server* srv) {
  Worker w;
  if (hipSetDevice(srv->device) != hipSuccess || hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) != hipSuccess) {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->err = "worker stream creation failed";
    return;
  }
  for (;;) {
    Request* q = nullptr;
    uint64_t ticket = 0;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->cv.wait(lk, [&] { return srv->stop || !srv->queue.empty(); });
      if (srv->queue.empty()) break;   // stop requested and nothing left
      q = srv->queue.front();
      srv->queue.pop_front();
      ticket = srv->next_ticket++;
      srv->picked++;
    }
    // the memory need: the surface buffers hold twice as many samples as particles (a
    // droplet at 8 per cell has 3 dx / R samples per particle), or the count an earlier
    // attempt found
    const mpm_params& p = q->r.params;
    const int dim = p.dim;
    const int64_t N = q->r.n_part;
    const int64_t cap_surf = q->cap_hint > 0 ? q->cap_hint : std::max<int64_t>(4096, 2 * N);
    size_t ws_bytes = 0;
    int rc = mpm_workspace_bytes(&p, N, cap_surf, &ws_bytes);
    const size_t R = p.precision == MPM_FP64 ? 8 : 4;
    size_t need = align_up(ws_bytes);
    for (int k = 0; k < 8; ++k) need += align_up((size_t)components(k, dim) * N * R);
    need += 2 * align_up((size_t)dim * cap_surf * R) + align_up((size_t)cap_surf * 4);
    size_t off = 0;
    bool admitted = false;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->cv.wait(lk, [&] { return srv->admit_turn == ticket; });
      if (rc == MPM_OK && need > srv->alloc.size()) rc = MPM_EBUDGET;
      if (rc == MPM_OK) {
        srv->cv.wait(lk, [&] { return srv->alloc.alloc(need, &off); });
        admitted = true;
        q->c.t_admit = now_s();
        q->c.bytes = (int64_t)need;
        srv->running++;
        srv->peak_running = std::max<int32_t>(srv->peak_running, (int32_t)srv->running);
        srv->peak_bytes = std::max<int64_t>(srv->peak_bytes, (int64_t)srv->alloc.used());
      }
      srv->admit_turn++;
      if (!admitted) finish(srv, q, rc);
    }
    srv->cv.notify_all();
    if (!admitted) continue;
    rc = run_request(srv, w, *q, srv->arena + off, ws_bytes, cap_surf);
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->alloc.release(off, need);
      srv->running--;
      if (rc == kResize) {
        // once more, first in line, with surface buffers for the count it found
        q->requeued = true;
        q->c.steps_done = 0;
        q->c.newton_iters = q->c.cg_iters = 0;
        srv->queue.push_front(q);
        srv->picked--;
      } else {
        finish(srv, q, rc);
      }
    }
    srv->cv.notify_all();
  }
  if (w.stage) (void)hipHostFree(w.stage);
  if (w.stream) (void)hipStreamDestroy(w.stream);
}

}  // namespace

extern "C" {

double mpm_server_clock(void) { return now_s(); }

int mpm_server_create(void* arena, size_t arena_bytes, int32_t max_concurrent, mpm_server** out) {
  if (!out || !arena || arena_bytes == 0 || (reinterpret_cast<uintptr_t>(arena) & (kAlign - 1)) ||
      max_concurrent < 1 || max_concurrent > 64)
    return MPM_EINVAL;
  *out = nullptr;
  mpm_server* srv = new mpm_server();
  srv->arena = (char*)arena;
  srv->alloc = Arena(arena_bytes / kAlign * kAlign);
  srv->workers = max_concurrent;
  if (hipGetDevice(&srv->device) != hipSuccess) {
    delete srv;
    return MPM_EHIP;
  }
  for (int k = 0; k < max_concurrent; ++k) srv->threads.emplace_back(worker_main, srv);
  *out = srv;
  return MPM_OK;
}

int mpm_server_submit(mpm_server* srv, const mpm_request* req) {
  if (!srv || !req) return MPM_EINVAL;
  const mpm_params& p = req->params;
  if ((p.dim != 2 && p.dim != 3) || req->n_part < 1 || req->n_steps < 1) return MPM_EINVAL;
  const double* src[8] = {req->x, req->v, req->A, req->J, req->V0, req->m, req->T, req->gradT};
  for (const double* s : src)
    if (!s) return MPM_EINVAL;
  Request* q = new Request();
  q->r = *req;
  for (int k = 0; k < 8; ++k) {
    if (req->borrow) {
      q->src[k] = src[k];
    } else {
      q->f[k].assign(src[k], src[k] + (size_t)components(k, p.dim) * req->n_part);
      q->src[k] = q->f[k].data();
    }
  }
  q->r.x = q->r.v = q->r.A = q->r.J = q->r.V0 = q->r.m = q->r.T = q->r.gradT = nullptr;
  q->c.id = req->id;
  q->c.n_part = req->n_part;
  q->c.t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop || srv->done.count(req->id)) {
      delete q;
      return MPM_EINVAL;
    }
    srv->queue.push_back(q);
    srv->submitted++;
  }
  srv->cv.notify_all();
  return MPM_OK;
}

int mpm_server_poll(mpm_server* srv, mpm_completion* out, int32_t cap, int32_t* n_out) {
  if (!srv || !n_out || cap < 0 || (cap > 0 && !out)) return MPM_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  int32_t n = (int32_t)std::min<size_t>(cap, srv->fresh.size());
  for (int32_t k = 0; k < n; ++k) out[k] = srv->fresh[k];
  srv->fresh.erase(srv->fresh.begin(), srv->fresh.begin() + n);
  *n_out = n;
  return MPM_OK;
}

int mpm_server_wait(mpm_server* srv, double timeout_s) {
  if (!srv) return MPM_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto idle = [&] { return srv->queue.empty() && srv->completed == srv->submitted; };
  if (timeout_s < 0) {
    srv->cv.wait(lk, idle);
    return MPM_OK;
  }
  bool ok = srv->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), idle);
  return ok ? MPM_OK : MPM_ENOCONV;
}

int mpm_server_result(mpm_server* srv, int64_t id, double* x, double* v, double* A, double* J, double* T,
                      double* gradT) {
  if (!srv) return MPM_EINVAL;
  Request* q = nullptr;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->done.find(id);
    if (it == srv->done.end()) return MPM_EINVAL;
    q = it->second;
    srv->done.erase(it);
  }
  const int dim = q->r.params.dim;
  const size_t N = (size_t)q->r.n_part;
  double* dst[8] = {x, v, A, J, nullptr, nullptr, T, gradT};
  // a request that failed (or borrowed its arrays and kept no result) has no state to copy
  for (int k = 0; k < 8; ++k)
    if (dst[k] && q->f[k].size() == (size_t)components(k, dim) * N)
      std::memcpy(dst[k], q->f[k].data(), q->f[k].size() * sizeof(double));
  const int status = q->c.status;
  delete q;
  return status;
}

int mpm_server_info_get(mpm_server* srv, mpm_server_info* out) {
  if (!srv || !out) return MPM_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  out->submitted = srv->submitted;
  out->completed = srv->completed;
  out->rejected = srv->rejected;
  out->queued = (int64_t)srv->queue.size();
  out->running = srv->running;
  out->arena_bytes = (int64_t)srv->alloc.size();
  out->bytes_in_use = (int64_t)srv->alloc.used();
  out->peak_bytes = srv->peak_bytes;
  out->peak_running = srv->peak_running;
  return MPM_OK;
}

int mpm_server_destroy(mpm_server* srv) {
  if (!srv) return MPM_EINVAL;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv.notify_all();
  for (auto& t : srv->threads) t.join();
  for (auto& kv : srv->done) delete kv.second;
  for (Request* q : srv->queue) delete q;
  delete srv;
  return MPM_OK;
}

}  // extern "C"
