// Serving loop over particle state resident in HBM: continuous batching of
// cell-pair tasks (density or force sums of one cell's i range over one
// neighbouring cell).
//
// Threads: the caller submits requests (any thread); a dispatcher thread
// forms batches from the requests whose arrival time has passed, in arrival
// order, as long as their result records fit in the largest free block of
// the device result pool, and launches each batch on a free stream (H2D copy
// of the descriptors, the task kernels, D2H copy of the records into pinned
// staging, an event); a completion thread polls the events of the batches
// in flight, copies each finished batch's records to the requests' host
// buffers, returns the pool block and time-stamps the tasks.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "sph_internal.h"

namespace sph {
sph_status host_fail(sph_status code, const char* msg);
}

namespace {

static_assert(sizeof(sph_task) == 20, "sph_task layout");
static_assert(sizeof(sph_task_result) == 32, "sph_task_result layout");
static_assert(sizeof(sph_request) == 40, "sph_request layout");
static_assert(sizeof(sph_task_done) == 48, "sph_task_done layout");

constexpr size_t kRec = sizeof(sph_task_result);
constexpr int kMaxStreams = 8;
constexpr int kMaxBatch = 4096;

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

int64_t clock_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

sph_status err(sph_status code, const std::string& msg) { return sph::host_fail(code, msg.c_str()); }

// Sizes derived from a configuration
struct Dims {
  int ti, k, streams, max_batch, max_items;
  size_t tasks_b, off_b, items_b, desc_b;   // per stream: descriptor arrays
  size_t pool_recs;
  size_t stage_recs;                        // per stream: pinned result staging
};

sph_status make_dims(const sph_server_config* cfg, Dims& d) {
  if (!cfg) return err(SPH_E_INVALID, "sph_server: config is NULL");
  d.ti = cfg->tile.ti ? cfg->tile.ti : 64;
  d.k = cfg->tile.k ? cfg->tile.k : 4;
  if (!sph::task_tile_supported(d.ti, d.k))
    return err(SPH_E_UNSUPPORTED, "sph_server: task tile not supported");
  if (cfg->streams < 1 || cfg->streams > kMaxStreams)
    return err(SPH_E_INVALID, "sph_server: streams must be 1..8");
  if (cfg->max_batch < 1 || cfg->max_batch > kMaxBatch)
    return err(SPH_E_INVALID, "sph_server: max_batch must be 1..4096");
  d.streams = cfg->streams;
  d.max_batch = cfg->max_batch;
  d.max_items = d.max_batch * ((SPH_TASK_MAX_I + d.ti - 1) / d.ti);
  d.tasks_b = al256(sizeof(sph_task) * (size_t)d.max_batch);
  d.off_b = al256(sizeof(int32_t) * (size_t)d.max_batch);
  d.items_b = al256(2 * sizeof(int32_t) * (size_t)d.max_items);
  d.desc_b = d.tasks_b + d.off_b + d.items_b;
  d.pool_recs = cfg->pool_bytes / kRec;
  if (d.pool_recs < (size_t)SPH_TASK_MAX_I)
    return err(SPH_E_INVALID, "sph_server: pool_bytes must hold SPH_TASK_MAX_I records");
  if (d.pool_recs > (size_t)0x7fffffff) return err(SPH_E_RANGE, "sph_server: pool too large");
  d.stage_recs = std::min(d.pool_recs, (size_t)d.max_batch * SPH_TASK_MAX_I);
  return SPH_OK;
}

// First-fit allocator of record ranges in the result pool
class Pool {
 public:
  void reset(size_t n) {
    free_.clear();
    if (n) free_[0] = n;
    used_ = 0;
  }
  size_t largest() const {
    size_t m = 0;
    for (const auto& b : free_) m = std::max(m, b.second);
    return m;
  }
  int64_t alloc(size_t n) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, rest = it->second - n;
      free_.erase(it);
      if (rest) free_[off + n] = rest;
      used_ += n;
      return (int64_t)off;
    }
    return -1;
  }
  void release(size_t off, size_t n) {
    if (!n) return;
    used_ -= n;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;   // offset -> length
  size_t used_ = 0;
};

struct Req {
  sph_request r;
  int64_t id;
  int n_i;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  char* desc_host = nullptr;            // pinned: tasks | out_off | items
  char* desc_dev = nullptr;
  sph_task_result* stage = nullptr;     // pinned result staging
  bool busy = false, launched = false;
  std::vector<Req> reqs;
  int64_t admit_ns = 0, launch_ns = 0;
  int batch = 0;
  size_t pool_off = 0, pool_n = 0;
};

}  // namespace

struct sph_server {
  Dims d{};
  sph_soa soa{};
  sph_precision prec{};
  sph_cells cells{};
  sph_params prm{};
  int device = 0;
  std::vector<int32_t> start;           // host copy of cell_start
  sph_task_result* pool_dev = nullptr;
  Pool pool;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_disp, cv_comp, cv_client;
  std::multimap<int64_t, Req> pending;  // by arrival time
  std::deque<sph_task_done> done;
  int64_t next_id = 0, submitted = 0, ndone = 0, batches = 0, adm_waits = 0;
  int64_t pool_hw = 0;
  int inflight = 0, max_inflight = 0;
  bool stop = false;
  sph_status fault = SPH_OK;
  std::string fault_msg;
  std::thread disp, comp;

  void set_fault(const std::string& m) {   // mu held
    if (fault == SPH_OK) {
      fault = SPH_E_HIP;
      fault_msg = m;
    }
    stop = true;
    cv_disp.notify_all();
    cv_comp.notify_all();
    cv_client.notify_all();
  }

  // Launch one batch on slot S (mu not held; S is owned by the dispatcher).
  hipError_t launch(Slot& S, sph_status& st) {
    const int nb = (int)S.reqs.size();
    sph_task* th = reinterpret_cast<sph_task*>(S.desc_host);
    int32_t* oh = reinterpret_cast<int32_t*>(S.desc_host + d.tasks_b);
    int32_t* ih = reinterpret_cast<int32_t*>(S.desc_host + d.tasks_b + d.off_b);
    size_t o = S.pool_off;
    int nd = 0, ni = 0;
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = 0; j < nb; ++j) {
        const sph_task& t = S.reqs[j].r.task;
        if (t.kind != pass) continue;
        for (int f = t.i_begin; f < t.i_end; f += d.ti) {
          ih[2 * ni] = j;
          ih[2 * ni + 1] = f;
          ++ni;
        }
      }
      if (pass == 0) nd = ni;
    }
    for (int j = 0; j < nb; ++j) {
      th[j] = S.reqs[j].r.task;
      oh[j] = (int32_t)o;
      o += (size_t)S.reqs[j].n_i;
    }
    hipError_t e = hipMemcpyAsync(S.desc_dev, th, sizeof(sph_task) * nb, hipMemcpyHostToDevice,
                                  S.stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(S.desc_dev + d.tasks_b, oh, sizeof(int32_t) * nb,
                         hipMemcpyHostToDevice, S.stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(S.desc_dev + d.tasks_b + d.off_b, ih, 2 * sizeof(int32_t) * ni,
                         hipMemcpyHostToDevice, S.stream);
    if (e != hipSuccess) return e;
    st = sph_tasks_run(&soa, &prec, &cells, &prm, sph_tile{d.ti, d.k},
                       reinterpret_cast<const sph_task*>(S.desc_dev), nb,
                       reinterpret_cast<const int32_t*>(S.desc_dev + d.tasks_b),
                       reinterpret_cast<const int32_t*>(S.desc_dev + d.tasks_b + d.off_b), nd,
                       ni - nd, pool_dev, (int32_t)d.pool_recs, S.stream);
    if (st != SPH_OK) return hipErrorLaunchFailure;
    e = hipMemcpyAsync(S.stage, pool_dev + S.pool_off, kRec * S.pool_n, hipMemcpyDeviceToHost,
                       S.stream);
    if (e == hipSuccess) e = hipEventRecord(S.ev, S.stream);
    return e;
  }

  void dispatcher() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    int batch_no = 0;
    while (!stop) {
      int si = -1;
      for (int i = 0; i < d.streams; ++i)
        if (!slots[i].busy) {
          si = i;
          break;
        }
      const int64_t t = clock_ns();
      const bool ready = !pending.empty() && pending.begin()->first <= t;
      if (si < 0 || !ready) {
        if (si >= 0 && !pending.empty())
          cv_disp.wait_for(lk, std::chrono::nanoseconds(pending.begin()->first - t));
        else
          cv_disp.wait(lk);
        continue;
      }
      // the batch: arrived requests in arrival order while their records fit
      const size_t room = pool.largest();
      std::vector<Req> batch;
      size_t need = 0;
      for (auto it = pending.begin();
           it != pending.end() && it->first <= t && (int)batch.size() < d.max_batch;) {
        if (need + (size_t)it->second.n_i > room) break;
        need += (size_t)it->second.n_i;
        batch.push_back(it->second);
        it = pending.erase(it);
      }
      if (batch.empty()) {   // pool full: wait for a completion
        ++adm_waits;
        cv_disp.wait(lk);
        continue;
      }
      const int64_t off = pool.alloc(need);
      pool_hw = std::max<int64_t>(pool_hw, (int64_t)(pool.used() * kRec));
      Slot& S = slots[si];
      S.busy = true;
      S.launched = false;
      S.reqs = std::move(batch);
      S.pool_off = (size_t)off;
      S.pool_n = need;
      S.batch = batch_no++;
      S.admit_ns = t;
      ++inflight;
      ++batches;
      max_inflight = std::max(max_inflight, inflight);
      lk.unlock();
      sph_status st = SPH_OK;
      const hipError_t e = launch(S, st);
      const int64_t tl = clock_ns();
      lk.lock();
      if (e != hipSuccess) {
        set_fault(std::string("sph_server: batch launch failed: ") + hipGetErrorString(e));
        break;
      }
      S.launch_ns = tl;
      S.launched = true;
      cv_comp.notify_all();
    }
  }

  void completer() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      bool busy = false, progress = false;
      for (int i = 0; i < d.streams; ++i) {
        Slot& S = slots[i];
        if (!S.busy) continue;
        busy = true;
        if (!S.launched) continue;
        lk.unlock();
        const hipError_t q = hipEventQuery(S.ev);
        lk.lock();
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) {
          set_fault(std::string("sph_server: batch failed: ") + hipGetErrorString(q));
          S.launched = false;   // never read its records
          continue;
        }
        const int64_t tdone = clock_ns();
        lk.unlock();
        size_t o = 0;
        for (const Req& r : S.reqs) {
          if (r.r.out) std::memcpy(r.r.out, S.stage + o, kRec * (size_t)r.n_i);
          o += (size_t)r.n_i;
        }
        lk.lock();
        pool.release(S.pool_off, S.pool_n);
        const int nb = (int)S.reqs.size();
        for (const Req& r : S.reqs)
          done.push_back(sph_task_done{r.id, r.r.arrival_ns, S.admit_ns, S.launch_ns, tdone,
                                       S.batch, nb});
        ndone += nb;
        --inflight;
        S.reqs.clear();
        S.busy = S.launched = false;
        progress = true;
        cv_disp.notify_all();
        cv_client.notify_all();
      }
      if (fault != SPH_OK) {
        // a failed batch leaves its slot busy; wait for the others only
        bool others = false;
        for (const Slot& S : slots) others |= S.busy && S.launched;
        if (!others) break;
      } else if (!busy) {
        if (stop) break;
        cv_comp.wait(lk);
        continue;
      }
      if (!progress) {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(4));
        lk.lock();
      }
    }
  }

  void release_device() {
    for (Slot& S : slots) {
      if (S.stream) (void)hipStreamSynchronize(S.stream);
      if (S.ev) (void)hipEventDestroy(S.ev);
      if (S.stream) (void)hipStreamDestroy(S.stream);
      if (S.desc_host) (void)hipHostFree(S.desc_host);
      if (S.stage) (void)hipHostFree(S.stage);
      S = Slot{};
    }
  }
};

extern "C" {

int64_t sph_now_ns(void) { return clock_ns(); }

sph_status sph_server_workspace_size(const sph_server_config* cfg, size_t* bytes) {
  Dims d;
  sph_status st = make_dims(cfg, d);
  if (st != SPH_OK) return st;
  if (!bytes) return err(SPH_E_INVALID, "sph_server_workspace_size: bytes is NULL");
  *bytes = (size_t)d.streams * d.desc_b + al256(kRec * d.pool_recs);
  return SPH_OK;
}

sph_status sph_server_create(const sph_server_config* cfg, const sph_soa* soa,
                             const sph_precision* prec, const sph_cells* cells,
                             const sph_params* params, void* workspace, size_t workspace_bytes,
                             sph_server** out) {
  Dims d;
  sph_status st = make_dims(cfg, d);
  if (st != SPH_OK) return st;
  if (!soa || !prec || !cells || !params || !out)
    return err(SPH_E_INVALID, "sph_server_create: NULL argument");
  *out = nullptr;
  if (cells->n < 0 || cells->n_c < 3 || cells->n_c > 1290 || !cells->cell_start)
    return err(SPH_E_INVALID, "sph_server_create: bad cell list");
  size_t need = 0;
  sph_server_workspace_size(cfg, &need);
  if (!workspace || workspace_bytes < need)
    return err(SPH_E_NOMEM, "sph_server_create: workspace too small");
  if (reinterpret_cast<uintptr_t>(workspace) & 255)
    return err(SPH_E_INVALID, "sph_server_create: workspace must be 256-byte aligned");
  auto* s = new sph_server();
  s->d = d;
  s->soa = *soa;
  s->prec = *prec;
  s->cells = *cells;
  s->prm = *params;
  const size_t C = (size_t)cells->n_c * cells->n_c * cells->n_c;
  s->start.resize(C + 1);
  hipError_t e = hipGetDevice(&s->device);
  if (e == hipSuccess)
    e = hipMemcpy(s->start.data(), cells->cell_start, sizeof(int32_t) * (C + 1),
                  hipMemcpyDeviceToHost);
  char* ws = static_cast<char*>(workspace);
  s->pool_dev = reinterpret_cast<sph_task_result*>(ws + (size_t)d.streams * d.desc_b);
  s->pool.reset(d.pool_recs);
  s->slots.resize(d.streams);
  for (int i = 0; i < d.streams && e == hipSuccess; ++i) {
    Slot& S = s->slots[i];
    S.desc_dev = ws + (size_t)i * d.desc_b;
    e = hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S.ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&S.desc_host), d.desc_b);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&S.stage), kRec * d.stage_recs);
  }
  if (e != hipSuccess) {
    s->release_device();
    delete s;
    return err(SPH_E_HIP, std::string("sph_server_create: ") + hipGetErrorString(e));
  }
  bool ok = true;
  for (size_t c = 0; c < C && ok; ++c) ok = s->start[c] <= s->start[c + 1];
  if (!ok || s->start[0] != 0 || s->start[C] != cells->n) {
    s->release_device();
    delete s;
    return err(SPH_E_INVALID, "sph_server_create: cell_start is not a cell list of n particles");
  }
  s->disp = std::thread([s] { s->dispatcher(); });
  s->comp = std::thread([s] { s->completer(); });
  *out = s;
  return SPH_OK;
}

sph_status sph_server_submit(sph_server* srv, const sph_request* req, int32_t n,
                             int64_t* first_id) {
  if (!srv || (n > 0 && !req) || n < 0) return err(SPH_E_INVALID, "sph_server_submit: bad arguments");
  const int n_c = srv->cells.n_c;
  const int C = n_c * n_c * n_c;
  for (int j = 0; j < n; ++j) {
    const sph_task& t = req[j].task;
    if ((t.kind != SPH_TASK_DENSITY && t.kind != SPH_TASK_FORCE) || req[j].reserved != 0)
      return err(SPH_E_INVALID, "sph_server_submit: task " + std::to_string(j) + ": bad kind");
    if (t.ci < 0 || t.ci >= C || t.cj < 0 || t.cj >= C)
      return err(SPH_E_RANGE, "sph_server_submit: task " + std::to_string(j) + ": cell out of range");
    const int lo = srv->start[t.ci], hi = srv->start[t.ci + 1];
    if (t.i_begin < lo || t.i_end > hi || t.i_end <= t.i_begin ||
        t.i_end - t.i_begin > SPH_TASK_MAX_I)
      return err(SPH_E_RANGE, "sph_server_submit: task " + std::to_string(j) +
                                  ": i range outside cell ci or longer than SPH_TASK_MAX_I");
    const int ax = t.ci % n_c, ay = (t.ci / n_c) % n_c, az = t.ci / (n_c * n_c);
    const int bx = t.cj % n_c, by = (t.cj / n_c) % n_c, bz = t.cj / (n_c * n_c);
    auto adj = [&](int a, int b) {
      const int dd = ((b - a) % n_c + n_c) % n_c;
      return dd == 0 || dd == 1 || dd == n_c - 1;
    };
    if (!adj(ax, bx) || !adj(ay, by) || !adj(az, bz))
      return err(SPH_E_INVALID, "sph_server_submit: task " + std::to_string(j) +
                                    ": cj is not one of the 27 cells around ci");
  }
  std::lock_guard<std::mutex> g(srv->mu);
  if (srv->fault != SPH_OK) return err(srv->fault, srv->fault_msg);
  if (srv->stop) return err(SPH_E_INVALID, "sph_server_submit: server stopped");
  if (first_id) *first_id = srv->next_id;
  for (int j = 0; j < n; ++j) {
    Req r{req[j], srv->next_id++, req[j].task.i_end - req[j].task.i_begin};
    srv->pending.emplace(req[j].arrival_ns, r);
  }
  srv->submitted += n;
  srv->cv_disp.notify_all();
  return SPH_OK;
}

sph_status sph_server_poll(sph_server* srv, sph_task_done* done, int32_t max, int32_t* n,
                           int32_t wait_ms) {
  if (!srv || !n || max < 0 || (max > 0 && !done))
    return err(SPH_E_INVALID, "sph_server_poll: bad arguments");
  std::unique_lock<std::mutex> lk(srv->mu);
  *n = 0;
  if (srv->done.empty() && wait_ms > 0 && srv->fault == SPH_OK)
    srv->cv_client.wait_for(lk, std::chrono::milliseconds(wait_ms),
                            [&] { return !srv->done.empty() || srv->fault != SPH_OK; });
  int k = 0;
  while (k < max && !srv->done.empty()) {
    done[k++] = srv->done.front();
    srv->done.pop_front();
  }
  *n = k;
  if (srv->fault != SPH_OK) return err(srv->fault, srv->fault_msg);
  return SPH_OK;
}

sph_status sph_server_get_stats(sph_server* srv, sph_server_stats* st) {
  if (!srv || !st) return err(SPH_E_INVALID, "sph_server_get_stats: NULL argument");
  std::lock_guard<std::mutex> g(srv->mu);
  *st = sph_server_stats{srv->submitted, srv->ndone,        srv->batches, srv->adm_waits,
                         srv->max_inflight, 0, srv->pool_hw};
  return SPH_OK;
}

sph_status sph_server_drain(sph_server* srv, int32_t timeout_ms) {
  if (!srv) return err(SPH_E_INVALID, "sph_server_drain: NULL server");
  std::unique_lock<std::mutex> lk(srv->mu);
  const bool ok = srv->cv_client.wait_for(
      lk, std::chrono::milliseconds(std::max(timeout_ms, 0)), [&] {
        return srv->fault != SPH_OK || (srv->pending.empty() && srv->inflight == 0);
      });
  if (srv->fault != SPH_OK) return err(srv->fault, srv->fault_msg);
  if (!ok) return err(SPH_E_RANGE, "sph_server_drain: timed out");
  return SPH_OK;
}

sph_status sph_server_destroy(sph_server* srv) {
  if (!srv) return SPH_OK;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
    srv->pending.clear();
    srv->cv_disp.notify_all();
    srv->cv_comp.notify_all();
  }
  if (srv->disp.joinable()) srv->disp.join();
  if (srv->comp.joinable()) srv->comp.join();
  srv->release_device();
  delete srv;
  return SPH_OK;
}

}  // extern "C"
