// Continuous-batching service for dynamics requests.
//
// Requests (model, operation, batch, host buffers) queue in arrival order. A
// dispatcher thread forms a launch group from the oldest request's (model,
// operation) class: as many queued requests of that class as fit the largest
// free block of the device arena (admission by device memory), and hands it to
// a free launch slot. A group is one block of the arena holding all of its
// inputs, then all of its outputs; it costs one host-to-device copy, one packed
// launch (every request of the group at once, tiles of 64 instances) and one
// device-to-host copy. The packed launch has a fixed grid of persistent waves
// that read the tile table from device memory, so one captured HIP graph per
// (slot, class, grid size) replays it for any group. Each slot is a stream and
// a worker thread: the worker stages the group's inputs into pinned memory,
// queues the copies and the launch, sleeps until a host callback queued behind
// the copy-back wakes it, copies the results into the clients' buffers, frees
// the arena block and records each request's latency (submit to results in
// host memory). Up to n_streams groups are in flight at once, so requests that
// arrive while others run are admitted as memory and slots free up, their work
// overlaps on the GPU, and the host copies of different groups run in
// parallel. A group that fails fails only its own requests. The host executor
// runs the same scheduler over host memory with a fixed stand-in computation,
// so admission, packing, completion, cancellation and failure handling can be
// tested without a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "rbd_internal.hpp"

namespace rbd {
namespace {

using Clock = std::chrono::steady_clock;
constexpr size_t kAlign = 256;
constexpr int kMaxTilesPerGroup = 16384;  // 1 M instances per launch
// By default a launch group stops growing at this many bytes of staged inputs
// and outputs (a single request larger than it still forms a group of its
// own). Host staging and the two copies dominate a group's latency, so a cap
// keeps a small request from waiting behind hundreds of megabytes; 16 MiB is
// about 40 000 humanoid or 140 000 seven-joint instances, enough to fill the
// GPU. rbd_server_config.max_group_bytes overrides it.
constexpr size_t kMaxGroupBytes = size_t(16) << 20;
constexpr int kGridClasses[] = {4, 32, 256, 1024};
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Request {
  uint64_t ticket = 0;
  const rbd_model* model = nullptr;
  int op = 0;
  int64_t batch = 0;
  int n_in = 0, n_out = 0;
  const float* in[4] = {nullptr, nullptr, nullptr, nullptr};
  float* out[3] = {nullptr, nullptr, nullptr};
  size_t in_n[4] = {0, 0, 0, 0};  // floats per array
  size_t out_n[3] = {0, 0, 0};
  size_t in_bytes = 0, out_bytes = 0;
  Clock::time_point t_submit;
  bool done = false;
  rbd_status status = RBD_OK;
};

// The rows per instance of every array of an operation.
void shape_of(const rbd_model* m, int op, int* n_in, int in_rows[4], int* n_out, int out_rows[3]) {
  if (op == RBD_OP_FWD_DYN || op == RBD_OP_RNEA) {
    *n_in = 3; in_rows[0] = m->nq; in_rows[1] = m->nv; in_rows[2] = m->nv;
    *n_out = 1; out_rows[0] = m->nv;
  } else {
    *n_in = 4; in_rows[0] = m->nq; in_rows[1] = m->nv; in_rows[2] = m->nv; in_rows[3] = m->nv;
    *n_out = 3; out_rows[0] = m->nq; out_rows[1] = m->nv; out_rows[2] = m->nv;
  }
}

// First-fit allocator over [0, size) with coalescing of neighbours.
class Arena {
 public:
  void init(size_t size) {
    free_.clear();
    free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t noff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }

 private:
  std::map<size_t, size_t> free_;
};

struct Group {
  rbd_server* srv = nullptr;
  int slot = -1;
  const rbd_model* model = nullptr;
  int op = 0;
  std::vector<std::shared_ptr<Request>> reqs;
  size_t off = 0, bytes = 0, in_bytes = 0, out_off = 0, out_bytes = 0;
  bool timed = false;  // its timeline events were recorded
  std::vector<size_t> in_pos, out_pos;  // per request, offsets inside the block
  int n_tiles = 0;
  rbd_status status = RBD_OK;
};

struct Slot {
  hipStream_t stream = nullptr;
  // device timeline of the slot's current group: before the input copy,
  // after it (the packed launch starts), after the launch, after the copy-back
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  uint8_t* d_table = nullptr;
  uint8_t* h_table = nullptr;
  bool busy = false;  // guarded by the server's mutex
  // captured launches by (model uid, op, grid), used by this slot's worker
  // only: a graph holds its model's table address, so the key must not be the
  // model's (reusable) address
  std::map<std::tuple<uint64_t, int, int>, hipGraphExec_t> graphs;
  // hand-off between the dispatcher, the worker and the stream callback
  std::mutex mu;
  std::condition_variable cv;
  Group* job = nullptr;    // the next group to run (guarded by mu)
  bool work_done = false;  // the stream reached the end of the job (guarded by mu)
  bool quit = false;       // guarded by mu
  std::thread worker;
};

size_t table_capacity(int max_req) {
  return align_up(sizeof(PackedHdr) + sizeof(int32_t) * kMaxTilesPerGroup) + sizeof(PackedReq) * (size_t)max_req;
}

}  // namespace
}  // namespace rbd

using namespace rbd;

struct rbd_server {
  rbd_server_config cfg{};
  bool host_exec = false;      // RBD_EXEC_HOST: arena and staging in host memory
  size_t group_cap = 0;        // bytes at which a launch group stops growing
  uint8_t* d_arena = nullptr;  // device arena (host memory for the host executor)
  uint8_t* h_stage = nullptr;
  Arena arena;
  std::vector<std::unique_ptr<Slot>> slots;
  std::mutex mu;
  std::mutex capture_mu;  // one graph capture at a time
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> pending;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets;
  int n_busy = 0;                // slots with a group (guarded by mu)
  uint64_t next_ticket = 1;
  int64_t n_groups = 0;          // launch groups formed so far
  bool stop = false;
  std::thread dispatcher;
  // statistics
  std::vector<double> lat_us;
  uint64_t n_req = 0, n_inst = 0, n_launch = 0;
  double busy_s = 0.0;
  Clock::time_point busy_since;
  // device timeline since the last reset: per group, the times (ms after
  // `ref`) of its four slot events
  hipStream_t ref_stream = nullptr;
  hipEvent_t ref = nullptr;
  std::vector<std::array<float, 4>> timeline;
};

namespace rbd {
namespace {

int free_slot(rbd_server* s) {
  for (size_t i = 0; i < s->slots.size(); ++i)
    if (!s->slots[i]->busy) return (int)i;
  return -1;
}

// Takes the oldest request's class and every queued request of that class that
// fits; returns nullptr when the head cannot be admitted yet. Caller holds mu.
Group* form_group(rbd_server* s) {
  if (s->pending.empty()) return nullptr;
  const auto head = s->pending.front();
  const size_t budget = s->arena.largest();
  const int max_req = s->cfg.per_request ? 1 : s->cfg.max_batch_requests;
  auto* g = new Group;
  g->model = head->model;
  g->op = head->op;
  size_t in_total = 0, out_total = 0;
  int tiles = 0;
  for (auto it = s->pending.begin(); it != s->pending.end() && (int)g->reqs.size() < max_req;) {
    const auto& r = *it;
    if (r->model != g->model || r->op != g->op) { ++it; continue; }
    const int rt = (int)((r->batch + kTileLanes - 1) / kTileLanes);
    if (tiles + rt > kMaxTilesPerGroup) break;
    const size_t grown = align_up(in_total + r->in_bytes) + out_total + r->out_bytes;
    if (grown > budget) break;
    if (!g->reqs.empty() && grown > s->group_cap) break;
    in_total += r->in_bytes;
    out_total += r->out_bytes;
    tiles += rt;
    g->reqs.push_back(r);
    it = s->pending.erase(it);
  }
  if (g->reqs.empty()) {
    delete g;
    return nullptr;
  }
  g->in_bytes = in_total;
  g->out_off = align_up(in_total);
  g->out_bytes = out_total;
  g->bytes = g->out_off + out_total;
  g->n_tiles = tiles;
  if (!s->arena.alloc(g->bytes, &g->off)) {  // cannot happen: budget is the largest block
    for (auto rit = g->reqs.rbegin(); rit != g->reqs.rend(); ++rit) s->pending.push_front(*rit);
    delete g;
    return nullptr;
  }
  return g;
}

int grid_class(int n_tiles) {
  const int blocks_needed = (n_tiles * kTileLanes + 255) / 256;
  for (int g : kGridClasses)
    if (g >= blocks_needed) return g;
  return kGridClasses[sizeof(kGridClasses) / sizeof(int) - 1];
}

// Captures the packed launch of (model, op) with `grid` blocks on `st` as a graph.
rbd_status capture_packed(const rbd_model* m, int op, const void* d_table, int grid, hipStream_t st,
                          hipGraphExec_t* out) {
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(RBD_E_LAUNCH, "server: stream capture failed");
  const rbd_status rs = launch_packed(m, op, d_table, grid, st);
  const hipError_t ce = hipStreamEndCapture(st, &graph);
  if (rs != RBD_OK || ce != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return rs != RBD_OK ? rs : fail(RBD_E_LAUNCH, "server: stream capture failed");
  }
  const hipError_t ie = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return fail(RBD_E_LAUNCH, "server: graph instantiation failed");
  return RBD_OK;
}

// Host executor: the documented stand-in computation, straight from the
// clients' inputs into the group's output block (host memory).
void host_launch(rbd_server* s, Group* g) {
  uint8_t* hb = s->h_stage + g->off;
  size_t opos = g->out_off;
  for (auto& rp : g->reqs) {
    const Request& r = *rp;
    int in_rows[4], out_rows[3], n_in, n_out;
    shape_of(r.model, r.op, &n_in, in_rows, &n_out, out_rows);
    for (int a = 0; a < r.n_out; ++a) {
      float* o = reinterpret_cast<float*>(hb + opos);
      const int src = a % r.n_in, rows = in_rows[src];
      for (int64_t i = 0; i < r.batch; ++i)
        for (int c = 0; c < out_rows[a]; ++c)
          o[i * out_rows[a] + c] = r.in[src][i * rows + c % rows] + 1000.0f * (float)a;
      opos += r.out_n[a] * sizeof(float);
    }
  }
}

// The stream reached the end of a slot's job: wake its worker (runs on the
// runtime's callback thread; no HIP calls here).
void on_group_done(void* arg) {
  Slot* sl = static_cast<Slot*>(arg);
  std::lock_guard<std::mutex> lk(sl->mu);
  sl->work_done = true;
  sl->cv.notify_all();
}

// Stage, launch and queue the copy-back of one group (its slot's worker, no lock).
rbd_status launch_group(rbd_server* s, Group* g) {
  if (s->host_exec) {
    host_launch(s, g);
    return RBD_OK;
  }
  Slot& sl = *s->slots[g->slot];
  uint8_t* hb = s->h_stage + g->off;
  uint8_t* db = s->d_arena + g->off;
  // pack inputs (instance-major, as given) and the tile table
  PackedHdr* hdr = reinterpret_cast<PackedHdr*>(sl.h_table);
  int32_t* tile_req = reinterpret_cast<int32_t*>(sl.h_table + sizeof(PackedHdr));
  const int32_t req_off = (int32_t)align_up(sizeof(PackedHdr) + sizeof(int32_t) * g->n_tiles);
  PackedReq* reqs = reinterpret_cast<PackedReq*>(sl.h_table + req_off);
  size_t ipos = 0, opos = g->out_off;
  int tile = 0;
  for (size_t k = 0; k < g->reqs.size(); ++k) {
    const Request& r = *g->reqs[k];
    PackedReq pr{};
    for (int a = 0; a < r.n_in; ++a) {
      std::memcpy(hb + ipos, r.in[a], r.in_n[a] * sizeof(float));
      pr.in[a] = reinterpret_cast<const float*>(db + ipos);
      ipos += r.in_n[a] * sizeof(float);
    }
    for (int a = 0; a < r.n_out; ++a) {
      pr.out[a] = reinterpret_cast<float*>(db + opos);
      opos += r.out_n[a] * sizeof(float);
    }
    pr.batch = (int32_t)r.batch;
    pr.first_tile = tile;
    const int rt = (int)((r.batch + kTileLanes - 1) / kTileLanes);
    for (int t = 0; t < rt; ++t) tile_req[tile++] = (int32_t)k;
    reqs[k] = pr;
  }
  hdr->n_tiles = g->n_tiles;
  hdr->n_req = (int32_t)g->reqs.size();
  hdr->req_offset = req_off;
  hdr->pad = 0;
  const size_t table_bytes = req_off + sizeof(PackedReq) * g->reqs.size();
  hipStream_t st = sl.stream;
  if (hipEventRecord(sl.ev[0], st) != hipSuccess ||
      hipMemcpyAsync(db, hb, g->in_bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(sl.d_table, sl.h_table, table_bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipEventRecord(sl.ev[1], st) != hipSuccess)
    return fail(RBD_E_LAUNCH, "server: input copy failed");
  const int grid = s->cfg.per_request ? std::max(1, (g->n_tiles * kTileLanes + 255) / 256) : grid_class(g->n_tiles);
  rbd_status rs = RBD_OK;
  if (s->cfg.use_graphs && !s->cfg.per_request) {
    auto key = std::make_tuple(g->model->uid, g->op, grid);
    auto it = sl.graphs.find(key);
    if (it == sl.graphs.end()) {
      // first group of this model on this slot: capture its graphs for every
      // operation and grid size now, so that none is captured mid-stream later
      // (a capture costs about a millisecond of this worker's time)
      std::lock_guard<std::mutex> cap(s->capture_mu);
      for (int op = RBD_OP_FWD_DYN; op <= RBD_OP_FWD_DYN_VJP; ++op) {
        rs = prepare_packed(g->model, op);  // a run-time-compiled kernel is loaded outside the capture
        if (rs != RBD_OK) return rs;
        for (int gc : kGridClasses) {
          auto k2 = std::make_tuple(g->model->uid, op, gc);
          if (sl.graphs.count(k2)) continue;
          hipGraphExec_t exec = nullptr;
          rs = capture_packed(g->model, op, sl.d_table, gc, st, &exec);
          if (rs != RBD_OK) return rs;
          sl.graphs.emplace(k2, exec);
        }
      }
      it = sl.graphs.find(key);
    }
    if (hipGraphLaunch(it->second, st) != hipSuccess) return fail(RBD_E_LAUNCH, "server: graph launch failed");
  } else {
    rs = launch_packed(g->model, g->op, sl.d_table, grid, st);
    if (rs != RBD_OK) return rs;
  }
  if (hipEventRecord(sl.ev[2], st) != hipSuccess ||
      hipMemcpyAsync(hb + g->out_off, db + g->out_off, g->out_bytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipEventRecord(sl.ev[3], st) != hipSuccess)
    return fail(RBD_E_LAUNCH, "server: result copy failed");
  g->timed = true;
  return RBD_OK;
}

void finish_group(rbd_server* s, Group* g, const Clock::time_point now) {
  // results -> client buffers (instance-major, as requested)
  if (g->status == RBD_OK) {
    const uint8_t* hb = s->h_stage + g->off;
    size_t opos = g->out_off;
    for (auto& rp : g->reqs) {
      Request& r = *rp;
      for (int a = 0; a < r.n_out; ++a) {
        std::memcpy(r.out[a], hb + opos, r.out_n[a] * sizeof(float));
        opos += r.out_n[a] * sizeof(float);
      }
    }
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (g->status == RBD_OK && g->timed) {
    const Slot& sl = *s->slots[g->slot];
    std::array<float, 4> t{};
    bool ok = true;
    for (int k = 0; k < 4; ++k) ok = ok && hipEventElapsedTime(&t[k], s->ref, sl.ev[k]) == hipSuccess;
    if (ok) s->timeline.push_back(t);
  }
  s->arena.release(g->off, g->bytes);
  s->slots[g->slot]->busy = false;
  if (--s->n_busy == 0) s->busy_s += std::chrono::duration<double>(now - s->busy_since).count();
  for (auto& rp : g->reqs) {
    rp->status = g->status;
    rp->done = true;
    s->lat_us.push_back(std::chrono::duration<double, std::micro>(now - rp->t_submit).count());
    s->n_req++;
    s->n_inst += (uint64_t)rp->batch;
  }
  s->n_launch++;
  delete g;
  s->cv_done.notify_all();
  s->cv_work.notify_all();
}

// One group on one slot, start to finish (the slot's worker thread).
void run_group(rbd_server* s, Slot& sl, Group* g) {
  if (g->status == RBD_OK) g->status = launch_group(s, g);
  if (!s->host_exec) {
    if (g->status != RBD_OK) {
      // copies queued before the failure may still run: drain them before the
      // block returns to the arena
      (void)hipStreamSynchronize(sl.stream);
    } else {
      if (hipLaunchHostFunc(sl.stream, on_group_done, &sl) == hipSuccess) {
        std::unique_lock<std::mutex> lk(sl.mu);
        sl.cv.wait(lk, [&] { return sl.work_done; });
      } else {
        (void)hipStreamSynchronize(sl.stream);  // no callback will come: wait here instead
      }
      // an error of the group's device work shows in its event
      if (hipEventQuery(sl.ev[3]) != hipSuccess) g->status = fail(RBD_E_LAUNCH, "server: launch failed on the device");
    }
  }
  finish_group(s, g, Clock::now());
}

void worker_main(rbd_server* s, int k) {
  Slot& sl = *s->slots[k];
  if (!s->host_exec) (void)hipSetDevice(s->cfg.device);
  for (;;) {
    Group* g = nullptr;
    {
      std::unique_lock<std::mutex> lk(sl.mu);
      sl.cv.wait(lk, [&] { return sl.job != nullptr || sl.quit; });
      if (!sl.job) return;  // asked to quit with nothing left to run
      g = sl.job;
      sl.job = nullptr;
      sl.work_done = false;
    }
    run_group(s, sl, g);
  }
}

void dispatcher_main(rbd_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    if (s->pending.empty()) {
      if (s->stop) break;
      s->cv_work.wait(lk);
      continue;
    }
    if (free_slot(s) < 0) {
      s->cv_work.wait(lk);
      continue;
    }
    // gather window: give a young head a moment to collect company
    if (s->cfg.max_wait_us > 0 && !s->cfg.per_request && !s->stop) {
      const auto ready = s->pending.front()->t_submit +
                         std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double, std::micro>(s->cfg.max_wait_us));
      if (Clock::now() < ready && (int)s->pending.size() < s->cfg.max_batch_requests) {
        s->cv_work.wait_until(lk, ready);
        continue;
      }
    }
    Group* g = form_group(s);
    if (!g) {  // the head does not fit the free memory yet: wait for a completion
      s->cv_work.wait(lk);
      continue;
    }
    g->slot = free_slot(s);
    g->srv = s;
    Slot& sl = *s->slots[g->slot];
    sl.busy = true;
    if (s->n_busy++ == 0) s->busy_since = Clock::now();
    if (s->cfg.fail_group > 0 && ++s->n_groups == s->cfg.fail_group)
      g->status = fail(RBD_E_LAUNCH, "server: injected failure of launch group %lld", (long long)s->cfg.fail_group);
    lk.unlock();
    {
      std::lock_guard<std::mutex> sk(sl.mu);
      sl.job = g;
    }
    sl.cv.notify_all();
    lk.lock();
  }
}

}  // namespace
}  // namespace rbd

extern "C" {

rbd_status rbd_server_create(const rbd_server_config* cfg, rbd_server** out) {
  if (!out) return fail(RBD_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(RBD_E_INVAL, "config is NULL");
  if (cfg->n_streams < 1 || cfg->n_streams > 8) return fail(RBD_E_INVAL, "n_streams = %d, expected 1..8", cfg->n_streams);
  if (cfg->max_batch_requests < 1 || cfg->max_batch_requests > kMaxPacked)
    return fail(RBD_E_INVAL, "max_batch_requests = %d, expected 1..%d", cfg->max_batch_requests, kMaxPacked);
  if (cfg->arena_bytes < (1u << 16)) return fail(RBD_E_INVAL, "arena_bytes must be at least 64 KiB");
  if (!(cfg->max_wait_us >= 0.0)) return fail(RBD_E_INVAL, "max_wait_us must be >= 0");
  if (cfg->executor != RBD_EXEC_DEVICE && cfg->executor != RBD_EXEC_HOST)
    return fail(RBD_E_INVAL, "executor = %d is unknown", cfg->executor);
  if (cfg->fail_group < 0) return fail(RBD_E_INVAL, "fail_group must be >= 0");
  const bool host = cfg->executor == RBD_EXEC_HOST;
  if (!host) {
    const int ndev = rbd_device_count();
    if (cfg->device < 0 || cfg->device >= ndev) return fail(RBD_E_NODEVICE, "device %d is not available", cfg->device);
    if (hipSetDevice(cfg->device) != hipSuccess) return fail(RBD_E_NODEVICE, "cannot select device %d", cfg->device);
  }
  auto* s = new (std::nothrow) rbd_server;
  if (!s) return fail(RBD_E_NOMEM, "host allocation failed");
  s->cfg = *cfg;
  s->host_exec = host;
  s->group_cap = cfg->max_group_bytes ? cfg->max_group_bytes : kMaxGroupBytes;
  s->arena.init(cfg->arena_bytes);
  for (int k = 0; k < cfg->n_streams; ++k) s->slots.push_back(std::make_unique<Slot>());
  bool ok = true;
  if (host) {
    s->h_stage = new (std::nothrow) uint8_t[cfg->arena_bytes];
    ok = s->h_stage != nullptr;
  } else {
    ok = hipMalloc(&s->d_arena, cfg->arena_bytes) == hipSuccess &&
         hipHostMalloc(&s->h_stage, cfg->arena_bytes, hipHostMallocDefault) == hipSuccess;
    const size_t tcap = table_capacity(cfg->max_batch_requests);
    for (auto& sl : s->slots) {
      ok = ok && hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) == hipSuccess &&
           hipEventCreate(&sl->ev[0]) == hipSuccess && hipEventCreate(&sl->ev[1]) == hipSuccess &&
           hipEventCreate(&sl->ev[2]) == hipSuccess && hipEventCreate(&sl->ev[3]) == hipSuccess &&
           hipMalloc(&sl->d_table, tcap) == hipSuccess &&
           hipHostMalloc(&sl->h_table, tcap, hipHostMallocDefault) == hipSuccess;
    }
    ok = ok && hipStreamCreateWithFlags(&s->ref_stream, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreate(&s->ref) == hipSuccess && hipEventRecord(s->ref, s->ref_stream) == hipSuccess &&
         hipEventSynchronize(s->ref) == hipSuccess;
  }
  if (!ok) {
    rbd_server_destroy(s);
    return fail(RBD_E_NOMEM, "server: allocation of %zu arena bytes failed", cfg->arena_bytes);
  }
  for (int k = 0; k < cfg->n_streams; ++k) s->slots[k]->worker = std::thread(worker_main, s, k);
  s->dispatcher = std::thread(dispatcher_main, s);
  *out = s;
  return RBD_OK;
}

rbd_status rbd_server_submit(rbd_server* s, const rbd_model* m, int op, int64_t batch, const float* const* host_in,
                             float* const* host_out, uint64_t* ticket) {
  if (!s || !m || !host_in || !host_out || !ticket) return fail(RBD_E_INVAL, "rbd_server_submit: NULL argument");
  if (op < RBD_OP_FWD_DYN || op > RBD_OP_FWD_DYN_VJP) return fail(RBD_E_INVAL, "rbd_server_submit: unknown op %d", op);
  if (batch < 1 || batch > (int64_t)kMaxTilesPerGroup * kTileLanes)
    return fail(RBD_E_INVAL, "rbd_server_submit: batch = %lld out of range", (long long)batch);
  if (s->host_exec ? m->device != -1 : m->device != s->cfg.device)
    return fail(RBD_E_INVAL, s->host_exec ? "rbd_server_submit: the host executor serves host-only models"
                                          : "rbd_server_submit: model lives on another device");
  auto r = std::make_shared<Request>();
  int in_rows[4], out_rows[3];
  shape_of(m, op, &r->n_in, in_rows, &r->n_out, out_rows);
  for (int a = 0; a < r->n_in; ++a) {
    if (!host_in[a]) return fail(RBD_E_INVAL, "rbd_server_submit: input %d is NULL", a);
    r->in[a] = host_in[a];
    r->in_n[a] = (size_t)in_rows[a] * (size_t)batch;
    r->in_bytes += r->in_n[a] * sizeof(float);
  }
  for (int a = 0; a < r->n_out; ++a) {
    if (!host_out[a]) return fail(RBD_E_INVAL, "rbd_server_submit: output %d is NULL", a);
    r->out[a] = host_out[a];
    r->out_n[a] = (size_t)out_rows[a] * (size_t)batch;
    r->out_bytes += r->out_n[a] * sizeof(float);
  }
  if (align_up(r->in_bytes) + r->out_bytes > s->cfg.arena_bytes)
    return fail(RBD_E_INVAL, "rbd_server_submit: request needs %zu bytes, more than the arena holds",
                align_up(r->in_bytes) + r->out_bytes);
  r->model = m;
  r->op = op;
  r->batch = batch;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return fail(RBD_E_SHUTDOWN, "rbd_server_submit: server is shutting down");
  r->ticket = s->next_ticket++;
  r->t_submit = Clock::now();
  s->tickets[r->ticket] = r;
  s->pending.push_back(r);
  *ticket = r->ticket;
  s->cv_work.notify_all();
  return RBD_OK;
}

rbd_status rbd_server_wait(rbd_server* s, uint64_t ticket, double timeout_s, rbd_status* req_status) {
  if (!s) return fail(RBD_E_INVAL, "rbd_server_wait: server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(RBD_E_INVAL, "rbd_server_wait: unknown ticket %llu", (unsigned long long)ticket);
  auto r = it->second;
  if (timeout_s < 0) {
    s->cv_done.wait(lk, [&] { return r->done; });
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return r->done; })) {
    return fail(RBD_E_TIMEOUT, "rbd_server_wait: ticket %llu not done", (unsigned long long)ticket);
  }
  if (req_status) *req_status = r->status;
  s->tickets.erase(ticket);
  return RBD_OK;
}

rbd_status rbd_server_cancel(rbd_server* s, uint64_t ticket) {
  if (!s) return fail(RBD_E_INVAL, "rbd_server_cancel: server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(RBD_E_INVAL, "rbd_server_cancel: unknown ticket %llu", (unsigned long long)ticket);
  auto pos = std::find(s->pending.begin(), s->pending.end(), it->second);
  if (pos == s->pending.end())
    return fail(RBD_E_INVAL, "rbd_server_cancel: ticket %llu already left the queue", (unsigned long long)ticket);
  s->pending.erase(pos);
  it->second->status = RBD_E_CANCELLED;
  it->second->done = true;
  s->cv_done.notify_all();
  s->cv_work.notify_all();
  return RBD_OK;
}

rbd_status rbd_server_get_stats(rbd_server* s, rbd_server_stats* out) {
  if (!s || !out) return fail(RBD_E_INVAL, "rbd_server_get_stats: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = rbd_server_stats{};
  out->requests = s->n_req;
  out->instances = s->n_inst;
  out->launches = s->n_launch;
  out->busy_s = s->busy_s;
  if (!s->lat_us.empty()) {
    std::vector<double> v(s->lat_us);
    auto pct = [&](double p) {
      const size_t k = std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5));
      std::nth_element(v.begin(), v.begin() + (ptrdiff_t)k, v.end());
      return v[k];
    };
    out->p50_us = pct(0.50);
    out->p99_us = pct(0.99);
    out->max_us = *std::max_element(v.begin(), v.end());
    double sum = 0.0;
    for (double x : s->lat_us) sum += x;
    out->mean_us = sum / (double)s->lat_us.size();
  }
  // device timeline: kernel intervals [t1, t2], copies [t0, t1] and [t2, t3]
  std::vector<std::pair<float, int>> kev, cev, aev;
  for (const auto& t : s->timeline) {
    kev.push_back({t[1], 1}); kev.push_back({t[2], -1});
    cev.push_back({t[0], 1}); cev.push_back({t[1], -1}); cev.push_back({t[2], 1}); cev.push_back({t[3], -1});
    aev.push_back({t[0], 1}); aev.push_back({t[3], -1});
  }
  // time (s) covered by at least `k` of the intervals
  auto covered = [](std::vector<std::pair<float, int>>& ev, int k) {
    std::sort(ev.begin(), ev.end());
    double tot = 0.0;
    int depth = 0;
    for (size_t i = 0; i < ev.size(); ++i) {
      if (i > 0 && depth >= k) tot += (double)(ev[i].first - ev[i - 1].first);
      depth += ev[i].second;
    }
    return tot * 1e-3;
  };
  double ksum = 0.0;
  for (const auto& t : s->timeline) ksum += (double)(t[2] - t[1]) * 1e-3;
  out->groups_timed = s->timeline.size();
  out->gpu_kernel_s = covered(kev, 1);
  out->gpu_kernel_overlap_s = covered(kev, 2);
  out->gpu_kernel_sum_s = ksum;
  out->gpu_copy_s = covered(cev, 1);
  out->gpu_active_s = covered(aev, 1);
  return RBD_OK;
}

rbd_status rbd_server_reset_stats(rbd_server* s) {
  if (!s) return fail(RBD_E_INVAL, "rbd_server_reset_stats: server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  s->lat_us.clear();
  s->n_req = s->n_inst = s->n_launch = 0;
  s->busy_s = 0.0;
  s->busy_since = Clock::now();
  s->timeline.clear();
  if (!s->host_exec) {  // a new origin for the device timeline
    (void)hipSetDevice(s->cfg.device);
    if (hipEventRecord(s->ref, s->ref_stream) != hipSuccess || hipEventSynchronize(s->ref) != hipSuccess)
      return fail(RBD_E_LAUNCH, "rbd_server_reset_stats: timeline origin could not be recorded");
  }
  return RBD_OK;
}

rbd_status rbd_server_destroy(rbd_server* s) {
  if (!s) return RBD_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->dispatcher.joinable()) s->dispatcher.join();  // every request has a slot now
  for (auto& sl : s->slots) {
    {
      std::lock_guard<std::mutex> lk(sl->mu);
      sl->quit = true;
    }
    sl->cv.notify_all();
    if (sl->worker.joinable()) sl->worker.join();  // after its last group
  }
  if (s->host_exec) {
    delete[] s->h_stage;
    delete s;
    return RBD_OK;
  }
  (void)hipSetDevice(s->cfg.device);
  for (auto& sl : s->slots) {
    for (auto& kv : sl->graphs) (void)hipGraphExecDestroy(kv.second);
    if (sl->stream) (void)hipStreamSynchronize(sl->stream);
    for (hipEvent_t e : sl->ev)
      if (e) (void)hipEventDestroy(e);
    if (sl->stream) (void)hipStreamDestroy(sl->stream);
    if (sl->d_table) (void)hipFree(sl->d_table);
    if (sl->h_table) (void)hipHostFree(sl->h_table);
  }
  if (s->ref) (void)hipEventDestroy(s->ref);
  if (s->ref_stream) (void)hipStreamDestroy(s->ref_stream);
  if (s->d_arena) (void)hipFree(s->d_arena);
  if (s->h_stage) (void)hipHostFree(s->h_stage);
  delete s;
  return RBD_OK;
}

}  // extern "C"
