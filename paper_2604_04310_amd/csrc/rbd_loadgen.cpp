// Open-loop load generator for the serving runtime (a measurement client, not
// part of the hot path): Poisson arrivals from a native thread, so that what
// is measured is the server and not the overhead of a scripting-language
// client. It uses only the public rbd_server_* calls.
#include <atomic>
#include <chrono>
#include <cmath>
#include <thread>
#include <vector>

#include "rbd_internal.hpp"

namespace rbd {
namespace {

using Clock = std::chrono::steady_clock;

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): the stream of arrival gaps.
struct SplitMix64 {
  uint64_t x;
  uint64_t next() {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }  // [0, 1)
};

int out_count(int op) { return op == RBD_OP_FWD_DYN_VJP ? 3 : 1; }

int64_t out_rows(const rbd_model* m, int op, int a) {
  if (op == RBD_OP_FWD_DYN_VJP && a == 0) return m->nq;
  return m->nv;
}

}  // namespace
}  // namespace rbd

using namespace rbd;

extern "C" rbd_status rbd_diag_serve_load(rbd_server* s, int n_spec, const rbd_load_request* spec,
                                          int64_t n_requests, double rate_per_s, int window, uint64_t seed,
                                          double* wall_s, int64_t* failed) {
  if (!s || !spec || !wall_s || !failed) return fail(RBD_E_INVAL, "rbd_diag_serve_load: NULL argument");
  if (n_spec < 1 || n_requests < 1 || window < 1 || !(rate_per_s >= 0.0))
    return fail(RBD_E_INVAL, "rbd_diag_serve_load: n_spec, n_requests and window must be >= 1, rate >= 0");
  for (int k = 0; k < n_spec; ++k) {
    const rbd_load_request& r = spec[k];
    if (!r.model || r.batch < 1 || r.op < RBD_OP_FWD_DYN || r.op > RBD_OP_FWD_DYN_VJP)
      return fail(RBD_E_INVAL, "rbd_diag_serve_load: request %d is malformed", k);
  }
  // output buffers: `copies` per spec, so that request j writes buffer j mod
  // (copies * n_spec), which no other outstanding request uses
  const int copies = (window + n_spec - 1) / n_spec;
  const int64_t n_buf = (int64_t)copies * n_spec;
  std::vector<std::vector<float>> bufs((size_t)n_buf * 3);
  for (int64_t b = 0; b < n_buf; ++b) {
    const rbd_load_request& r = spec[b % n_spec];
    for (int a = 0; a < out_count(r.op); ++a) bufs[(size_t)b * 3 + a].resize((size_t)(out_rows(r.model, r.op, a) * r.batch));
  }
  std::vector<uint64_t> tickets((size_t)n_requests);
  std::atomic<int64_t> submitted{0}, completed{0}, n_failed{0};
  std::atomic<bool> abort{false};
  Clock::time_point t_last;

  // waiter: tickets in submission order
  std::thread waiter([&] {
    for (int64_t j = 0; j < n_requests; ++j) {
      while (submitted.load(std::memory_order_acquire) <= j) {
        if (abort.load()) return;
        std::this_thread::yield();
      }
      rbd_status st = RBD_OK;
      if (rbd_server_wait(s, tickets[(size_t)j], -1.0, &st) != RBD_OK || st != RBD_OK) n_failed++;
      completed.store(j + 1, std::memory_order_release);
    }
    t_last = Clock::now();
  });

  SplitMix64 rng{seed};
  rbd_status result = RBD_OK;
  const Clock::time_point t0 = Clock::now();
  double t_next = 0.0;  // seconds after t0
  for (int64_t j = 0; j < n_requests; ++j) {
    while (j - completed.load(std::memory_order_acquire) >= n_buf) std::this_thread::yield();  // window full
    if (rate_per_s > 0.0) {
      t_next += -std::log1p(-rng.uniform()) / rate_per_s;
      while (std::chrono::duration<double>(Clock::now() - t0).count() < t_next) {
      }
    }
    const rbd_load_request& r = spec[j % n_spec];
    const int64_t b = j % n_buf;
    float* outs[3] = {nullptr, nullptr, nullptr};
    for (int a = 0; a < out_count(r.op); ++a) outs[a] = bufs[(size_t)b * 3 + a].data();
    result = rbd_server_submit(s, r.model, r.op, r.batch, r.in, outs, &tickets[(size_t)j]);
    if (result != RBD_OK) {
      abort = true;
      break;
    }
    submitted.store(j + 1, std::memory_order_release);
  }
  if (result != RBD_OK) {
    // let the waiter finish what was submitted, then report the submit error
    const int64_t sent = submitted.load();
    while (completed.load() < sent) std::this_thread::yield();
    waiter.join();
    return result;
  }
  waiter.join();
  *wall_s = std::chrono::duration<double>(t_last - t0).count();
  *failed = n_failed.load();
  return RBD_OK;
}
