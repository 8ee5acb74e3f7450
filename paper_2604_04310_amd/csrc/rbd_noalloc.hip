// The packed launch of the serving runtime without any allocation: requests
// whose arrays are already in device memory, run by the same packed kernels,
// with their descriptor table in a static device array instead of memory the
// library allocates. For callers that cannot allocate device memory (code
// under graph capture, tight serving loops).
//
// The table (header, tile -> request map, request descriptors; the layout the
// packed kernels read) is written on the stream by a small kernel from its
// launch arguments, so nothing is copied from host memory and every call is
// a fixed sequence of kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "rbd_internal.hpp"

namespace rbd {
namespace {

constexpr int kStaticMaxReq = 1024;
constexpr int kStaticMaxTiles = 32768;  // 2 097 152 instances per call
constexpr size_t align16(size_t x) { return (x + 15) / 16 * 16; }
constexpr size_t kScratchBytes =
    align16(sizeof(PackedHdr) + sizeof(int32_t) * kStaticMaxTiles) + sizeof(PackedReq) * kStaticMaxReq;
static_assert(kScratchBytes <= (256u << 10), "the static table stays under 256 KiB");

// The static table of each device (in host code this name is a stand-in, not
// a device address: the address comes from hipGetSymbolAddress).
__device__ __align__(256) uint8_t scratch[kScratchBytes];

// Request descriptors handed to the table writer by value, kChunk at a time
// (2 KiB of kernel arguments).
constexpr int kChunk = 32;
struct Chunk {
  PackedReq req[kChunk];
  int32_t first;  // table index of req[0]
  int32_t count;
  int32_t n_tiles, n_req, req_off;  // the header of the whole table
};

__global__ __launch_bounds__(256) void k_write_table(uint8_t* __restrict__ table, Chunk c) {
  int32_t* tile_req = reinterpret_cast<int32_t*>(table + sizeof(PackedHdr));
  PackedReq* reqs = reinterpret_cast<PackedReq*>(table + c.req_off);
  const bool leader = blockIdx.x == 0 && threadIdx.x == 0;
  if (leader && c.first == 0) {
    PackedHdr* h = reinterpret_cast<PackedHdr*>(table);
    h->n_tiles = c.n_tiles;
    h->n_req = c.n_req;
    h->req_offset = c.req_off;
    h->pad = 0;
  }
  const int stride = (int)(gridDim.x * blockDim.x);
  for (int k = 0; k < c.count; ++k) {
    const PackedReq& r = c.req[k];
    const int nt = (r.batch + kTileLanes - 1) / kTileLanes;
    for (int j = (int)(blockIdx.x * blockDim.x + threadIdx.x); j < nt; j += stride)
      tile_req[r.first_tile + j] = c.first + k;
    if (leader) reqs[c.first + k] = r;
  }
}

// Device address of `scratch`, looked up once per device with it current.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

rbd_status scratch_of(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fail(RBD_E_NODEVICE, "device %d is out of range", device);
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(RBD_E_LAUNCH, "rbd_packed_static: no address for the static table on device %d: %s", device,
                  hipGetErrorString(e));
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return RBD_OK;
}

struct Current {  // makes `dev` current for the call, restores the caller's
  int prev = -1, dev;
  rbd_status st = RBD_OK;
  explicit Current(int d) : dev(d) {
    if (hipGetDevice(&prev) != hipSuccess) {
      prev = -1;
      st = fail(RBD_E_NODEVICE, "no HIP device");
    } else if (prev != dev && hipSetDevice(dev) != hipSuccess) {
      st = fail(RBD_E_NODEVICE, "cannot select device %d", dev);
    }
  }
  ~Current() {
    if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
  }
};

int n_inputs(int op) { return op == RBD_OP_FWD_DYN_VJP ? 4 : 3; }
int n_outputs(int op) { return op == RBD_OP_FWD_DYN_VJP ? 3 : 1; }

}  // namespace
}  // namespace rbd

using namespace rbd;

extern "C" rbd_status rbd_packed_static(const rbd_model* m, int op, int n_req, const rbd_packed_request* reqs,
                                        hipStream_t s) {
  if (!m) return fail(RBD_E_INVAL, "rbd_packed_static: model is NULL");
  if (m->device < 0) return fail(RBD_E_INVAL, "rbd_packed_static: the model is host-only");
  if (op < RBD_OP_FWD_DYN || op > RBD_OP_FWD_DYN_VJP) return fail(RBD_E_INVAL, "rbd_packed_static: bad op %d", op);
  if (n_req < 0 || n_req > kStaticMaxReq)
    return fail(RBD_E_INVAL, "rbd_packed_static: %d requests (at most %d per call)", n_req, kStaticMaxReq);
  if (n_req == 0) return RBD_OK;
  if (!reqs) return fail(RBD_E_INVAL, "rbd_packed_static: reqs is NULL");
  int64_t tiles = 0;
  for (int k = 0; k < n_req; ++k) {
    const rbd_packed_request& r = reqs[k];
    if (r.batch < 0) return fail(RBD_E_INVAL, "rbd_packed_static: request %d has batch %lld", k, (long long)r.batch);
    for (int a = 0; a < n_inputs(op); ++a)
      if (r.batch > 0 && !r.in[a]) return fail(RBD_E_INVAL, "rbd_packed_static: request %d input %d is NULL", k, a);
    for (int a = 0; a < n_outputs(op); ++a)
      if (r.batch > 0 && !r.out[a]) return fail(RBD_E_INVAL, "rbd_packed_static: request %d output %d is NULL", k, a);
    tiles += (r.batch + kTileLanes - 1) / kTileLanes;
    if (tiles > kStaticMaxTiles)
      return fail(RBD_E_INVAL, "rbd_packed_static: more than %d tiles of %d instances (%d instances) in one call",
                  kStaticMaxTiles, kTileLanes, kStaticMaxTiles * kTileLanes);
  }
  if (tiles == 0) return RBD_OK;
  if (!packed_ready(m, op))
    return fail(RBD_E_INVAL,
                "rbd_packed_static: this tree's kernels are compiled at run time and its packed kernel is not loaded "
                "yet (loading code allocates): run one request of this model and op through rbd_server_submit first");
  Current cur(m->device);
  if (cur.st != RBD_OK) return cur.st;
  void* table = nullptr;
  rbd_status st = scratch_of(m->device, &table);
  if (st != RBD_OK) return st;

  Chunk c{};
  c.n_tiles = (int32_t)tiles;
  c.n_req = n_req;
  c.req_off = (int32_t)align16(sizeof(PackedHdr) + sizeof(int32_t) * (size_t)tiles);
  int32_t tile = 0;
  for (int first = 0; first < n_req; first += kChunk) {
    c.first = first;
    c.count = std::min(kChunk, n_req - first);
    int32_t most = 1;
    for (int k = 0; k < c.count; ++k) {
      const rbd_packed_request& r = reqs[first + k];
      PackedReq& p = c.req[k];
      for (int a = 0; a < 4; ++a) p.in[a] = a < n_inputs(op) ? r.in[a] : nullptr;
      for (int a = 0; a < 3; ++a) p.out[a] = a < n_outputs(op) ? r.out[a] : nullptr;
      p.batch = (int32_t)r.batch;
      p.first_tile = tile;
      const int32_t nt = (int32_t)((r.batch + kTileLanes - 1) / kTileLanes);
      tile += nt;
      most = std::max(most, nt);
    }
    const int blocks = std::min(64, (most + 255) / 256);
    hipLaunchKernelGGL(k_write_table, dim3(blocks), dim3(256), 0, s, static_cast<uint8_t*>(table), c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RBD_E_LAUNCH, "rbd_packed_static: table write failed: %s", hipGetErrorString(e));
  }
  // one wave per tile of 64 instances, four waves per block
  const int grid = (int)((tiles * kTileLanes + 255) / 256);
  return launch_packed(m, op, table, grid, s);
}
