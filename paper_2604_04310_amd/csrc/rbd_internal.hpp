// Internal declarations shared by the host API, the kernel dispatch and the
// serving runtime of librbd.so.
#pragma once

#include <stdint.h>

#include <atomic>
#include <string>
#include <vector>

#include "rbd.h"
#include "rbd_kernel_ids.hpp"
#include "rbd_shared.hpp"

namespace rbd {
// The kernels serving a model: those of a topology compiled ahead of time
// (host stub addresses, launched with hipLaunchKernel), or those compiled at
// run time for a new topology and loaded on one device (module functions,
// launched with hipModuleLaunchKernel). A set lives until the process ends.
struct KernelSet {
  const void* aot[KID_COUNT] = {};
  mutable std::atomic<hipFunction_t> jit[KID_COUNT] = {};  // filled on first launch
  bool is_jit = false;
  const char* name = "";
  void* jit_owner = nullptr;  // the run-time topology (rbd_jit.cpp)
  int device = 0;
};
}  // namespace rbd

struct rbd_model {
  int device = 0;
  int topo = -1;               // index into the compiled topology list (-1: compiled at run time)
  const rbd::KernelSet* ks = nullptr;
  int n = 0, nq = 0, nv = 0;
  bool floating = false;
  float* d_tab = nullptr;      // device tables (see rbd_lane.hpp)
  std::vector<float> h_tab;    // the tables of a host-only model (device -1)
  std::vector<int32_t> parent; // topology (for run-time compiled per-frame kernels)
  size_t tab_floats = 0;
  uint64_t uid = 0;            // unique over the process (a new model never reuses one)
};

namespace rbd {

// FP32 device tables of a validated tree (layout in rbd_lane.hpp)
std::vector<float> make_tables(const rbd_tree_desc* d);

// Whether forward dynamics issues all input loads at kernel entry: the
// topology's compiled default, unless the environment variable RBD_PRELOAD
// (0 or 1) overrides it for measurement.
bool preload_inputs(bool topology_default);

// error reporting (thread-local message)
rbd_status fail(rbd_status s, const char* fmt, ...);
void clear_error();

// ---- compiled topologies
struct TopoInfo {
  const char* name;
  bool floating;
  int n;
  const int* parent;
};
int n_topologies();
const TopoInfo& topology(int id);
int find_topology(bool floating, int n, const int32_t* parent);
const KernelSet* aot_kernels(int id);

// ---- run-time compilation of a topology that has no compiled kernels
// (rbd_jit.cpp). jit_kernels returns the topology's kernel set for `device`
// (shared by every model of the topology, alive until the process ends);
// jit_function compiles (or reads from the code-object cache) and loads one of
// its kernels on first use.
rbd_status jit_kernels(bool floating, int n, const int32_t* parent, int device, const KernelSet** out);
rbd_status jit_function(const KernelSet* ks, KernelId id, hipFunction_t* out);
// The differential-IK (osc = false) or operational-space-control kernel of
// one frame, compiled at run time for frames other than the last body (any
// topology), loaded once per device.
rbd_status jit_frame_function(bool floating, int n, const int32_t* parent, int device, bool osc, int frame,
                              hipFunction_t* out);
// Compiles kernel `kernel` of the topology (-1: every kernel of the list;
// KID_COUNT + 2 f (+1): the diff-IK (OSC) kernel of frame f) into the cache
// directory (NULL: the default one); needs no device.
rbd_status jit_precompile(bool floating, int n, const int32_t* parent, const char* cache_dir, int kernel);

// ---- kernel dispatch (rbd_kernels.hip); arguments are already validated
rbd_status launch_fk(const rbd_model* m, int64_t batch, int64_t ld, const float* q, float* T, hipStream_t s);
rbd_status launch_jacobian(const rbd_model* m, int64_t batch, int64_t ld, const float* q, int32_t n_frames,
                           const int32_t* frames, float* J, hipStream_t s);
rbd_status launch_rnea(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                       const float* qdd, const float* fext, float* tau, hipStream_t s);
rbd_status launch_crba(const rbd_model* m, int64_t batch, int64_t ld, const float* q, float* M, hipStream_t s);
rbd_status launch_fwd_dyn(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                          const float* tau, const float* fext, float* qdd, hipStream_t s);
rbd_status launch_aba(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                      const float* tau, const float* fext, float* qdd, hipStream_t s);
rbd_status launch_rnea_jvp(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                           const float* qdd, const float* fext, const float* dq, const float* dqd, const float* dqdd,
                           const float* dfext, float* dtau, hipStream_t s);
rbd_status launch_rnea_vjp(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                           const float* qdd, const float* fext, const float* lam, float* gq, float* gqd, float* gqdd,
                           float* gfext, hipStream_t s);
rbd_status launch_fwd_dyn_jvp(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                              const float* tau, const float* fext, const float* dq, const float* dqd,
                              const float* dtau, const float* dfext, float* qdd, float* dqdd, hipStream_t s);
rbd_status launch_diff_ik(const rbd_model* m, int64_t batch, int64_t ld, const float* q, int frame, const float* tgt,
                          float gain, float lam2, float* qd, hipStream_t s);
rbd_status launch_osc(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd, int frame,
                      const float* tgt, float kp, float kd, float kn, float* tau, hipStream_t s);
rbd_status launch_fwd_dyn_vjp(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                              const float* tau, const float* fext, const float* gqdd, float* gq, float* gqd,
                              float* gtau, float* gfext, hipStream_t s);


// Packed serving launch of one (model, op): d_table holds a PackedHdr-led
// descriptor table in device memory; grid blocks of 256 threads stride over it.
constexpr int kMaxPacked = 4096;
rbd_status launch_packed(const rbd_model* m, int op, const void* d_table, int grid, hipStream_t s);
// Loads the packed kernel of `op` (compiling it if the model's kernels are
// compiled at run time), so that a later launch does nothing but launch.
rbd_status prepare_packed(const rbd_model* m, int op);
// Whether a launch of the packed kernel of `op` loads nothing first (a
// topology compiled ahead of time, or a run-time one whose kernel is loaded).
bool packed_ready(const rbd_model* m, int op);

}  // namespace rbd
