// Topology registry and dispatch of the C entry points: each launcher picks a
// kernel of the model's kernel set (variant and launch shape from the model's
// sizes) and launches it, ahead-of-time and run-time-compiled kernels alike.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <vector>

#include "rbd_internal.hpp"
#include "rbd_topologies.hpp"

namespace rbd {

static_assert(kOpFwdDyn == RBD_OP_FWD_DYN && kOpRnea == RBD_OP_RNEA && kOpFwdDynVjp == RBD_OP_FWD_DYN_VJP,
              "packed operation ids differ from rbd_op");

#define RBD_DECL(name, fr, ...)                                                                              \
  void kernels_##name##_p1(const void**);                                                                    \
  void kernels_##name##_p2(const void**);                                                                    \
  void kernels_##name##_p3(const void**);                                                                    \
  void kernels_##name##_p4(const void**);                                                                    \
  void kernels_##name##_p5(const void**);                                                                    \
  void kernels_##name##_p6(const void**);                                                                    \
  void kernels_##name##_p7(const void**);                                                                    \
  void kernels_##name##_p8(const void**);
RBD_TOPOLOGIES(RBD_DECL)
#undef RBD_DECL

#define RBD_PARENTS(name, fr, ...) static const int k_par_##name[] = {__VA_ARGS__};
RBD_TOPOLOGIES(RBD_PARENTS)
#undef RBD_PARENTS

static const TopoInfo k_topos[] = {
#define RBD_INFO(name, fr, ...) {#name, fr, (int)(sizeof(k_par_##name) / sizeof(int)), k_par_##name},
    RBD_TOPOLOGIES(RBD_INFO)
#undef RBD_INFO
};

using FillFn = void (*)(const void**);
static const FillFn k_fill[][kParts] = {
#define RBD_TAB(name, fr, ...)                                                                            \
  {&kernels_##name##_p1, &kernels_##name##_p2, &kernels_##name##_p3, &kernels_##name##_p4, \
   &kernels_##name##_p5, &kernels_##name##_p6, &kernels_##name##_p7, &kernels_##name##_p8},
    RBD_TOPOLOGIES(RBD_TAB)
#undef RBD_TAB
};

int n_topologies() { return (int)(sizeof(k_topos) / sizeof(k_topos[0])); }
const TopoInfo& topology(int id) { return k_topos[id]; }

// The kernel table of a compiled topology: its parts merged (built on first
// use).
const KernelSet* aot_kernels(int id) {
  static const std::vector<KernelSet> all = [] {
    std::vector<KernelSet> v(n_topologies());
    for (int i = 0; i < n_topologies(); ++i) {
      for (int p = 0; p < kParts; ++p) k_fill[i][p](v[i].aot);
      v[i].name = k_topos[i].name;
    }
    return v;
  }();
  return (id >= 0 && id < n_topologies()) ? &all[id] : nullptr;
}

int find_topology(bool floating, int n, const int32_t* parent) {
  for (int id = 0; id < n_topologies(); ++id) {
    const TopoInfo& t = k_topos[id];
    if (t.floating != floating || t.n != n) continue;
    bool same = true;
    for (int i = 0; i < n && same; ++i) same = t.parent[i] == parent[i];
    if (same) return id;
  }
  return -1;
}

bool preload_inputs(bool topology_default) {
  static const int env = [] {
    const char* e = std::getenv("RBD_PRELOAD");
    if (!e) return -1;
    return std::strcmp(e, "0") == 0 ? 0 : 1;
  }();
  return env < 0 ? topology_default : env == 1;
}

// Whether the adjoint of a large tree at a batch up to half the chip runs on
// two waves per 64 instances: yes, unless the environment variable
// RBD_VJP_SPLIT is 0 (for measurement).
static bool split_adjoint() {
  static const bool on = [] {
    const char* e = std::getenv("RBD_VJP_SPLIT");
    return !(e && std::strcmp(e, "0") == 0);
  }();
  return on;
}

// ------------------------------------------------------------------ launch
static inline unsigned grid_for(int64_t batch) { return (unsigned)((batch + kBlock - 1) / kBlock); }

// Launch shape of the heavy per-lane kernels (forward dynamics, ABA, the two
// derivatives, OSC), which are register-bound to one wave per SIMD. Up to
// 65536 lanes (one wave for each of the 256 CUs x 4 SIMDs) they run in 64-lane
// blocks: below that size 256-lane blocks would leave whole CUs idle and stack
// four waves on the others, while 64-lane blocks spread the waves over every
// CU (the humanoid's VJP and JVP at batch 32768 measured 3-5 % faster; at
// 65536 the two shapes are equal). Larger batches keep 256-lane blocks, which
// are as fast or faster there.
constexpr int64_t kOneWavePerSimd = 256 * 4 * 64;
struct Shape {
  dim3 grid, block;
  unsigned lds = 0;  // dynamic LDS bytes per block
};
static inline Shape heavy_shape(int64_t batch) {
  const unsigned blk = batch <= kOneWavePerSimd ? 64 : kBlock;
  return {dim3((unsigned)((batch + blk - 1) / blk)), dim3(blk)};
}
static inline Shape plain_shape(int64_t batch) { return {dim3(grid_for(batch)), dim3(kBlock)}; }

// Trees above 16 DoFs: the large-tree choices the kernels are tuned for
// (scalar-base addressing is chosen in the kernels themselves).
static inline bool large(const rbd_model* m) { return m->nv > 16; }

// Launches kernel `id` of the model's set; args point to the kernel's
// arguments in order.
static rbd_status launch(const rbd_model* m, KernelId id, Shape sh, void** args, hipStream_t s, const char* what) {
  const KernelSet* ks = m->ks;
  if (!ks) return fail(RBD_E_UNSUPPORTED, "%s: the model has no kernels", what);
  hipError_t e;
  if (ks->is_jit) {
    hipFunction_t f = nullptr;
    const rbd_status st = jit_function(ks, id, &f);
    if (st != RBD_OK) return st;
    e = hipModuleLaunchKernel(f, sh.grid.x, sh.grid.y, sh.grid.z, sh.block.x, sh.block.y, sh.block.z, sh.lds, s,
                              args, nullptr);
  } else {
    if (!ks->aot[id]) return fail(RBD_E_UNSUPPORTED, "%s: kernel %d was not compiled", what, (int)id);
    e = hipLaunchKernel(ks->aot[id], sh.grid, sh.block, args, sh.lds, s);
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return fail(RBD_E_LAUNCH, "%s: launch failed: %s", what, hipGetErrorString(e));
  return RBD_OK;
}

rbd_status launch_fk(const rbd_model* m, int64_t batch, int64_t ld, const float* q, float* T, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  const float* tab = m->d_tab;
  void* a[] = {&tab, &batch, &ld, &q, &T};
  return launch(m, KID_FK, plain_shape(batch), a, s, "rbd_fk");
}

rbd_status launch_jacobian(const rbd_model* m, int64_t batch, int64_t ld, const float* q, int32_t n_frames,
                           const int32_t* frames, float* J, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  JacSlots js{};
  js.n_frames = n_frames;
  int count[65] = {0};
  for (int f = 0; f < n_frames; ++f) count[frames[f]]++;
  js.beg[0] = 0;
  for (int i = 0; i < 64; ++i) js.beg[i + 1] = (int16_t)(js.beg[i] + count[i]);
  int fill[65] = {0};
  for (int f = 0; f < n_frames; ++f) {
    const int i = frames[f];
    js.slot[js.beg[i] + fill[i]++] = (int16_t)f;
  }
  const float* tab = m->d_tab;
  void* a[] = {&tab, &batch, &ld, &q, &js, &J};
  return launch(m, KID_JACOBIAN, plain_shape(batch), a, s, "rbd_jacobian");
}

// Large trees issue every input load at kernel entry (without external
// forces); small ones keep their occupancy instead (measured).
rbd_status launch_rnea(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                       const float* qdd, const float* fext, float* tau, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  KernelId id;
  if (fext) id = qdd ? KID_RNEA_EXT : KID_RNEA_BIAS_EXT;
  else if (large(m) && preload_inputs(true)) id = qdd ? KID_RNEA_PRE : KID_RNEA_BIAS_PRE;
  else id = qdd ? KID_RNEA : KID_RNEA_BIAS;
  const float* tab = m->d_tab;
  void* a[] = {&tab, &batch, &ld, &q, &qd, &qdd, &fext, &tau};
  return launch(m, id, plain_shape(batch), a, s, "rbd_rnea");
}

rbd_status launch_crba(const rbd_model* m, int64_t batch, int64_t ld, const float* q, float* M, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  const float* tab = m->d_tab;
  void* a[] = {&tab, &batch, &ld, &q, &M};
  return launch(m, KID_CRBA, plain_shape(batch), a, s, "rbd_crba");
}

rbd_status launch_fwd_dyn(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                          const float* tau, const float* fext, float* qdd, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  const bool pre = preload_inputs(large(m));
  const KernelId id = fext ? (pre ? KID_FWD_DYN_PRE_EXT : KID_FWD_DYN_EXT) : (pre ? KID_FWD_DYN_PRE : KID_FWD_DYN);
  const float* tab = m->d_tab;
  void* a[] = {&tab, &batch, &ld, &q, &qd, &tau, &fext, &qdd};
  return launch(m, id, heavy_shape(batch), a, s, "rbd_fwd_dyn");
}

// With external forces the articulated-body sweep is faster loading its
// inputs in place (humanoid: 77.8 vs 81.6 us).
rbd_status launch_aba(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                      const float* tau, const float* fext, float* qdd, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  const bool pre = preload_inputs(large(m) && !fext);
  const KernelId id = fext ? (pre ? KID_ABA_PRE_EXT : KID_ABA_EXT) : (pre ? KID_ABA_PRE : KID_ABA);
  const float* tab = m->d_tab;
  void* a[] = {&tab, &batch, &ld, &q, &qd, &tau, &fext, &qdd};
  return launch(m, id, heavy_shape(batch), a, s, "rbd_aba");
}

rbd_status launch_fwd_dyn_jvp(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                              const float* tau, const float* fext, const float* dq, const float* dqd,
                              const float* dtau, const float* dfext, float* qdd, float* dqdd, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  const float* tab = m->d_tab;
  void* a[] = {&tab, &batch, &ld, &q, &qd, &tau, &dq, &dqd, &dtau, &qdd, &dqdd, &fext, &dfext};
  const bool ext = fext || dfext;
  if (large(m) && batch <= kOneWavePerSimd / 2) {
    // two waves per 64 instances: the factor of M on its own wave, in
    // parallel with the solve for qdd and the tangent
    const Shape sh{dim3((unsigned)((batch + kTileLanes - 1) / kTileLanes)), dim3(2 * kTileLanes),
                   (unsigned)(2 * m->nv * kTileLanes * sizeof(float))};
    return launch(m, ext ? KID_JVP_EXT_SPLIT : KID_JVP_SPLIT, sh, a, s, "rbd_fwd_dyn_jvp");
  }
  return launch(m, ext ? KID_JVP_EXT : KID_JVP, heavy_shape(batch), a, s, "rbd_fwd_dyn_jvp");
}

rbd_status launch_rnea_jvp(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                           const float* qdd, const float* fext, const float* dq, const float* dqd, const float* dqdd,
                           const float* dfext, float* dtau, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  const float* tab = m->d_tab;
  void* a[] = {&tab, &batch, &ld, &q, &qd, &qdd, &dq, &dqd, &dqdd, &dtau, &fext, &dfext};
  const bool ext = fext || dfext;
  const KernelId id = ext ? KID_RNEA_JVP_EXT : (preload_inputs(large(m)) ? KID_RNEA_JVP_PRE : KID_RNEA_JVP);
  return launch(m, id, heavy_shape(batch), a, s, "rbd_rnea_jvp");
}

rbd_status launch_rnea_vjp(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                           const float* qdd, const float* fext, const float* lam, float* gq, float* gqd, float* gqdd,
                           float* gfext, hipStream_t s) {
  if (batch == 0 || (!gq && !gqd && !gqdd && !gfext)) return RBD_OK;
  // external forces matter to g_q and the force cotangent only
  const bool ext = gfext || (fext && gq);
  const float* tab = m->d_tab;
  void* a[] = {&tab, &batch, &ld, &q, &qd, &qdd, &lam, &gq, &gqd, &gqdd, &fext, &gfext};
  return launch(m, ext ? KID_RNEA_VJP_EXT : KID_RNEA_VJP, heavy_shape(batch), a, s, "rbd_rnea_vjp");
}

// The controller kernel of `frame`: the set's own for the last body, else one
// compiled for that frame at run time on first use.
static rbd_status launch_frame(const rbd_model* m, bool osc, int frame, Shape sh, void** args, hipStream_t s,
                               const char* what) {
  if (frame == m->n - 1) return launch(m, osc ? KID_OSC : KID_DIFF_IK, sh, args, s, what);
  hipFunction_t f = nullptr;
  const rbd_status st = jit_frame_function(m->floating, m->n, m->parent.data(), m->device, osc, frame, &f);
  if (st != RBD_OK) return st;
  hipError_t e = hipModuleLaunchKernel(f, sh.grid.x, sh.grid.y, sh.grid.z, sh.block.x, sh.block.y, sh.block.z, 0, s,
                                       args, nullptr);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return fail(RBD_E_LAUNCH, "%s: launch failed: %s", what, hipGetErrorString(e));
  return RBD_OK;
}

rbd_status launch_diff_ik(const rbd_model* m, int64_t batch, int64_t ld, const float* q, int frame, const float* tgt,
                          float gain, float lam2, float* qd, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  const float* tab = m->d_tab;
  void* a[] = {&tab, &batch, &ld, &q, &tgt, &gain, &lam2, &qd};
  return launch_frame(m, false, frame, plain_shape(batch), a, s, "rbd_diff_ik");
}

rbd_status launch_osc(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd, int frame,
                      const float* tgt, float kp, float kd, float kn, float* tau, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  const float* tab = m->d_tab;
  void* a[] = {&tab, &batch, &ld, &q, &qd, &tgt, &kp, &kd, &kn, &tau};
  return launch_frame(m, true, frame, heavy_shape(batch), a, s, "rbd_osc");
}

// Between the solve and the adjoint sweep, q-double-dot and lam park: for a
// large tree in LDS, whatever outputs are requested (64-lane blocks, one wave
// each, 2 nv floats per lane); for a small tree in the g_qd and g_tau rows
// when both are requested (the adjoint overwrites them only after reading
// them), else in registers.
rbd_status launch_fwd_dyn_vjp(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                              const float* tau, const float* fext, const float* gqdd, float* gq, float* gqd,
                              float* gtau, float* gfext, hipStream_t s) {
  if (batch == 0 || (!gq && !gqd && !gtau && !gfext)) return RBD_OK;
  // external forces matter to g_q and g_qd (through qdd) and the force
  // cotangent; g_tau = M^-1 g_qdd does not depend on them
  const bool ext = gfext || (fext && (gq || gqd));
  const float* tab = m->d_tab;
  void* a[] = {&tab, &batch, &ld, &q, &qd, &tau, &gqdd, &gq, &gqd, &gtau, &fext, &gfext};
  if (large(m) && (gq || gqd || gfext)) {
    const unsigned grid = (unsigned)((batch + kTileLanes - 1) / kTileLanes);
    const unsigned lds = (unsigned)(2 * m->nv * kTileLanes * sizeof(float));
    if (batch <= kOneWavePerSimd / 2 && split_adjoint()) {
      // two waves per 64 instances: lam = M^-1 g_qdd on its own wave, in
      // parallel with the solve for qdd
      return launch(m, ext ? KID_VJP_EXT_SPLIT : KID_VJP_SPLIT, Shape{dim3(grid), dim3(2 * kTileLanes), lds}, a, s,
                    "rbd_fwd_dyn_vjp");
    }
    return launch(m, ext ? KID_VJP_EXT_LDS : KID_VJP_LDS, Shape{dim3(grid), dim3(kTileLanes), lds}, a, s,
                  "rbd_fwd_dyn_vjp");
  }
  KernelId id;
  if (ext) id = (gqd && gtau) ? KID_VJP_EXT_PARK : KID_VJP_EXT_REGS;
  else if (gqd && gtau) id = KID_VJP_PARK;
  else if (gq || gqd) id = KID_VJP_REGS;
  else id = KID_VJP_TAU;
  return launch(m, id, heavy_shape(batch), a, s, "rbd_fwd_dyn_vjp");
}

static KernelId packed_id(int op) {
  return op == kOpFwdDynVjp ? KID_PACKED_VJP : (op == kOpFwdDyn ? KID_PACKED_FWD_DYN : KID_PACKED_RNEA);
}

rbd_status prepare_packed(const rbd_model* m, int op) {
  const KernelSet* ks = m->ks;
  if (!ks) return fail(RBD_E_UNSUPPORTED, "packed launch: the model has no kernels");
  if (!ks->is_jit) return RBD_OK;
  hipFunction_t f = nullptr;
  return jit_function(ks, packed_id(op), &f);
}

bool packed_ready(const rbd_model* m, int op) {
  const KernelSet* ks = m->ks;
  if (!ks) return false;
  if (!ks->is_jit) return ks->aot[packed_id(op)] != nullptr;
  return ks->jit[packed_id(op)].load(std::memory_order_acquire) != nullptr;
}

rbd_status launch_packed(const rbd_model* m, int op, const void* d_table, int grid, hipStream_t s) {
  const KernelId id = packed_id(op);
  const float* tab = m->d_tab;
  const uint8_t* t = static_cast<const uint8_t*>(d_table);
  void* a[] = {&tab, &t};
  return launch(m, id, Shape{dim3((unsigned)grid), dim3(kBlock)}, a, s, "packed launch");
}

}  // namespace rbd
