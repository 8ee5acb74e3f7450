// Topology registry and dispatch of the C entry points to the kernels of the
// model's compiled topology.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <vector>

#include "rbd_internal.hpp"
#include "rbd_topologies.hpp"

namespace rbd {

#define RBD_DECL(name, fr, ...) \
  extern const LaunchTable launch_table_##name##_p1, launch_table_##name##_p2, launch_table_##name##_p3, \
      launch_table_##name##_p4, launch_table_##name##_p5, launch_table_##name##_p6, launch_table_##name##_p7;
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

static const LaunchTable* const k_parts[][7] = {
#define RBD_TAB(name, fr, ...)                                                                                  \
  {&launch_table_##name##_p1, &launch_table_##name##_p2, &launch_table_##name##_p3, &launch_table_##name##_p4, \
   &launch_table_##name##_p5, &launch_table_##name##_p6, &launch_table_##name##_p7},
    RBD_TOPOLOGIES(RBD_TAB)
#undef RBD_TAB
};

// The seven parts of a topology merged into one table (built on first use).
static const LaunchTable* merged(int id) {
  static const std::vector<LaunchTable> all = [] {
    std::vector<LaunchTable> v(sizeof(k_parts) / sizeof(k_parts[0]));
    for (size_t i = 0; i < v.size(); ++i) {
      const LaunchTable &a = *k_parts[i][0], &b = *k_parts[i][1], &c = *k_parts[i][2], &d = *k_parts[i][3],
                        &e = *k_parts[i][4], &f = *k_parts[i][5], &g = *k_parts[i][6];
      v[i] = LaunchTable{a.fk,     a.jacobian,   a.rnea,     a.crba,        b.fwd_dyn, c.vjp, d.aba,
                         b.packed, c.packed_vjp, e.rnea_ext, e.fwd_dyn_ext, e.aba_ext, f.jvp, g.diff_ik, g.osc};
    }
    return v;
  }();
  return &all[id];
}

int n_topologies() { return (int)(sizeof(k_topos) / sizeof(k_topos[0])); }
const TopoInfo& topology(int id) { return k_topos[id]; }
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

static const LaunchTable* table_of(const rbd_model* m) {
  return (m->topo >= 0 && m->topo < n_topologies()) ? merged(m->topo) : nullptr;
}

#define RBD_TABLE_OR_FAIL(m)                                                     \
  const LaunchTable* lt = table_of(m);                                           \
  if (!lt) return fail(RBD_E_UNSUPPORTED, "no compiled kernel for this model");

rbd_status launch_fk(const rbd_model* m, int64_t batch, int64_t ld, const float* q, float* T, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  RBD_TABLE_OR_FAIL(m);
  return lt->fk(m->d_tab, batch, ld, q, T, s);
}

rbd_status launch_jacobian(const rbd_model* m, int64_t batch, int64_t ld, const float* q, int32_t n_frames,
                           const int32_t* frames, float* J, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  RBD_TABLE_OR_FAIL(m);
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
  return lt->jacobian(m->d_tab, batch, ld, q, js, J, s);
}

rbd_status launch_rnea(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                       const float* qdd, const float* fext, float* tau, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  RBD_TABLE_OR_FAIL(m);
  return (fext ? lt->rnea_ext : lt->rnea)(m->d_tab, batch, ld, q, qd, qdd, fext, tau, s);
}

rbd_status launch_crba(const rbd_model* m, int64_t batch, int64_t ld, const float* q, float* M, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  RBD_TABLE_OR_FAIL(m);
  return lt->crba(m->d_tab, batch, ld, q, M, s);
}

rbd_status launch_fwd_dyn(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                          const float* tau, const float* fext, float* qdd, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  RBD_TABLE_OR_FAIL(m);
  return (fext ? lt->fwd_dyn_ext : lt->fwd_dyn)(m->d_tab, batch, ld, q, qd, tau, fext, qdd, s);
}

rbd_status launch_aba(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                      const float* tau, const float* fext, float* qdd, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  RBD_TABLE_OR_FAIL(m);
  return (fext ? lt->aba_ext : lt->aba)(m->d_tab, batch, ld, q, qd, tau, fext, qdd, s);
}

rbd_status launch_fwd_dyn_jvp(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                              const float* tau, const float* dq, const float* dqd, const float* dtau, float* qdd,
                              float* dqdd, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  RBD_TABLE_OR_FAIL(m);
  return lt->jvp(m->d_tab, batch, ld, q, qd, tau, dq, dqd, dtau, qdd, dqdd, s);
}

rbd_status launch_diff_ik(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* tgt,
                          float gain, float lam2, float* qd, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  RBD_TABLE_OR_FAIL(m);
  return lt->diff_ik(m->d_tab, batch, ld, q, tgt, gain, lam2, qd, s);
}

rbd_status launch_osc(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                      const float* tgt, float kp, float kd, float kn, float* tau, hipStream_t s) {
  if (batch == 0) return RBD_OK;
  RBD_TABLE_OR_FAIL(m);
  return lt->osc(m->d_tab, batch, ld, q, qd, tgt, kp, kd, kn, tau, s);
}

rbd_status launch_fwd_dyn_vjp(const rbd_model* m, int64_t batch, int64_t ld, const float* q, const float* qd,
                              const float* tau, const float* gqdd, float* gq, float* gqd, float* gtau,
                              hipStream_t s) {
  if (batch == 0 || (!gq && !gqd && !gtau)) return RBD_OK;
  RBD_TABLE_OR_FAIL(m);
  return lt->vjp(m->d_tab, batch, ld, q, qd, tau, gqdd, gq, gqd, gtau, s);
}

rbd_status launch_packed(const rbd_model* m, int op, const void* d_table, int grid, hipStream_t s) {
  RBD_TABLE_OR_FAIL(m);
  if (op == RBD_OP_FWD_DYN_VJP) return lt->packed_vjp(op, m->d_tab, d_table, grid, s);
  return lt->packed(op, m->d_tab, d_table, grid, s);
}

}  // namespace rbd
