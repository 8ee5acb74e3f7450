// HIP kernels for gfx950, templated on the compiled tree type, and the host
// launch wrappers each topology's translation unit instantiates. The per-lane
// algorithms live in rbd_lane.hpp.
#pragma once

#include <hip/hip_runtime.h>

#include "rbd_internal.hpp"
#include "rbd_lane.hpp"

namespace rbd {

constexpr int kBlock = 256;

RBD_DI uint32_t lane_id() { return blockIdx.x * blockDim.x + threadIdx.x; }

// The same pointer value, hidden from the optimiser (an empty asm on its
// scalar register, no instruction). A kernel that runs several sweeps gives
// each its own copies of the table and input pointers and of the row stride,
// so model constants, inputs, row addresses and what is computed from them
// (joint sines and cosines) are reloaded and recomputed in each sweep instead
// of being held in registers across all of them.
RBD_DI const float* opaque(const float* p) {
  asm volatile("" : "+s"(p));
  return p;
}
RBD_DI int64_t opaque(int64_t x) {
  asm volatile("" : "+s"(x));
  return x;
}
// Views of outputs that a later sweep of the same kernel reads back: not
// restrict-qualified, so the compiler keeps every load before the store that
// later overwrites the same element.
template <bool SB>
struct InAliasT {
  const float* base;
  int64_t ld;
  uint32_t lane;
  RBD_DI float operator()(int c) const {
    if constexpr (SB) return *lane_ptr(base + c * ld, lane);
    else return (base + c * ld)[lane];
  }
};
template <bool SB>
struct OutAliasT {
  float* base;
  int64_t ld;
  uint32_t lane;
  RBD_DI void operator()(int c, float v) const {
    if constexpr (SB) *lane_ptr(base + c * ld, lane) = v;
    else (base + c * ld)[lane] = v;
  }
};
using InAlias = InAliasT<true>;
using OutAlias = OutAliasT<true>;
template <bool SB>
struct OutAliasPT : OutAliasT<SB> {
  using In = InAliasT<SB>;
};
using OutAliasP = OutAliasPT<true>;

// The lane I/O views of a tree's kernels (kScalarBase picks the address form).
#define RBD_LANE_IO(TP)                           \
  constexpr bool kSB_ = kScalarBase<TP>;          \
  using In = InT<kSB_>;                           \
  using Out = OutT<kSB_>;                         \
  using InAlias = InAliasT<kSB_>;                 \
  using OutAlias = OutAliasT<kSB_>;               \
  using OutAliasP = OutAliasPT<kSB_>;             \
  (void)kSB_

// Between two sweeps: keeps the scheduler from starting the next sweep's
// loads inside the previous one, where its registers are all in use.
RBD_DI void sweep_boundary() { __builtin_amdgcn_sched_barrier(0); }

// Registers of one lane holding a preloaded input vector.
struct RegView {
  const float* x;
  RBD_DI float operator()(int k) const { return x[k]; }
};

template <class TP>
__global__ __launch_bounds__(kBlock) void k_fk(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                               const float* __restrict__ q, float* __restrict__ T) {
  RBD_LANE_IO(TP);
  const uint32_t b = lane_id();
  if (b >= batch) return;
  fk_lane<TP>(tab, In{q, ld, b}, OutNT{T, ld, b});
}

template <class TP>
__global__ __launch_bounds__(kBlock) void k_jacobian(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                     const float* __restrict__ q, JacSlots js,
                                                     float* __restrict__ J) {
  RBD_LANE_IO(TP);
  const uint32_t b = lane_id();
  if (b >= batch) return;
  jac_lane<TP>(tab, In{q, ld, b}, js, J, ld, b);
}

// EXT: per-body external forces (fext, [6 n][ld]) enter the force balance.
// PRE (no external forces): every input load is issued at entry, as in
// k_fwd_dyn.
template <class TP, bool HAS_QDD, bool EXT, bool PRE = false>
__global__ __launch_bounds__(kBlock) void k_rnea(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                 const float* __restrict__ q, const float* __restrict__ qd,
                                                 const float* __restrict__ qdd, const float* __restrict__ fext,
                                                 float* __restrict__ tau) {
  RBD_LANE_IO(TP);
  const uint32_t b = lane_id();
  if (b >= batch) return;
  if constexpr (PRE && !EXT) {
    constexpr int NQ = TP::NQ, NV = TP::NV;
    float qv[NQ], qdv[NV], qddv[NV];
    const In qi{q, ld, b}, qdi{qd, ld, b}, qddi{HAS_QDD ? qdd : qd, ld, b};
    sfor<0, NQ>([&](auto K_) __attribute__((always_inline)) { qv[decltype(K_)::value] = qi(decltype(K_)::value); });
    sfor<0, NV>([&](auto K_) __attribute__((always_inline)) {
      qdv[decltype(K_)::value] = qdi(decltype(K_)::value);
      if constexpr (HAS_QDD) qddv[decltype(K_)::value] = qddi(decltype(K_)::value);
    });
    rnea_lane<TP, HAS_QDD>(tab, RegView{qv}, RegView{qdv}, RegView{HAS_QDD ? qddv : qdv}, Out{tau, ld, b});
  } else if constexpr (EXT)
    rnea_lane<TP, HAS_QDD>(tab, In{q, ld, b}, In{qd, ld, b}, In{HAS_QDD ? qdd : q, ld, b}, Out{tau, ld, b},
                           FextIn{{fext, ld, b}});
  else
    rnea_lane<TP, HAS_QDD>(tab, In{q, ld, b}, In{qd, ld, b}, In{HAS_QDD ? qdd : q, ld, b}, Out{tau, ld, b});
}

template <class TP>
__global__ __launch_bounds__(kBlock) void k_crba(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                 const float* __restrict__ q, float* __restrict__ M) {
  RBD_LANE_IO(TP);
  const uint32_t b = lane_id();
  if (b >= batch) return;
  crba_lane<TP>(tab, In{q, ld, b}, M, ld, b);
}

template <class X>
struct RhsOne {
  X tau;
  RBD_DI float operator()(int, int k) const { return tau(k); }
};
template <class Y>
struct SinkOne {
  Y x;
  RBD_DI void operator()(int, int k, float v) const { x(k, v); }
};

// PRE = true issues every input load of the lane at entry (106 for the
// humanoid), so their latency overlaps the first bodies' arithmetic instead of
// stalling the single wave of each SIMD at every body.
// The external-force view of a kernel: FextIn over fext, or nothing.
template <bool EXT>
RBD_DI auto fext_view(const float* fext, int64_t ld, uint32_t b) {
  if constexpr (EXT) return FextIn{{fext, ld, b}};
  else return NoFext{};
}

// EXT as for k_rnea.
template <class TP, bool PRE, bool EXT>
__global__ __launch_bounds__(kBlock) void k_fwd_dyn(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                    const float* __restrict__ q, const float* __restrict__ qd,
                                                    const float* __restrict__ tau, const float* __restrict__ fext,
                                                    float* __restrict__ qdd) {
  RBD_LANE_IO(TP);
  const uint32_t b = lane_id();
  if (b >= batch) return;
  const auto fx = fext_view<EXT>(fext, ld, b);
  if constexpr (PRE) {
    constexpr int NQ = TP::NQ, NV = TP::NV;
    float qv[NQ], qdv[NV], tv[NV];
    const In qi{q, ld, b}, qdi{qd, ld, b}, ti{tau, ld, b};
    sfor<0, NQ>([&](auto K_) __attribute__((always_inline)) { qv[decltype(K_)::value] = qi(decltype(K_)::value); });
    sfor<0, NV>([&](auto K_) __attribute__((always_inline)) {
      qdv[decltype(K_)::value] = qdi(decltype(K_)::value);
      tv[decltype(K_)::value] = ti(decltype(K_)::value);
    });
    fwd_dyn_lane<TP, 1>(tab, RegView{qv}, RegView{qdv}, RhsOne<RegView>{RegView{tv}}, SinkOne<Out>{Out{qdd, ld, b}},
                        fx);
  } else {
    fwd_dyn_lane<TP, 1>(tab, In{q, ld, b}, In{qd, ld, b}, RhsOne<In>{In{tau, ld, b}}, SinkOne<Out>{Out{qdd, ld, b}},
                        fx);
  }
}

// Forward dynamics by the articulated-body algorithm; PRE as for k_fwd_dyn,
// EXT as for k_rnea.
template <class TP, bool PRE, bool EXT>
__global__ __launch_bounds__(kBlock) void k_aba(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                const float* __restrict__ q, const float* __restrict__ qd,
                                                const float* __restrict__ tau, const float* __restrict__ fext,
                                                float* __restrict__ qdd) {
  RBD_LANE_IO(TP);
  const uint32_t b = lane_id();
  if (b >= batch) return;
  const auto fx = fext_view<EXT>(fext, ld, b);
  if constexpr (PRE) {
    constexpr int NQ = TP::NQ, NV = TP::NV;
    float qv[NQ], qdv[NV], tv[NV];
    const In qi{q, ld, b}, qdi{qd, ld, b}, ti{tau, ld, b};
    sfor<0, NQ>([&](auto K_) __attribute__((always_inline)) { qv[decltype(K_)::value] = qi(decltype(K_)::value); });
    sfor<0, NV>([&](auto K_) __attribute__((always_inline)) {
      qdv[decltype(K_)::value] = qdi(decltype(K_)::value);
      tv[decltype(K_)::value] = ti(decltype(K_)::value);
    });
    aba_lane<TP>(tab, RegView{qv}, RegView{qdv}, RegView{tv}, Out{qdd, ld, b}, fx);
  } else {
    aba_lane<TP>(tab, In{q, ld, b}, In{qd, ld, b}, In{tau, ld, b}, Out{qdd, ld, b}, fx);
  }
}

// ---- fwd_dyn adjoint: solve M [qdd, lam] = [tau - h, gbar] with one factor,
// write g_tau = lam, then run the inverse-dynamics adjoint at (q, qd, qdd).
template <class X>
struct RhsTwo {
  X tau, gbar;
  RBD_DI float operator()(int r, int k) const { return r == 0 ? tau(k) : gbar(k); }
};
struct SinkRegs {
  float* qdd;
  float* lam;
  RBD_DI void operator()(int r, int k, float v) const {
    if (r == 0) qdd[k] = v; else lam[k] = v;
  }
};
// An output that may be absent (null base).
template <class Y>
struct OutOpt {
  Y y;
  bool on;
  RBD_DI void operator()(int c, float v) const {
    if (on) y(c, v);
  }
};
// q-double-dot and lam parked in the g_qd and g_tau outputs go through the
// alias views above.
template <class Y>
struct SinkTwo {
  Y qdd, lam;
  RBD_DI void operator()(int r, int k, float v) const {
    if (r == 0) qdd(k, v); else lam(k, v);
  }
};

template <class TP, bool ADJ, class QI, class X, class GQ, class GQD, class GT>
RBD_DI void vjp_lane(const float* __restrict__ tab, const QI& q, const X& qd, const X& tau, const X& gqdd,
                     const GQ& gq, const GQD& gqd, const GT& gtau) {
  constexpr int NV = TP::NV;
  float qddv[NV], lam[NV];
  fwd_dyn_lane<TP, 2>(tab, q, qd, RhsTwo<X>{tau, gqdd}, SinkRegs{qddv, lam});
  sfor<0, NV>([&](auto K_) __attribute__((always_inline)) {
    constexpr int K = decltype(K_)::value;
    gtau(K, lam[K]);
  });
  if constexpr (ADJ) id_adjoint_lane<TP>(tab, q, qd, RegView{qddv}, RegView{lam}, gq, gqd);
}

// q-double-dot parked in g_qd and lam in g_tau between the solve and the
// adjoint sweep, instead of 2 nv registers held across it. Every element is
// read by its body's forward step before that body's backward step
// overwrites g_qd.
template <class TP, class QI, class X, class GQ, class P>
RBD_DI void vjp_lane_parked(const float* __restrict__ tab, const QI& q, const X& qd, const X& tau, const X& gqdd,
                            const GQ& gq, const P& gqd_out, const P& gtau_out, const typename P::In& gqd_in,
                            const typename P::In& gtau_in) {
  fwd_dyn_lane<TP, 2>(tab, q, qd, RhsTwo<X>{tau, gqdd}, SinkTwo<P>{gqd_out, gtau_out});
  id_adjoint_lane<TP>(tab, q, qd, gqd_in, gtau_in, gq, gqd_out);
}

struct RowAlias {
  float* p;
  RBD_DI void operator()(int c, float v) const { p[c] = v; }
  struct In {
    const float* p;
    RBD_DI float operator()(int c) const { return p[c]; }
  };
};

// MODE 0: g_tau only; 1: adjoint with q-double-dot and lam in registers (some
// output absent); 2: adjoint with both parked in g_qd and g_tau (passed again
// as park_qdd and park_lam); 3 (large trees): as 2, parked where the launcher
// chooses, g_qd optional.
template <class TP, int MODE>
__global__ __launch_bounds__(kBlock) void k_fwd_dyn_vjp(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                        const float* __restrict__ q, const float* __restrict__ qd,
                                                        const float* __restrict__ tau,
                                                        const float* __restrict__ gqdd, float* gq, float* gqd,
                                                        float* gtau, float* park_qdd, float* park_lam) {
  RBD_LANE_IO(TP);
  const uint32_t b = lane_id();
  if (b >= batch) return;
  const In qi{q, ld, b}, qdi{qd, ld, b}, ti{tau, ld, b}, gi{gqdd, ld, b};
  const OutOpt<OutAlias> gqo{OutAlias{gq, ld, b}, gq != nullptr};
  if constexpr (MODE >= 2 && TP::NV > 16) {
    // the two sweeps of vjp_lane_parked, the second on fresh views (its own
    // table and input pointers and row stride): a large tree's first sweep
    // uses every register, and values kept for the second one spill
    // (measured: 1028 -> 400 B/lane of scratch, 126 -> 108 us for the
    // humanoid; a small tree is faster keeping them)
    // q-double-dot and lam park in g_qd and g_tau (MODE 2) or in park_qdd and
    // park_lam (MODE 3, see the launcher)
    float* const pq = MODE == 2 ? gqd : park_qdd;
    float* const pl = MODE == 2 ? gtau : park_lam;
    const OutAliasP pd{{pq, ld, b}}, pt{{pl, ld, b}};
    fwd_dyn_lane<TP, 2>(tab, qi, qdi, RhsTwo<In>{ti, gi}, SinkTwo<OutAliasP>{pd, pt});
    sweep_boundary();
    const int64_t l2 = opaque(ld);
    const OutOpt<OutAlias> gqo2{OutAlias{gq, l2, b}, gq != nullptr};
    if constexpr (MODE == 2)
      id_adjoint_lane<TP>(opaque(tab), In{opaque(q), l2, b}, In{opaque(qd), l2, b}, InAlias{pq, l2, b},
                          InAlias{pl, l2, b}, gqo2, OutAlias{gqd, l2, b});
    else
      id_adjoint_lane<TP>(opaque(tab), In{opaque(q), l2, b}, In{opaque(qd), l2, b}, InAlias{pq, l2, b},
                          InAlias{pl, l2, b}, gqo2, OutOpt<OutAlias>{OutAlias{gqd, l2, b}, gqd != nullptr});
  } else if constexpr (MODE == 2) {
    const OutAliasP pd{{gqd, ld, b}}, pt{{gtau, ld, b}};
    vjp_lane_parked<TP>(tab, qi, qdi, ti, gi, gqo, pd, pt, InAlias{gqd, ld, b}, InAlias{gtau, ld, b});
  } else {
    vjp_lane<TP, MODE == 1>(tab, qi, qdi, ti, gi, gqo, OutOpt<OutAlias>{OutAlias{gqd, ld, b}, gqd != nullptr},
                            OutOpt<OutAlias>{OutAlias{gtau, ld, b}, gtau != nullptr});
  }
}

// ---- fwd_dyn tangent, three sweeps of one lane: qdd by the fused solve
// (parked in the qdd output when one is given, else in dqdd), the tangent of
// inverse dynamics writing dtau - d(ID) into dqdd, and the solve with M in
// place (each right-hand-side entry is read when its subtree closes, every
// result written after the sweep). Neither output is restrict-qualified, so
// loads of parked values stay ordered with the stores.
template <class TP>
__global__ __launch_bounds__(kBlock) void k_fwd_dyn_jvp(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                        const float* __restrict__ q, const float* __restrict__ qd,
                                                        const float* __restrict__ tau, const float* __restrict__ dq,
                                                        const float* __restrict__ dqd,
                                                        const float* __restrict__ dtau, float* qdd, float* dqdd) {
  RBD_LANE_IO(TP);
  const uint32_t b = lane_id();
  if (b >= batch) return;
  float* park = qdd ? qdd : dqdd;
  fwd_dyn_lane<TP, 1>(tab, In{q, ld, b}, In{qd, ld, b}, RhsOne<In>{In{tau, ld, b}},
                      SinkOne<OutAlias>{OutAlias{park, ld, b}});
  // a large tree gives each sweep fresh views (see k_fwd_dyn_vjp)
  constexpr bool kFresh = TP::NV > 16;
  auto view = [](auto x) __attribute__((always_inline)) {
    if constexpr (kFresh) return opaque(x);
    else return x;
  };
  const int64_t ld2 = view(ld);
  id_tangent_lane<TP>(view(tab), In{view(q), ld2, b}, In{view(qd), ld2, b}, InAlias{park, ld2, b},
                      In{dq, ld2, b}, In{dqd, ld2, b}, In{dtau, ld2, b}, OutAlias{dqdd, ld2, b});
  const int64_t ld3 = view(ld2);
  fwd_dyn_lane<TP, 1, In, In, RhsOne<InAlias>, SinkOne<OutAlias>, NoFext, false>(
      view(tab), In{view(q), ld3, b}, In{qd, ld3, b}, RhsOne<InAlias>{InAlias{dqdd, ld3, b}},
      SinkOne<OutAlias>{OutAlias{dqdd, ld3, b}});
}

// ---- controller workloads for the end effector E = the last body (a leaf).
template <class TP>
__global__ __launch_bounds__(kBlock) void k_diff_ik(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                    const float* __restrict__ q, const float* __restrict__ tgt,
                                                    float gain, float lam2, float* __restrict__ qd) {
  RBD_LANE_IO(TP);
  const uint32_t b = lane_id();
  if (b >= batch) return;
  diff_ik_lane<TP, TP::N - 1>(tab, In{q, ld, b}, In{tgt, ld, b}, gain, lam2, Out{qd, ld, b});
}

// Inputs are loaded where they are used: preloading them (as k_fwd_dyn does
// for large trees) held 83 more registers across a sweep that already spills,
// and measured 99 us against 81 us for the humanoid at batch 65536.
template <class TP>
__global__ __launch_bounds__(kBlock) void k_osc(const float* __restrict__ tab, int64_t batch, int64_t ld,
                                                const float* __restrict__ q, const float* __restrict__ qd,
                                                const float* __restrict__ tgt, float kp, float kd, float kn,
                                                float* __restrict__ tau) {
  RBD_LANE_IO(TP);
  const uint32_t b = lane_id();
  if (b >= batch) return;
  osc_lane<TP, TP::N - 1>(tab, In{q, ld, b}, In{qd, ld, b}, In{tgt, ld, b}, kp, kd, kn, Out{tau, ld, b});
}

// ---- packed launch for the serving runtime. One launch serves many requests
// of one (model, operation): the work is cut into tiles of 64 instances (one
// wave), every tile belongs to one request, and a fixed grid of waves strides
// over the tiles, so the same launch (and a graph that captured it) serves any
// number of requests. Request arrays are instance-major, exactly as the client
// handed them over: coordinate c of instance i at p[i * n + c].
template <class TP, int OP>
__global__ __launch_bounds__(kBlock) void k_packed(const float* __restrict__ tab,
                                                   const uint8_t* __restrict__ table) {
  const PackedHdr* hdr = reinterpret_cast<const PackedHdr*>(table);
  const int32_t* tile_req = reinterpret_cast<const int32_t*>(table + sizeof(PackedHdr));
  const PackedReq* reqs = reinterpret_cast<const PackedReq*>(table + hdr->req_offset);
  const int n_tiles = hdr->n_tiles;
  const int lane = threadIdx.x & (kTileLanes - 1);
  const int wave = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kTileLanes);
  const int n_waves = (int)(((int64_t)gridDim.x * blockDim.x) / kTileLanes);
  constexpr int NQ = TP::NQ, NV = TP::NV;
  for (int t = wave; t < n_tiles; t += n_waves) {
    const int r = __builtin_amdgcn_readfirstlane(tile_req[t]);
    const PackedReq& R = reqs[r];
    const int64_t i = (int64_t)(t - R.first_tile) * kTileLanes + lane;
    if (i >= R.batch) continue;
    const InRow q{R.in[0] + i * NQ}, qd{R.in[1] + i * NV}, x2{R.in[2] + i * NV};
    if constexpr (OP == RBD_OP_FWD_DYN) {
      fwd_dyn_lane<TP, 1>(tab, q, qd, RhsOne<InRow>{x2}, SinkOne<OutRow>{OutRow{R.out[0] + i * NV}});
    } else if constexpr (OP == RBD_OP_RNEA) {
      rnea_lane<TP, true>(tab, q, qd, x2, OutRow{R.out[0] + i * NV});
    } else {
      float* gqd = R.out[1] + i * NV;
      float* gtau = R.out[2] + i * NV;
      vjp_lane_parked<TP>(tab, q, qd, x2, InRow{R.in[3] + i * NV}, OutRow{R.out[0] + i * NQ}, RowAlias{gqd},
                          RowAlias{gtau}, RowAlias::In{gqd}, RowAlias::In{gtau});
    }
  }
}

// ------------------------------------------------------------------ launchers
static inline int grid_for(int64_t batch) { return (int)((batch + kBlock - 1) / kBlock); }

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
};
static inline Shape heavy_shape(int64_t batch) {
  const int blk = batch <= kOneWavePerSimd ? 64 : kBlock;
  return {dim3((unsigned)((batch + blk - 1) / blk)), dim3(blk)};
}

static inline rbd_status check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RBD_E_LAUNCH, "%s: launch failed: %s", what, hipGetErrorString(e));
  return RBD_OK;
}

template <class TP>
struct Launch {
  static rbd_status fk(const float* tab, int64_t batch, int64_t ld, const float* q, float* T, hipStream_t s) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fk<TP>), dim3(grid_for(batch)), dim3(kBlock), 0, s, tab, batch, ld, q, T);
    return check_launch("rbd_fk");
  }
  static rbd_status jacobian(const float* tab, int64_t batch, int64_t ld, const float* q, const JacSlots& js,
                             float* J, hipStream_t s) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_jacobian<TP>), dim3(grid_for(batch)), dim3(kBlock), 0, s, tab, batch, ld,
                       q, js, J);
    return check_launch("rbd_jacobian");
  }
  template <bool EXT>
  static rbd_status rnea_t(const float* tab, int64_t batch, int64_t ld, const float* q, const float* qd,
                           const float* qdd, const float* fext, float* tau, hipStream_t s) {
    constexpr bool kPre = TP::NV > 16 && !EXT;
    if (kPre && preload_inputs(kPre)) {
      if (qdd)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rnea<TP, true, EXT, kPre>), dim3(grid_for(batch)), dim3(kBlock), 0, s,
                           tab, batch, ld, q, qd, qdd, fext, tau);
      else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rnea<TP, false, EXT, kPre>), dim3(grid_for(batch)), dim3(kBlock), 0, s,
                           tab, batch, ld, q, qd, qdd, fext, tau);
    } else if (qdd) {
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rnea<TP, true, EXT>), dim3(grid_for(batch)), dim3(kBlock), 0, s, tab,
                         batch, ld, q, qd, qdd, fext, tau);
    } else {
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rnea<TP, false, EXT>), dim3(grid_for(batch)), dim3(kBlock), 0, s, tab,
                         batch, ld, q, qd, qdd, fext, tau);
    }
    return check_launch("rbd_rnea");
  }
  static rbd_status crba(const float* tab, int64_t batch, int64_t ld, const float* q, float* M, hipStream_t s) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_crba<TP>), dim3(grid_for(batch)), dim3(kBlock), 0, s, tab, batch, ld, q,
                       M);
    return check_launch("rbd_crba");
  }
  // Large trees run one wave per SIMD and gain from issuing all input loads up
  // front; small ones keep their occupancy instead (measured).
  template <bool EXT>
  static rbd_status fwd_dyn_t(const float* tab, int64_t batch, int64_t ld, const float* q, const float* qd,
                              const float* tau, const float* fext, float* qdd, hipStream_t s) {
    const Shape sh = heavy_shape(batch);
    constexpr bool kPre = TP::NV > 16;
    if (preload_inputs(kPre))
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fwd_dyn<TP, true, EXT>), sh.grid, sh.block, 0, s, tab,
                         batch, ld, q, qd, tau, fext, qdd);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fwd_dyn<TP, false, EXT>), sh.grid, sh.block, 0, s,
                         tab, batch, ld, q, qd, tau, fext, qdd);
    return check_launch("rbd_fwd_dyn");
  }
  template <bool EXT>
  static rbd_status aba_t(const float* tab, int64_t batch, int64_t ld, const float* q, const float* qd,
                          const float* tau, const float* fext, float* qdd, hipStream_t s) {
    const Shape sh = heavy_shape(batch);
    // with external forces the articulated-body sweep is faster loading its
    // inputs in place (humanoid: 77.8 vs 81.6 us)
    constexpr bool kPre = TP::NV > 16 && !EXT;
    if (preload_inputs(kPre))
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_aba<TP, true, EXT>), sh.grid, sh.block, 0, s, tab,
                         batch, ld, q, qd, tau, fext, qdd);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_aba<TP, false, EXT>), sh.grid, sh.block, 0, s, tab,
                         batch, ld, q, qd, tau, fext, qdd);
    return check_launch("rbd_aba");
  }
  static rbd_status vjp(const float* tab, int64_t batch, int64_t ld, const float* q, const float* qd,
                        const float* tau, const float* gqdd, float* gq, float* gqd, float* gtau, hipStream_t s) {
    const Shape sh = heavy_shape(batch);
    // Between the solve and the adjoint sweep, q-double-dot and lam park in
    // output rows that the adjoint overwrites only after reading them: g_qd
    // and g_tau, or, for a large tree missing one of those, g_q shifted by
    // nq - nv rows, so that DoF k lands in the q slot of its own body (the
    // adjoint reads a body's entries in its forward step and writes that
    // body's g_q in its backward step).
    constexpr bool kVjpParkInGq = TP::NV > 16;
    float* const gq_shift = gq ? gq + (TP::NQ - TP::NV) * ld : nullptr;
    if (gqd && gtau)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fwd_dyn_vjp<TP, 2>), sh.grid, sh.block, 0, s, tab,
                         batch, ld, q, qd, tau, gqdd, gq, gqd, gtau, gqd, gtau);
    else if (kVjpParkInGq && gq && (gqd || gtau))
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fwd_dyn_vjp<TP, kVjpParkInGq ? 3 : 2>), sh.grid, sh.block, 0, s, tab,
                         batch, ld, q, qd, tau, gqdd, gq, gqd, gtau, gqd ? gqd : gq_shift, gtau ? gtau : gq_shift);
    else if (gq || gqd)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fwd_dyn_vjp<TP, 1>), sh.grid, sh.block, 0, s, tab,
                         batch, ld, q, qd, tau, gqdd, gq, gqd, gtau, gqd, gtau);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fwd_dyn_vjp<TP, 0>), sh.grid, sh.block, 0, s, tab,
                         batch, ld, q, qd, tau, gqdd, gq, gqd, gtau, gqd, gtau);
    return check_launch("rbd_fwd_dyn_vjp");
  }
  static rbd_status jvp(const float* tab, int64_t batch, int64_t ld, const float* q, const float* qd,
                        const float* tau, const float* dq, const float* dqd, const float* dtau, float* qdd,
                        float* dqdd, hipStream_t s) {
    const Shape sh = heavy_shape(batch);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fwd_dyn_jvp<TP>), sh.grid, sh.block, 0, s, tab, batch, ld,
                       q, qd, tau, dq, dqd, dtau, qdd, dqdd);
    return check_launch("rbd_fwd_dyn_jvp");
  }
  static rbd_status diff_ik(const float* tab, int64_t batch, int64_t ld, const float* q, const float* tgt, float gain,
                            float lam2, float* qd, hipStream_t s) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_diff_ik<TP>), dim3(grid_for(batch)), dim3(kBlock), 0, s, tab, batch, ld, q,
                       tgt, gain, lam2, qd);
    return check_launch("rbd_diff_ik");
  }
  static rbd_status osc(const float* tab, int64_t batch, int64_t ld, const float* q, const float* qd,
                        const float* tgt, float kp, float kd, float kn, float* tau, hipStream_t s) {
    const Shape sh = heavy_shape(batch);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_osc<TP>), sh.grid, sh.block, 0, s, tab, batch, ld, q, qd, tgt, kp, kd, kn,
                       tau);
    return check_launch("rbd_osc");
  }
  static rbd_status packed(int op, const float* tab, const void* table, int grid, hipStream_t s) {
    const uint8_t* t = static_cast<const uint8_t*>(table);
    if (op == RBD_OP_FWD_DYN)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_packed<TP, RBD_OP_FWD_DYN>), dim3(grid), dim3(kBlock), 0, s, tab, t);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_packed<TP, RBD_OP_RNEA>), dim3(grid), dim3(kBlock), 0, s, tab, t);
    return check_launch("packed launch");
  }
  static rbd_status packed_vjp(int, const float* tab, const void* table, int grid, hipStream_t s) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_packed<TP, RBD_OP_FWD_DYN_VJP>), dim3(grid), dim3(kBlock), 0, s, tab,
                       static_cast<const uint8_t*>(table));
    return check_launch("packed launch");
  }
  // Part 1: kinematics, inverse dynamics, mass matrix. Part 2: forward dynamics
  // and the packed forward-dynamics and inverse-dynamics launches. Part 3: the
  // adjoint and its packed launch. Part 4: the articulated-body algorithm.
  // Part 5: the external-force variants of inverse and forward dynamics. Part
  // 6: the forward-mode derivative. Part 7: the controller workloads. Each part
  // is its own translation unit and instantiates only its own kernels.
  template <int K>
  static LaunchTable part() {
    LaunchTable t{};
    if constexpr (K == 1) {
      t.fk = &Launch::fk;
      t.jacobian = &Launch::jacobian;
      t.rnea = &Launch::rnea_t<false>;
      t.crba = &Launch::crba;
    } else if constexpr (K == 2) {
      t.fwd_dyn = &Launch::fwd_dyn_t<false>;
      t.packed = &Launch::packed;
    } else if constexpr (K == 3) {
      t.vjp = &Launch::vjp;
      t.packed_vjp = &Launch::packed_vjp;
    } else if constexpr (K == 4) {
      t.aba = &Launch::aba_t<false>;
    } else if constexpr (K == 5) {
      t.rnea_ext = &Launch::rnea_t<true>;
      t.fwd_dyn_ext = &Launch::fwd_dyn_t<true>;
      t.aba_ext = &Launch::aba_t<true>;
    } else if constexpr (K == 6) {
      t.jvp = &Launch::jvp;
    } else {
      t.diff_ik = &Launch::diff_ik;
      t.osc = &Launch::osc;
    }
    return t;
  }
};

}  // namespace rbd
